"""aim_align_batch_static, the entry point that allocates nothing (its scratch
is a static device array): bit for bit the results of aim_align_batch, on two
calls in a row of which the second is smaller, for every algorithm; and an
oversized batch is refused with an error rather than run.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run, to_device  # noqa: E402


def _run_static(ctx, b, alg, pen, max_score, enc):
    dev, e = to_device(b, enc)
    n = b.n
    max_len = int(max(b.pat_len.max(initial=0), b.txt_len.max(initial=0)))
    score = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    status = torch.full((n,), 9, dtype=torch.int8, device="cuda")
    cap = int((b.pat_len.astype(np.int64) + b.txt_len + 1).sum()) + 1
    cigar = torch.zeros(cap, dtype=torch.int32, device="cuda")
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    ctx.align_batch_static(*dev, enc=e, max_len=max_len, alg=alg, pen=pen, max_score=max_score,
                           score=score, status=status, cigar=cigar, cigar_off=off, stream=stream)
    torch.cuda.synchronize()
    return score.cpu().numpy(), status.cpu().numpy(), cigar.cpu().numpy().view(np.uint32), off.cpu().numpy()


def _mixed(seed, count, lmin, lmax):
    rng = np.random.default_rng(seed)
    lens = synth.log_uniform_int(rng, lmin, lmax, count)
    rates = rng.uniform(0.005, 0.10, count)
    return synth._gen_chunk(rng, count, lens, rates, None)


CASES = [
    # (label, algorithm, penalties, threshold, encoding, first batch, second smaller batch)
    ("nw100", "nw", (0, 1, 0, 1), 5, "ascii",
     lambda: synth.workload("nw100", n=6000), lambda: synth.workload("nw100", start=6000, n=1500)),
    ("swg150", "swg", (0, 4, 6, 2), -1, "2bit",
     lambda: synth.workload("swg150", n=20000), lambda: synth.workload("swg150", start=20000, n=3000)),
    ("wfa250", "wfa", (0, 4, 6, 2), 200, "2bit",
     lambda: synth.workload("wfa250", n=20000), lambda: synth.workload("wfa250", start=20000, n=2500)),
    ("wfa_100_3000", "wfa", (0, 4, 6, 2), -1, "2bit",
     lambda: _mixed(11, 1500, 100, 3000), lambda: _mixed(12, 300, 100, 1500)),
    ("swg_100_2000", "swg", (0, 4, 6, 2), -1, "code",
     lambda: _mixed(13, 800, 100, 2000), lambda: _mixed(14, 200, 100, 800)),
    ("wfa_adaptive_150", "wfa_adaptive", (0, 4, 6, 2), -1, "2bit",
     lambda: synth.workload("wfa_adaptive_150", n=20000),
     lambda: synth.workload("wfa_adaptive_150", start=20000, n=3000)),
    ("genasm150", "genasm", (0, 1, 0, 1), 15, "2bit",
     lambda: synth.workload("genasm150", n=20000), lambda: synth.workload("genasm150", start=20000, n=3000)),
]
ADAPTIVE = (10, 50)  # the reduction rule of the WFA-adaptive cases


def _oracle(sub, alg, pen, smax):
    if alg == "genasm":
        return oracle.genasm_batch(sub, smax)
    if alg == "wfa_adaptive":
        return oracle.wfa_batch(sub, pen, smax, adaptive=ADAPTIVE)
    return oracle.align_batch(sub, alg, pen, smax)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_static_entry_matches_align_batch(case):
    label, alg, pen, smax, enc, first, second = case
    b1, b2 = first(), second()
    assert b2.n < b1.n
    print("static entry point: %s, %d then %d pairs" % (label, b1.n, b2.n), flush=True)
    with aim.Context(0) as ctx:
        ctx.wfa_adaptive_params(*ADAPTIVE)
        want1 = run(ctx, b1, alg, pen, smax, enc=enc)
        want2 = run(ctx, b2, alg, pen, smax, enc=enc)
    with aim.Context(0, static_scratch=True) as sctx:
        sctx.wfa_adaptive_params(*ADAPTIVE)
        got1 = _run_static(sctx, b1, alg, pen, smax, enc)
        got2 = _run_static(sctx, b2, alg, pen, smax, enc)
    for b, got, want in ((b1, got1, want1), (b2, got2, want2)):
        bad = compare(got, want)
        assert not bad, describe(b, bad[0], got, want)
        assert (got[1] != aim.PAIR_CIGAR_OVERFLOW).all() and (got[1] != aim.PAIR_INVALID).all()
    # and both against the oracle on a sample of the second batch
    idx = np.arange(0, b2.n, max(1, b2.n // 200))
    sub = b2.subset(idx)
    ws, wst, wc, wo = _oracle(sub, alg, pen, smax)
    s, st, cg, off = got2
    for t, i in enumerate(idx):
        assert (s[i], st[i]) == (ws[t], wst[t]), (label, i)
        assert np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]]), (label, i)


def test_static_entry_refuses_oversized_batch_then_still_works():
    big = synth.workload("swg150", n=1_000_000)
    small = synth.workload("swg150", n=2000)
    with aim.Context(0) as sctx:
        with pytest.raises(aim.AimError) as ei:
            _run_static(sctx, big, "swg", (0, 4, 6, 2), -1, "2bit")
        assert ei.value.code == -1 and "static array" in str(ei.value)
        got = _run_static(sctx, small, "swg", (0, 4, 6, 2), -1, "2bit")
    want = oracle.align_batch(small, "swg", (0, 4, 6, 2), -1)
    bad = compare(got, want)
    assert not bad, describe(small, bad[0], got, want)
