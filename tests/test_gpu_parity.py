"""Bit-exact parity of the GPU path (through the C ABI) against the CPU oracle.

Every comparison is element by element: score, status, and the CIGAR runs of
every pair, on seeded inputs.  Cases cover several tiles and ragged tails,
the band tiers (32- and 64-diagonal bands, full-matrix fallback), the plain
kernel, thresholds, empty and degenerate pairs, invalid input and CIGAR
capacity overflow.
"""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run  # noqa: E402

NW, SWG = (0, 1, 0, 1), (0, 4, 6, 2)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = aim.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_plain():
    c = aim.Context(0, kernel="plain")
    yield c
    c.close()


def check(ctx, batch, alg, pen, max_score=-1, enc="2bit", **kw):
    got = run(ctx, batch, alg, pen, max_score, enc=enc, **kw)
    want = oracle.align_batch(batch, alg, pen, max_score)
    bad = compare(got, want)
    assert not bad, "%d mismatches, first: %s" % (len(bad), describe(batch, bad[0], got, want))
    return got


def _tiny_all(alphabet, maxlen):
    seqs = [np.array(s, np.uint8) for L in range(maxlen + 1) for s in itertools.product(alphabet, repeat=L)]
    pats, txts = zip(*[(p, t) for p in seqs for t in seqs])
    return synth.from_lists(list(pats), list(txts))


@pytest.mark.parametrize("alg,pen", [("nw", NW), ("swg", SWG), ("nw", (0, 3, 0, 4)), ("swg", (0, 3, 4, 1)),
                                     ("swg", (0, 9, 1, 1)), ("nw", (0, 2, 0, 1))])
def test_exhaustive_tiny(ctx, alg, pen):
    check(ctx, _tiny_all(range(4), 3), alg, pen)


def test_exhaustive_tiny_binary(ctx):
    b = _tiny_all(range(2), 5)
    for alg, pen in [("swg", SWG), ("swg", (0, 2, 1, 1)), ("nw", NW), ("nw", (0, 3, 0, 1))]:
        check(ctx, b, alg, pen)


def test_nw100_full_workload(ctx):
    w = synth.WORKLOADS["nw100"]
    b = synth.workload("nw100")
    got = check(ctx, b, "nw", w["pen"], w["max_score"], enc="ascii")
    assert 0.005 < (got[1] == aim.PAIR_REJECTED).mean() < 0.03


def test_swg150_first_20k(ctx):
    b = synth.workload("swg150", n=20_000)
    check(ctx, b, "swg", SWG, -1)


def test_plain_kernel_equals_oracle(ctx_plain):
    b = synth.workload("swg150", n=3000)
    check(ctx_plain, b, "swg", SWG, -1)
    b = synth.workload("nw100", n=3000)
    check(ctx_plain, b, "nw", NW, 5, enc="code")


def _mixed_batch(seed, count, lmin, lmax, rates):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(count):
        L = int(rng.integers(lmin, lmax + 1))
        T = rng.integers(0, 4, L).astype(np.uint8)
        r = float(rng.choice(rates))
        if r >= 1.0:
            P = rng.integers(0, 4, int(rng.integers(lmin, lmax + 1))).astype(np.uint8)
        else:
            b = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, b.txt, b.txt_off, [r])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("alg,pen", [("swg", SWG), ("nw", NW)])
def test_tiers_and_fallback(ctx, alg, pen):
    # noisy and unrelated pairs of uneven length push pairs through the
    # 64-diagonal band and the full-matrix fallback
    b = _mixed_batch(21, 1500, 1, 400, [0.0, 0.02, 0.1, 0.3, 1.0])
    check(ctx, b, alg, pen)


def _length_gap_batch(seed, count, lmin, lmax, dmax, rates):
    """Pairs whose lengths differ by up to dmax (one block inserted into or
    deleted from the text) plus point noise: they pass the 32-diagonal band
    and reach the 64-diagonal tier or the full-matrix tier."""
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(count):
        L = int(rng.integers(lmin, lmax + 1))
        T = rng.integers(0, 4, L).astype(np.uint8)
        k = int(rng.integers(0, dmax + 1))
        at = int(rng.integers(0, L + 1))
        if rng.random() < 0.5:
            P = np.concatenate([T[:at], rng.integers(0, 4, k).astype(np.uint8), T[at:]])
        else:
            P = np.concatenate([T[:at], T[min(L, at + k):]])
        r = float(rng.choice(rates))
        if r > 0:
            b = synth.from_lists([P], [P])
            P, _ = synth.mutate(rng, b.txt, b.txt_off, [r])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("alg,pen", [("swg", SWG), ("nw", NW), ("swg", (0, 3, 4, 1))])
def test_second_tier(ctx, alg, pen):
    b = _length_gap_batch(40, 700, 40, 320, 80, [0.0, 0.02, 0.08])
    full = check(ctx, b, alg, pen)
    check(ctx, b, alg, pen, 150)
    s_, st_, _, off = run(ctx, b, alg, pen, want_cigar=False)
    assert np.array_equal(s_, full[0]) and np.array_equal(st_, full[1]) and not off.any()


def test_second_tier_capacity():
    # a small scratch limit leaves room for few second-tier chunks; the pairs
    # beyond it go to the full-matrix tier
    c = aim.Context(0, scratch_limit=4 << 20)
    try:
        b = _length_gap_batch(41, 300, 300, 400, 60, [0.0, 0.03])
        check(c, b, "swg", SWG)
    finally:
        c.close()


@pytest.mark.parametrize("smax", [0, 1, 6, 20, 200])
def test_thresholds(ctx, smax):
    b = _mixed_batch(22, 800, 0, 160, [0.0, 0.01, 0.05, 0.2, 1.0])
    check(ctx, b, "swg", SWG, smax)
    check(ctx, b, "nw", NW, smax)


def test_degenerate_pairs(ctx):
    pats = ["", "", "A", "", "ACGT", "A" * 300, "", "ACGTACGT" * 40, "T" * 200, "G"]
    txts = ["", "A", "", "ACGTACGTAC", "", "", "C" * 257, "ACGTACGT" * 40, "A" * 200, "G" * 500]
    b = synth.from_lists(pats, txts)
    for alg, pen in [("swg", SWG), ("nw", NW), ("swg", (0, 3, 4, 1))]:
        check(ctx, b, alg, pen)
        check(ctx, b, alg, pen, 10)


def test_score_only_and_encodings(ctx):
    b = synth.workload("nw100", n=2000)
    full = run(ctx, b, "nw", NW, 5, enc="ascii")
    for enc in ("code", "2bit"):
        s, st, _, off = run(ctx, b, "nw", NW, 5, enc=enc)
        assert np.array_equal(s, full[0]) and np.array_equal(st, full[1])
    s, st, _, off = run(ctx, b, "nw", NW, 5, enc="ascii", want_cigar=False)
    assert np.array_equal(s, full[0]) and np.array_equal(st, full[1]) and not off.any()


def test_invalid_input_and_length_bound(ctx):
    b = synth.from_lists(["ACGT", "ACGT", "ACGTA"], ["ACGT", "ACGT", "ACGT"])
    dev_seq = synth.ascii_from_codes(b.pat).copy()
    dev_seq[b.pat_off[1] + 1] = ord("N")  # a non-ACGT base in pair 1
    import torch as T
    ps = T.from_numpy(dev_seq).cuda()
    po = T.from_numpy(b.pat_off[:-1].copy()).cuda()
    pl = T.from_numpy(b.pat_len).cuda()
    ts = T.from_numpy(synth.ascii_from_codes(b.txt).copy()).cuda()
    to = T.from_numpy(b.txt_off[:-1].copy()).cuda()
    tl = T.from_numpy(b.txt_len).cuda()
    s, st, cg, off = run(ctx, b, "swg", SWG, dev=((ps, po, pl, ts, to, tl), aim.ENC_ASCII), max_len=4)
    assert st.tolist() == [aim.PAIR_ALIGNED, aim.PAIR_INVALID, aim.PAIR_INVALID]
    assert s.tolist()[1:] == [-1, -1] and s[0] == 0
    assert off.tolist() == [0, 1, 1, 1]


def test_cigar_capacity_cut(ctx):
    b = synth.workload("swg150", n=500)
    want = oracle.align_batch(b, "swg", SWG, -1)
    runs = np.diff(want[3])
    cap = int(runs[:200].sum())  # exactly the first 200 pairs fit
    s, st, cg, off = run(ctx, b, "swg", SWG, cigar_cap=cap)
    assert np.array_equal(s, want[0])
    assert (st[:200] == 0).all() and (st[200:][runs[200:] > 0] == aim.PAIR_CIGAR_OVERFLOW).all()
    assert off[200] == cap and (off[200:] == cap).all()
    assert np.array_equal(cg[:cap], want[2][:cap])


def test_long_runs_spill_path(ctx):
    # alternating mismatches give many runs per pair: more than the per-pair
    # slot holds, so the in-place re-run path writes those CIGARs
    rng = np.random.default_rng(5)
    pats, txts = [], []
    for _ in range(64):
        T = rng.integers(0, 4, 150).astype(np.uint8)
        P = T.copy()
        P[::3] = (P[::3] + 1) % 4
        pats.append(P)
        txts.append(T)
    check(ctx, synth.from_lists(pats, txts), "swg", (0, 1, 6, 2))


@pytest.mark.parametrize("alg,pen,smax", [("nw", (0, 2, 0, 2), 41), ("swg", (0, 6, 3, 3), 100),
                                         ("swg", (0, 6, 3, 3), -1), ("nw", (0, 2, 0, 2), -1)])
def test_long_reads_common_divisor(ctx, alg, pen, smax):
    # Reads over 256 bases that no band certifies go to the wavefront passes,
    # which run on the penalties divided by their common divisor (2 and 3
    # here); thresholds that are not multiples of it must still split
    # accepted from rejected pairs exactly.
    b = _mixed_batch(37, 80, 300, 700, [0.01, 0.04, 0.1, 1.0])
    check(ctx, b, alg, pen, smax)


@pytest.mark.parametrize("seed", [1, 2])
def test_long_reads(ctx, seed):
    b = _mixed_batch(30 + seed, 60, 500, 1500, [0.01, 0.05])
    check(ctx, b, "swg", SWG)
    check(ctx, b, "nw", NW)


@pytest.mark.parametrize("enc", ["ascii", "code"])
def test_pack_2bit_entry_point(ctx, enc):
    # aim_pack_2bit against the host packer: compact word-aligned CSR, flags
    # for bytes outside the alphabet, a capacity that cuts the last sequences
    rng = np.random.default_rng(17)
    lens = np.concatenate([[0, 1, 31, 32, 33, 64, 65], rng.integers(0, 700, 2000)]).astype(np.int64)
    off = np.zeros(len(lens) + 1, np.int64)
    off[1:] = np.cumsum(lens)
    codes = rng.integers(0, 4, int(off[-1])).astype(np.uint8)
    data = synth.ascii_from_codes(codes) if enc == "ascii" else codes.copy()
    bad = [5, 100, 1500]
    for i in bad:
        if lens[i]:
            data[off[i] + lens[i] // 2] = ord("N") if enc == "ascii" else 7
    words, woff = synth.pack_2bit(codes, off)
    d_seq = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(off[:-1].copy()).cuda()
    d_len = torch.from_numpy(lens.astype(np.int32)).cuda()
    out = torch.zeros(len(words) + 4, dtype=torch.int64, device="cuda")
    out_off = torch.zeros(len(lens) + 1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(len(lens), dtype=torch.int8, device="cuda")
    e = aim.ENC_ASCII if enc == "ascii" else aim.ENC_CODE
    ctx.pack_2bit(e, d_seq, d_off, d_len, out, out_off, flags)
    torch.cuda.synchronize()
    assert np.array_equal(out_off.cpu().numpy(), woff)
    f = flags.cpu().numpy()
    want_flags = np.zeros(len(lens), np.int8)
    want_flags[[i for i in bad if lens[i]]] = 1
    assert np.array_equal(f != 0, want_flags != 0)
    got = out.cpu().numpy().view(np.uint64)[:len(words)]
    ok = np.repeat(f == 0, np.diff(woff))
    assert np.array_equal(got[ok], words[ok])
    # capacity: only the words below words_cap are written, the rest are flagged
    cap = int(woff[1000])
    out2 = torch.zeros(cap, dtype=torch.int64, device="cuda")
    flags2 = torch.zeros(len(lens), dtype=torch.int8, device="cuda")
    ctx.pack_2bit(e, d_seq, d_off, d_len, out2, out_off, flags2)
    torch.cuda.synchronize()
    f2 = flags2.cpu().numpy()
    cut = np.nonzero((woff[1:] > cap) & (np.diff(woff) > 0))[0]  # empty sequences write nothing
    assert (f2[cut] != 0).all() and (f2[:1000][want_flags[:1000] == 0] == 0).all()
    got2 = out2.cpu().numpy().view(np.uint64)
    ok2 = np.repeat((f2 == 0)[:1000], np.diff(woff)[:1000])
    assert np.array_equal(got2[:int(woff[1000])][ok2], words[:int(woff[1000])][ok2])
