"""Helpers for the GPU tests: move seeded batches to the device in the
library's encodings, call the C ABI through the binding, bring results back."""
from __future__ import annotations

import numpy as np
import torch

import synth
import paper_2208_01243_amd as aim


def to_device(batch: synth.PairBatch, enc: str = "2bit", device="cuda"):
    """Device tensors (pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len), enc id."""
    def one(codes, off):
        lens = np.diff(off).astype(np.int32)
        if enc == "2bit":
            words, woff = synth.pack_2bit(codes, off)
            seq = torch.from_numpy(words.view(np.int64).copy() if len(words) else np.zeros(1, np.int64))
            o = torch.from_numpy(woff[:-1].copy())
        else:
            data = synth.ascii_from_codes(codes) if enc == "ascii" else codes
            seq = torch.from_numpy(np.ascontiguousarray(data, np.uint8) if len(data) else np.zeros(1, np.uint8))
            o = torch.from_numpy(off[:-1].astype(np.int64).copy())
        return seq.to(device), o.to(device), torch.from_numpy(lens).to(device)
    ps, po, pl = one(batch.pat, batch.pat_off)
    ts, to, tl = one(batch.txt, batch.txt_off)
    e = {"2bit": aim.ENC_2BIT, "ascii": aim.ENC_ASCII, "code": aim.ENC_CODE}[enc]
    return (ps, po, pl, ts, to, tl), e


def run(ctx, batch, alg, pen, max_score=-1, enc="2bit", want_cigar=True, cigar_cap=None,
        max_len=None, dev=None, stream=None):
    """Align on the GPU; returns numpy (score, status, cigar, cigar_off)."""
    if dev is None:
        dev, e = to_device(batch, enc)
    else:
        dev, e = dev
    n = batch.n
    if max_len is None:
        max_len = int(max(batch.pat_len.max(initial=0), batch.txt_len.max(initial=0)))
    score = torch.empty(n, dtype=torch.int32, device="cuda")
    status = torch.empty(n, dtype=torch.int8, device="cuda")
    if cigar_cap is None:
        cigar_cap = int((batch.pat_len.astype(np.int64) + batch.txt_len + 1).sum()) + 1
    cigar = torch.empty(max(cigar_cap, 1), dtype=torch.int32, device="cuda") if want_cigar else None
    if want_cigar and cigar_cap == 0:
        cigar = torch.empty(0, dtype=torch.int32, device="cuda")
    cigar_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ctx.align_batch(*dev, enc=e, max_len=max_len, alg=alg, pen=pen, max_score=max_score,
                    score=score, status=status, cigar=cigar, cigar_off=cigar_off,
                    want_cigar=want_cigar, stream=stream)
    torch.cuda.synchronize()
    cg = cigar.cpu().numpy().view(np.uint32) if want_cigar else np.zeros(0, np.uint32)
    return score.cpu().numpy(), status.cpu().numpy(), cg, cigar_off.cpu().numpy()


def compare(got, want, batch=None, label=""):
    """Bit-exact comparison of (score, status, cigar, cigar_off); returns list of bad pair ids."""
    gs, gst, gc, go = got
    ws, wst, wc, wo = want
    n = len(ws)
    bad = np.nonzero((gs != ws) | (gst != wst))[0].tolist()
    if not bad and np.array_equal(go, wo) and np.array_equal(gc[:go[-1]], wc[:wo[-1]]):
        return []
    for i in range(n):
        if not np.array_equal(gc[go[i]:go[i + 1]], wc[wo[i]:wo[i + 1]]):
            bad.append(i)
    return sorted(set(bad))


def describe(batch, i, got, want):
    import oracle
    return "pair %d m=%d n=%d got (%d,%d,%s) want (%d,%d,%s)" % (
        i, batch.pat_len[i], batch.txt_len[i], got[0][i], got[1][i],
        oracle.cigar_string(got[2][got[3][i]:got[3][i + 1]]), want[0][i], want[1][i],
        oracle.cigar_string(want[2][want[3][i]:want[3][i + 1]]))
