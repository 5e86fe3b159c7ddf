"""Seeded synthetic read-pair generators.

This module is shared input plumbing: the CPU oracle and the GPU library both
consume what it produces, and it contains none of the alignment arithmetic.

The paper evaluates on real read-reference pairs (100/150/250 bp reads mapped
to GRCh37) and on long synthetic pairs (500 bp - 10 kbp) at 0-5 % edit
distance (Evaluation, Table 2).  Those datasets are not available here; the
workloads below are seeded stand-ins with the same read lengths, error levels
and structure.

Error model (applied per text base, independently): with probability ``rate``
an error occurs whose type is uniform over {substitution, insertion,
deletion}.  A substitution emits one of the three other bases, an insertion
emits a uniform random base followed by the original one, a deletion emits
nothing.  The *text* (reference window) therefore has exactly the nominal
length and the *pattern* (read) length varies with the indels.

Bases are codes 0..3 for A, C, G, T.  ``pack_2bit`` gives the 2-bit layout the
library reads: base t of a sequence sits at bits 2*(t % 32) of the uint64
word t // 32, and every sequence starts on a word boundary.

Randomness: numpy's PCG64 seeded from ``SeedSequence([seed, chunk])`` for
chunks of ``CHUNK`` pairs, so that any range of pairs of a workload can be
regenerated on its own (the oracle samples large workloads this way).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os

import numpy as np

CHUNK = 1024
ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class PairBatch:
    """A CSR batch of pattern/text pairs as base codes 0..3 (uint8)."""

    pat: np.ndarray      # uint8 codes, concatenated
    pat_off: np.ndarray  # int64 [n+1]
    txt: np.ndarray
    txt_off: np.ndarray

    @property
    def n(self) -> int:
        return len(self.pat_off) - 1

    @property
    def pat_len(self) -> np.ndarray:
        return np.diff(self.pat_off).astype(np.int32)

    @property
    def txt_len(self) -> np.ndarray:
        return np.diff(self.txt_off).astype(np.int32)

    def pattern(self, i: int) -> np.ndarray:
        return self.pat[self.pat_off[i]:self.pat_off[i + 1]]

    def text(self, i: int) -> np.ndarray:
        return self.txt[self.txt_off[i]:self.txt_off[i + 1]]

    def subset(self, idx) -> "PairBatch":
        idx = np.asarray(idx, dtype=np.int64)
        return from_lists([self.pattern(i) for i in idx], [self.text(i) for i in idx])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.pat, self.pat_off, self.txt, self.txt_off):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def from_lists(pats, txts) -> PairBatch:
    """Build a batch from lists of code arrays (or 'ACGT' strings)."""
    def conv(s):
        if isinstance(s, str):
            return codes_from_ascii(s)
        return np.asarray(s, dtype=np.uint8)
    pats = [conv(p) for p in pats]
    txts = [conv(t) for t in txts]
    po = np.zeros(len(pats) + 1, np.int64)
    po[1:] = np.cumsum([len(p) for p in pats])
    to = np.zeros(len(txts) + 1, np.int64)
    to[1:] = np.cumsum([len(t) for t in txts])
    cat = lambda xs: np.concatenate(xs).astype(np.uint8) if xs and sum(map(len, xs)) else np.zeros(0, np.uint8)
    return PairBatch(cat(pats), po, cat(txts), to)


def codes_from_ascii(s: str) -> np.ndarray:
    lut = np.full(256, 255, np.uint8)
    for c, v in zip(b"ACGT", range(4)):
        lut[c] = v
    out = lut[np.frombuffer(s.encode(), np.uint8)]
    if (out == 255).any():
        raise ValueError("only A, C, G, T are accepted")
    return out


def ascii_from_codes(c: np.ndarray) -> np.ndarray:
    return ASCII[np.asarray(c, dtype=np.uint8)]


def _concat(batches) -> PairBatch:
    pats, txts, po, to = [], [], [np.zeros(1, np.int64)], [np.zeros(1, np.int64)]
    pb = tb = 0
    for b in batches:
        pats.append(b.pat)
        txts.append(b.txt)
        po.append(b.pat_off[1:] + pb)
        to.append(b.txt_off[1:] + tb)
        pb += len(b.pat)
        tb += len(b.txt)
    return PairBatch(np.concatenate(pats) if pats else np.zeros(0, np.uint8), np.concatenate(po),
                     np.concatenate(txts) if txts else np.zeros(0, np.uint8), np.concatenate(to))


def mutate(rng: np.random.Generator, txt: np.ndarray, txt_off: np.ndarray,
           rate_per_pair: np.ndarray):
    """Apply the per-base error model to every text; returns (pat, pat_off)."""
    nt = len(txt)
    n = len(txt_off) - 1
    lens = np.diff(txt_off)
    rate = np.repeat(np.asarray(rate_per_pair, np.float64), lens)
    err = rng.random(nt) < rate
    kind = rng.integers(0, 3, nt)          # 0 sub, 1 ins, 2 del
    sub = rng.integers(1, 4, nt)
    ins = rng.integers(0, 4, nt).astype(np.uint8)
    t = txt.astype(np.int64)
    first = np.where(err & (kind == 0), (t + sub) % 4, t).astype(np.uint8)
    first = np.where(err & (kind == 1), ins, first)
    cnt = np.ones(nt, np.int64)
    cnt[err & (kind == 1)] = 2
    cnt[err & (kind == 2)] = 0
    vals = np.stack([first, txt], axis=1)
    mask = np.stack([cnt >= 1, cnt == 2], axis=1)
    pat = vals.reshape(-1)[mask.reshape(-1)]
    seg = np.repeat(np.arange(n), lens)
    plen = np.bincount(seg, weights=cnt, minlength=n).astype(np.int64) if nt else np.zeros(n, np.int64)
    po = np.zeros(n + 1, np.int64)
    po[1:] = np.cumsum(plen)
    return pat.astype(np.uint8), po


def _chunk_rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))


def log_uniform_int(rng, a: int, b: int, size) -> np.ndarray:
    v = np.floor(np.exp(rng.uniform(math.log(a), math.log(b + 1), size)))
    return np.clip(v, a, b).astype(np.int64)


def _gen_chunk(rng, n, lens, rates, unrelated):
    lens = np.asarray(lens, np.int64)
    to = np.zeros(n + 1, np.int64)
    to[1:] = np.cumsum(lens)
    txt = rng.integers(0, 4, int(to[-1])).astype(np.uint8)
    pat, po = mutate(rng, txt, to, rates)
    if unrelated is not None and unrelated.any():
        # unrelated pairs: an independent random pattern of the nominal length
        rnd = rng.integers(0, 4, int(to[-1])).astype(np.uint8)
        pats = []
        plen = np.diff(po).copy()
        for i in range(n):
            if unrelated[i]:
                pats.append(rnd[to[i]:to[i + 1]])
                plen[i] = lens[i]
            else:
                pats.append(pat[po[i]:po[i + 1]])
        pat = np.concatenate(pats) if pats else np.zeros(0, np.uint8)
        po = np.zeros(n + 1, np.int64)
        po[1:] = np.cumsum(plen)
    return PairBatch(pat, po, txt, to)


# --------------------------------------------------------------------------
# Workloads.  Each returns a PairBatch of pairs [start, start + n).
# --------------------------------------------------------------------------

def _chunked(seed, start, n, total, make):
    if n is None:
        n = total - start
    c0 = start // CHUNK
    c1 = (start + n - 1) // CHUNK if n > 0 else c0 - 1

    def one(c):
        b = make(_chunk_rng(seed, c), c * CHUNK, min(CHUNK, total - c * CHUNK))
        lo = max(start, c * CHUNK) - c * CHUNK
        hi = min(start + n, c * CHUNK + b.n) - c * CHUNK
        return b.subset(range(lo, hi)) if (lo, hi) != (0, b.n) else b

    chunks = range(c0, c1 + 1)
    if len(chunks) > 4:
        # every chunk has its own generator, so generating them on a few
        # threads (numpy releases the interpreter lock inside its loops)
        # gives the same pairs
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            out = list(ex.map(one, chunks))
    else:
        out = [one(c) for c in chunks]
    return _concat(out) if out else from_lists([], [])


def fixed_length(seed, total, L, rate, start=0, n=None, unrelated_frac=0.0) -> PairBatch:
    """``total`` pairs with text length L and per-base error ``rate``;
    a fraction ``unrelated_frac`` of pairs are independent random sequences."""
    def make(rng, first, k):
        unrel = rng.random(k) < unrelated_frac if unrelated_frac > 0 else None
        return _gen_chunk(rng, k, np.full(k, L), np.full(k, rate), unrel)
    return _chunked(seed, start, n, total, make)


def mixed_length(seed, total, lmin, lmax, rmin, rmax, start=0, n=None) -> PairBatch:
    """Text lengths log-uniform in [lmin, lmax], error rates uniform in [rmin, rmax]."""
    def make(rng, first, k):
        lens = log_uniform_int(rng, lmin, lmax, k)
        rates = rng.uniform(rmin, rmax, k)
        return _gen_chunk(rng, k, lens, rates, None)
    return _chunked(seed, start, n, total, make)


# Penalties are (match, mismatch, gap_open, gap_extend); a gap of length L
# costs gap_open + L * gap_extend.
NW_EDIT = (0, 1, 0, 1)
AFFINE_462 = (0, 4, 6, 2)

WORKLOADS = {
    # NW edit distance, 10k x 100 bp at 2 %, threshold 5 % of 100 bp, ASCII bytes
    "nw100": dict(seed=1, total=10_000, L=100, rate=0.02, alg="nw", pen=NW_EDIT,
                  max_score=5, enc="ascii"),
    # Gotoh 4/6/2, 1M x 150 bp at 4 %, 2-bit, no threshold
    "swg150": dict(seed=2, total=1_000_000, L=150, rate=0.04, alg="swg", pen=AFFINE_462,
                   max_score=-1, enc="2bit"),
    # WFA 4/6/2, 1M x 250 bp: 80 % at 5 %, 20 % unrelated; threshold 25 edits x 8 = 200
    "wfa250": dict(seed=3, total=1_000_000, L=250, rate=0.05, alg="wfa", pen=AFFINE_462,
                   max_score=200, enc="2bit", unrelated_frac=0.2),
    # WFA 4/6/2, 500k pairs, 100..10k bp log-uniform, 0.5..10 %
    "wfa_mixed": dict(seed=4, total=500_000, lmin=100, lmax=10_000, rmin=0.005, rmax=0.10,
                      alg="wfa", pen=AFFINE_462, max_score=-1, enc="2bit"),
    # WFA-adaptive 4/6/2 (reduction after 10 diagonals, 50 bases of slack) at
    # the read lengths and error rates of the paper's GPU comparison: 150 bp
    # at 2 %, 1,000 bp at 5 %, 10,000 bp at 5 %
    "wfa_adaptive_150": dict(seed=6, total=1_000_000, L=150, rate=0.02, alg="wfa_adaptive", pen=AFFINE_462,
                             max_score=-1, enc="2bit", adaptive=(10, 50)),
    "wfa_adaptive_1k": dict(seed=7, total=100_000, L=1000, rate=0.05, alg="wfa_adaptive", pen=AFFINE_462,
                            max_score=-1, enc="2bit", adaptive=(10, 50)),
    "wfa_adaptive_10k": dict(seed=8, total=10_000, L=10_000, rate=0.05, alg="wfa_adaptive", pen=AFFINE_462,
                             max_score=-1, enc="2bit", adaptive=(10, 50)),
    # GenASM (unit edits, k = 10 % of the read length): 1M x 150 bp at 4 %,
    # 100k x 1,000 bp at 5 %
    "genasm150": dict(seed=9, total=1_000_000, L=150, rate=0.04, alg="genasm", pen=NW_EDIT,
                      max_score=15, enc="2bit"),
    "genasm1k": dict(seed=10, total=100_000, L=1000, rate=0.05, alg="genasm", pen=NW_EDIT,
                     max_score=100, enc="2bit"),
}


def workload(name: str, start: int = 0, n: int | None = None) -> PairBatch:
    w = WORKLOADS[name]
    if "L" in w:
        return fixed_length(w["seed"], w["total"], w["L"], w["rate"], start, n,
                            w.get("unrelated_frac", 0.0))
    return mixed_length(w["seed"], w["total"], w["lmin"], w["lmax"], w["rmin"], w["rmax"],
                        start, n)


# --------------------------------------------------------------------------
# Serving workload: Poisson arrivals of requests of varied sizes.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    t_arrival: float
    alg: str
    pen: tuple
    rate: float
    n_pairs: int
    seed: int  # pairs of this request: fixed_lengths via request_pairs()


SERVE = dict(seed=5, rate_hz=2000.0, duration_s=60.0, pmin=1, pmax=4096, lmin=100, lmax=1000,
             rmin=0.01, rmax=0.08)


def serving_schedule(seed=SERVE["seed"], rate_hz=SERVE["rate_hz"], duration_s=SERVE["duration_s"],
                     pmin=SERVE["pmin"], pmax=SERVE["pmax"]):
    """Open-loop Poisson arrivals; algorithm uniform over NW edit, SWG 4/6/2, WFA 4/6/2."""
    rng = _chunk_rng(seed, 0)
    reqs = []
    t = 0.0
    algs = [("nw", NW_EDIT), ("swg", AFFINE_462), ("wfa", AFFINE_462)]
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        a = algs[int(rng.integers(0, 3))]
        reqs.append(Request(t, a[0], a[1], float(rng.uniform(SERVE["rmin"], SERVE["rmax"])),
                            int(log_uniform_int(rng, pmin, pmax, 1)[0]), len(reqs)))
    return reqs


def request_pairs(req: Request, lmin=SERVE["lmin"], lmax=SERVE["lmax"]) -> PairBatch:
    rng = _chunk_rng(SERVE["seed"] * 1_000_003 + req.seed, 1)
    lens = rng.integers(lmin, lmax + 1, req.n_pairs)
    return _gen_chunk(rng, req.n_pairs, lens, np.full(req.n_pairs, req.rate), None)


# --------------------------------------------------------------------------
# Encodings handed to the library.
# --------------------------------------------------------------------------

def pack_2bit(codes: np.ndarray, off: np.ndarray):
    """Pack code sequences into word-aligned 2-bit CSR: (words uint64, woff int64[n+1])."""
    lens = np.diff(off)
    nw = (lens + 31) // 32
    woff = np.zeros(len(lens) + 1, np.int64)
    woff[1:] = np.cumsum(nw)
    total = int(woff[-1])
    # one byte per base slot, each sequence starting on a 32-slot boundary
    slots = np.zeros(total * 32, np.uint8)
    if len(codes):
        if len(lens) * 64 < len(codes):
            for i in range(len(lens)):
                slots[woff[i] * 32:woff[i] * 32 + lens[i]] = codes[off[i]:off[i + 1]]
        else:
            seq = np.repeat(np.arange(len(lens)), lens)
            pos = np.arange(len(codes)) - np.repeat(off[:-1], lens)
            slots[woff[seq] * 32 + pos] = codes
    # four slots per byte (slot t at bits 2 (t mod 4)); the little-endian
    # uint64 view of 8 such bytes puts slot t at bits 2 (t mod 32)
    packed = np.zeros(total * 8, np.uint8)
    step = 1 << 24
    for a in range(0, len(packed), step):
        q = slots[4 * a:4 * (a + step)].reshape(-1, 4)
        packed[a:a + len(q)] = q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)
    return packed.view("<u8").astype(np.uint64, copy=False), woff


def unpack_2bit(words: np.ndarray, woff: np.ndarray, lens: np.ndarray) -> np.ndarray:
    out = []
    for i in range(len(lens)):
        w = words[woff[i]:woff[i + 1]]
        t = np.arange(lens[i])
        out.append(((w[t // 32] >> (2 * (t % 32)).astype(np.uint64)) & np.uint64(3)).astype(np.uint8))
    return np.concatenate(out) if out else np.zeros(0, np.uint8)
