"""CPU oracle for batched global pairwise alignment (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It is independent of the GPU library: it
shares no code, headers or tables with ``paper_2208_01243_amd`` and never
imports it.

* ``aim_oracle.c`` -- full-matrix int32 Needleman-Wunsch (linear gaps) and
  Smith-Waterman-Gotoh (affine gaps) with the canonical traceback and the
  threshold rule; see that file's header for the definitions it writes out.
* ``wfa_scalar.c`` -- a scalar wavefront algorithm, a second route to the
  same optimum used to pin the first one (and to count wavefront work), and
  its adaptive (heuristic) variant, WFA-adaptive.
* ``genasm.c`` -- GenASM: windowed bitap distance calculation with a
  traceback over its intermediate bit-vectors (unit edits, threshold k); see
  that file's header for the reading it writes out.
* ``rescore.py`` -- replays a CIGAR over the two sequences and recomputes its
  cost from the gap model, without any DP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .rescore import rescore, cigar_string, parse_runs  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, f) for f in ("aim_oracle.c", "wfa_scalar.c", "genasm.c")]

ALG = {"nw": 0, "swg": 1, "wfa": 2}
ALIGNED, REJECTED = 0, 1

_lib = None
_lock = threading.Lock()


def build(force: bool = True, path: str = LIB, native: bool = False) -> str:
    """Compile the C oracle with gcc into ``path`` (``oracle/liboracle.so``).
    ``native``: -O3 -march=native for the host that runs it (the CPU baseline
    builds such a copy where it is timed; the in-tree library stays portable,
    since it is built on one machine and may run on another)."""
    if not force and os.path.exists(path):
        return path
    tmp = path + ".tmp%d" % os.getpid()
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
                           "-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    return path


class WfaStats(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("compared", ctypes.c_int64),
                ("wavefronts", ctypes.c_int64), ("words", ctypes.c_int64),
                ("lo_min", ctypes.c_int32), ("hi_max", ctypes.c_int32), ("dropped", ctypes.c_int64)]


def bind(path: str):
    """Load an oracle shared library and declare its entry points."""
    L = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.oracle_align_pair.argtypes = [p, i32, p, i32, i32, i32, i32, i32, i32, i32,
                                    p, p, p, i32, p]
    L.oracle_align_pair.restype = ctypes.c_int
    L.oracle_align_batch.argtypes = [i64, p, p, p, p, i32, i32, i32, i32, i32, i32, i32,
                                     p, p, p, p, p]
    L.oracle_align_batch.restype = ctypes.c_int
    L.oracle_wfa.argtypes = [p, i32, p, i32, i32, i32, i32, i32, i32, p, p, p, i32, p,
                             ctypes.POINTER(WfaStats)]
    L.oracle_wfa.restype = ctypes.c_int
    L.oracle_wfa_adaptive.argtypes = [p, i32, p, i32, i32, i32, i32, i32, i32, i32, i32, p, p, p, i32, p,
                                      ctypes.POINTER(WfaStats)]
    L.oracle_wfa_adaptive.restype = ctypes.c_int
    L.oracle_genasm.argtypes = [p, i32, p, i32, i32, i32, i32, i32, p, p, p, i32, p, p]
    L.oracle_genasm.restype = ctypes.c_int
    L.oracle_genasm_dc.argtypes = [p, i32, p, i32, i32, i32, p]
    L.oracle_genasm_dc.restype = ctypes.c_int
    L.oracle_genasm_batch.argtypes = [i64, p, p, p, p, i32, i32, i32, i32, i32, p, p, p, p, p, p]
    L.oracle_genasm_batch.restype = ctypes.c_int
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            _lib = bind(LIB)
        return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _codes(s):
    if isinstance(s, str):
        lut = {"A": 0, "C": 1, "G": 2, "T": 3}
        return np.array([lut[c] for c in s], np.uint8)
    return np.ascontiguousarray(s, dtype=np.uint8)


def _check_pen(alg, pen):
    a, x, o, e = pen
    if a != 0 or x <= 0 or e <= 0 or o < 0:
        raise ValueError("penalties need match 0, mismatch > 0, gap_extend > 0, gap_open >= 0")
    if alg == "nw" and o != 0:
        raise ValueError("linear NW takes gap_open 0 (a gap base costs gap_extend)")


def align_pair(P, T, alg: str, pen, max_score: int = -1, want_cigar: bool = True, handle=None):
    """Align one pair.  Returns (status, score, runs) with runs a list of uint32.
    ``handle`` selects another build of the oracle (see ``bind``)."""
    _check_pen(alg, pen)
    P, T = _codes(P), _codes(T)
    m, n = len(P), len(T)
    cap = m + n + 1
    runs = np.zeros(cap, np.uint32)
    score = np.zeros(1, np.int32)
    status = np.zeros(1, np.int8)
    nr = np.zeros(1, np.int32)
    Pb = P if m else np.zeros(1, np.uint8)
    Tb = T if n else np.zeros(1, np.uint8)
    (handle or lib()).oracle_align_pair(_ptr(Pb), m, _ptr(Tb), n, ALG[alg], pen[1], pen[2], pen[3], max_score,
                            int(want_cigar), _ptr(score), _ptr(status), _ptr(runs), cap, _ptr(nr))
    if status[0] < 0:
        raise RuntimeError("oracle failure %d" % status[0])
    return int(status[0]), int(score[0]), [int(r) for r in runs[:nr[0]]]


ADAPTIVE_DEFAULT = (10, 50)  # (min_len, max_dist) of the reduction, as wfa_scalar.c describes


def wfa_pair(P, T, pen, max_score: int = -1, want_cigar: bool = True, handle=None, adaptive=None):
    """Scalar WFA.  Returns (status, score, runs, stats dict); the stats are
    the work counters of ``wfa_scalar.c`` (cells, wavefronts, compared, words,
    lo_min, hi_max, dropped).  ``adaptive`` = (min_len, max_dist) runs
    WFA-adaptive instead (a heuristic: a valid alignment, cost >= optimum)."""
    _check_pen("wfa", pen)
    P, T = _codes(P), _codes(T)
    m, n = len(P), len(T)
    cap = m + n + 1
    runs = np.zeros(cap, np.uint32)
    score = np.zeros(1, np.int32)
    status = np.zeros(1, np.int8)
    nr = np.zeros(1, np.int32)
    st = WfaStats()
    Pb = P if m else np.zeros(1, np.uint8)
    Tb = T if n else np.zeros(1, np.uint8)
    L = handle or lib()
    if adaptive is None:
        rc = L.oracle_wfa(_ptr(Pb), m, _ptr(Tb), n, pen[1], pen[2], pen[3], max_score,
                          int(want_cigar), _ptr(score), _ptr(status), _ptr(runs), cap, _ptr(nr),
                          ctypes.byref(st))
    else:
        rc = L.oracle_wfa_adaptive(_ptr(Pb), m, _ptr(Tb), n, pen[1], pen[2], pen[3], max_score,
                                   int(want_cigar), int(adaptive[0]), int(adaptive[1]), _ptr(score),
                                   _ptr(status), _ptr(runs), cap, _ptr(nr), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("wfa oracle failure %d" % rc)
    return (int(status[0]), int(score[0]), [int(r) for r in runs[:nr[0]]],
            {"cells": st.cells, "compared": st.compared, "wavefronts": st.wavefronts,
             "words": st.words, "lo_min": st.lo_min, "hi_max": st.hi_max, "dropped": st.dropped})


def wfa_batch(batch, pen, max_score: int = -1, adaptive=None, want_cigar: bool = True,
              nthreads: int | None = None):
    """``wfa_pair`` over every pair of a ``synth.PairBatch`` on host threads.
    Returns (score int32[n], status int8[n], cigar uint32[...], cigar_off
    int64[n+1]) like ``align_batch``."""
    from concurrent.futures import ThreadPoolExecutor
    n = batch.n
    L = lib()

    def one(i):
        st, sc, runs, _ = wfa_pair(batch.pattern(i), batch.text(i), pen, max_score, want_cigar, L, adaptive)
        return st, sc, runs

    with ThreadPoolExecutor(nthreads or os.cpu_count() or 1) as ex:
        res = list(ex.map(one, range(n)))
    score = np.array([r[1] for r in res], np.int32)
    status = np.array([r[0] for r in res], np.int8)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r[2]) for r in res])
    cigar = np.array([x for r in res for x in r[2]], np.uint32)
    return score, status, cigar, off


def align_batch(batch, alg: str, pen, max_score: int = -1, want_cigar: bool = True,
                nthreads: int | None = None, handle=None):
    """Align every pair of a ``synth.PairBatch`` (codes).  Returns
    (score int32[n], status int8[n], cigar uint32[...], cigar_off int64[n+1]).
    ``handle`` selects another build of the oracle (see ``bind``)."""
    _check_pen(alg, pen)
    n = batch.n
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    plen, tlen = batch.pat_len.astype(np.int64), batch.txt_len.astype(np.int64)
    slot = np.zeros(n + 1, np.int64)
    slot[1:] = np.cumsum(plen + tlen + 1) if want_cigar else 0
    runs = np.zeros(max(int(slot[-1]), 1), np.uint32)
    score = np.zeros(n, np.int32)
    status = np.zeros(n, np.int8)
    nr = np.zeros(n, np.int32)
    pat = batch.pat if len(batch.pat) else np.zeros(1, np.uint8)
    txt = batch.txt if len(batch.txt) else np.zeros(1, np.uint8)
    if want_cigar:
        slot_arr = slot
    else:
        slot_arr = np.zeros(n + 1, np.int64)
    rc = (handle or lib()).oracle_align_batch(n, _ptr(pat), _ptr(np.ascontiguousarray(batch.pat_off)),
                                  _ptr(txt), _ptr(np.ascontiguousarray(batch.txt_off)), ALG[alg],
                                  pen[1], pen[2], pen[3], max_score, int(want_cigar), nthreads,
                                  _ptr(score), _ptr(status), _ptr(runs), _ptr(slot_arr), _ptr(nr))
    if rc != 0 or (status < 0).any():
        raise RuntimeError("oracle batch failure")
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(nr)
    if want_cigar and n:
        idx = np.repeat(slot[:-1], nr) + (np.arange(int(off[-1])) - np.repeat(off[:-1], nr))
        cigar = runs[idx]
    else:
        cigar = np.zeros(0, np.uint32)
    return score, status, cigar, off


GENASM_WINDOW, GENASM_OVERLAP = 64, 24  # window bases and overlap of the GPU library


def genasm_pair(P, T, k: int = -1, window: int = GENASM_WINDOW, overlap: int = GENASM_OVERLAP,
                want_cigar: bool = True, handle=None, stats: bool = False):
    """GenASM of one pair (``genasm.c``): unit edits, at most ``k`` of them
    (-1: no threshold).  Returns (status, score, runs), plus the work
    counters {windows, updates, tb_steps} when ``stats``."""
    P, T = _codes(P), _codes(T)
    m, n = len(P), len(T)
    cap = m + n + 1
    runs = np.zeros(cap, np.uint32)
    score = np.zeros(1, np.int32)
    status = np.zeros(1, np.int8)
    nr = np.zeros(1, np.int32)
    Pb = P if m else np.zeros(1, np.uint8)
    Tb = T if n else np.zeros(1, np.uint8)
    st = np.zeros(3, np.int64)
    rc = (handle or lib()).oracle_genasm(_ptr(Pb), m, _ptr(Tb), n, int(k), int(window), int(overlap),
                                         int(want_cigar), _ptr(score), _ptr(status), _ptr(runs), cap, _ptr(nr),
                                         _ptr(st))
    if rc != 0:
        raise RuntimeError("genasm oracle failure %d" % rc)
    out = (int(status[0]), int(score[0]), [int(r) for r in runs[:nr[0]]])
    if stats:
        return out + ({"windows": int(st[0]), "updates": int(st[1]), "tb_steps": int(st[2])},)
    return out


def genasm_dc(p, t, anchored: bool, levels: int, handle=None):
    """Status bits of one GenASM window: array [b + 1, levels + 1, a + 1]
    with [j, d, i] = [D(i, j) <= d] (``genasm.c``'s distance calculation)."""
    p, t = _codes(p), _codes(t)
    a, b = len(p), len(t)
    out = np.zeros((b + 1) * (levels + 1) * (a + 1), np.uint8)
    pb = p if a else np.zeros(1, np.uint8)
    tb = t if b else np.zeros(1, np.uint8)
    rc = (handle or lib()).oracle_genasm_dc(_ptr(pb), a, _ptr(tb), b, int(anchored), int(levels), _ptr(out))
    if rc != 0:
        raise RuntimeError("genasm dc failure %d" % rc)
    return out.reshape(b + 1, levels + 1, a + 1)


def genasm_batch(batch, k: int = -1, want_cigar: bool = True, window: int = GENASM_WINDOW,
                 overlap: int = GENASM_OVERLAP, nthreads: int | None = None, handle=None, stats=None):
    """``genasm_pair`` over every pair of a ``synth.PairBatch`` on host
    threads.  Returns (score int32[n], status int8[n], cigar uint32[...],
    cigar_off int64[n+1]) like ``align_batch``.  ``stats``: an int64 array
    [n, 3] that receives each pair's work counters."""
    n = batch.n
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    plen, tlen = batch.pat_len.astype(np.int64), batch.txt_len.astype(np.int64)
    slot = np.zeros(n + 1, np.int64)
    if want_cigar:
        slot[1:] = np.cumsum(plen + tlen + 1)
    runs = np.zeros(max(int(slot[-1]), 1), np.uint32)
    score = np.zeros(n, np.int32)
    status = np.zeros(n, np.int8)
    nr = np.zeros(n, np.int32)
    pat = batch.pat if len(batch.pat) else np.zeros(1, np.uint8)
    txt = batch.txt if len(batch.txt) else np.zeros(1, np.uint8)
    rc = (handle or lib()).oracle_genasm_batch(
        n, _ptr(pat), _ptr(np.ascontiguousarray(batch.pat_off)), _ptr(txt),
        _ptr(np.ascontiguousarray(batch.txt_off)), int(k), int(window), int(overlap), int(want_cigar),
        nthreads, _ptr(score), _ptr(status), _ptr(runs), _ptr(slot), _ptr(nr),
        _ptr(stats) if stats is not None else None)
    if rc != 0 or (status < 0).any():
        raise RuntimeError("genasm oracle batch failure %d" % rc)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(nr)
    if want_cigar and n:
        idx = np.repeat(slot[:-1], nr) + (np.arange(int(off[-1])) - np.repeat(off[:-1], nr))
        cigar = runs[idx]
    else:
        cigar = np.zeros(0, np.uint32)
    return score, status, cigar, off
