"""Python binding of libaim.so (batched pairwise alignment on MI355X).

Argument marshalling only: every step of the alignment runs in the HIP
kernels of ``libaim.so``; this module turns torch tensors (device memory) and
torch streams into the plain pointers of the C ABI declared in
``include/aim.h``, and C error codes into exceptions.  There is no fallback:
if the library is not built, importing the entry points raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaim.so")

NW_LINEAR, SWG_AFFINE, WFA_AFFINE, WFA_ADAPTIVE, GENASM = 0, 1, 2, 3, 4
ALGORITHMS = {"nw": NW_LINEAR, "swg": SWG_AFFINE, "wfa": WFA_AFFINE, "wfa_adaptive": WFA_ADAPTIVE,
              "genasm": GENASM}
ENC_ASCII, ENC_CODE, ENC_2BIT = 0, 1, 2
KERNEL_AUTO, KERNEL_PLAIN = 0, 1
FLAG_TIMING = 1
FLAG_STATIC_SCRATCH = 2
FLAG_NO_PREFILTER = 4
FLAG_HARD_LIMIT = 8
PAIR_ALIGNED, PAIR_REJECTED, PAIR_CIGAR_OVERFLOW, PAIR_INVALID = 0, 1, 2, 3
OP_MATCH, OP_MISMATCH, OP_INS, OP_DEL = 0, 1, 2, 3

ERRORS = {-1: "AIM_ERR_INVALID_ARG", -2: "AIM_ERR_UNSUPPORTED", -3: "AIM_ERR_OOM",
          -4: "AIM_ERR_HIP", -5: "AIM_ERR_BUSY", -6: "AIM_ERR_NOT_FOUND"}

i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class Penalties(ctypes.Structure):
    _fields_ = [("match", i32), ("mismatch", i32), ("gap_open", i32), ("gap_extend", i32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_pairs", i64), ("enc", i32), ("max_len", i32),
                ("pat_seq", vp), ("pat_off", vp), ("pat_len", vp),
                ("txt_seq", vp), ("txt_off", vp), ("txt_len", vp)]


class Results(ctypes.Structure):
    _fields_ = [("score", vp), ("status", vp), ("cigar", vp), ("cigar_off", vp),
                ("cigar_cap", i64), ("want_cigar", i32)]


class Options(ctypes.Structure):
    _fields_ = [("kernel", i32), ("flags", i32), ("scratch_limit", i64)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("n_streams", i32), ("flags", i32), ("budget_bytes", i64), ("max_batch_pairs", i64)]


class Request(ctypes.Structure):
    _fields_ = [("alg", i32), ("pen", Penalties), ("max_score", i32), ("want_cigar", i32), ("enc", i32),
                ("n_pairs", i64), ("pat", vp), ("pat_off", vp), ("pat_len", vp),
                ("txt", vp), ("txt_off", vp), ("txt_len", vp)]


class RequestResult(ctypes.Structure):
    _fields_ = [("n_pairs", i64), ("score", vp), ("status", vp), ("cigar", vp), ("cigar_off", vp),
                ("latency_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", i64), ("completed", i64), ("pairs_completed", i64), ("batches", i64),
                ("queued", i64), ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double), ("bytes_in_use", i64),
                ("peak_bytes", i64), ("budget_bytes", i64), ("elapsed_s", ctypes.c_double)]


class CallStats(ctypes.Structure):
    _fields_ = [("n_pairs", i64), ("band_escalated", i32), ("band_escalated2", i32), ("wfa_wide", i32),
                ("wfa_walk_failed", i32), ("wfa_walk_skipped", i32), ("full_store", i32 * 4),
                ("cigar_reruns", i32), ("wfa_window", i32), ("wfa_class_pairs", i32 * 4),
                ("wfa_class_window", i32 * 4), ("prefilter_rejected", i32), ("wfa_adaptive_dropped", i64),
                ("wfa_long_pairs", i32), ("wfa_long_failed", i32)]


class AimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "AIM_ERR"), code, msg))
        self.code = code


# Entry points: name -> (argtypes, restype).  The same names as the C ABI.
SIGNATURES = {
    "aim_create": ([ctypes.POINTER(vp), i32, ctypes.POINTER(Options)], i32),
    "aim_destroy": ([vp], None),
    "aim_align_batch": ([vp, ctypes.POINTER(Batch), i32, Penalties, i32, ctypes.POINTER(Results), vp], i32),
    "aim_align_batch_static": ([vp, ctypes.POINTER(Batch), i32, Penalties, i32, ctypes.POINTER(Results),
                                vp], i32),
    "aim_prefilter": ([vp, ctypes.POINTER(Batch), i32, Penalties, i32, vp, vp, vp], i32),
    "aim_scratch_usage": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
    "aim_wfa_adaptive_params": ([vp, i32, i32], i32),
    "aim_pack_2bit": ([vp, i64, i32, vp, vp, vp, vp, i64, vp, vp, vp], i32),
    "aim_timing": ([vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                    ctypes.POINTER(i64)], i32),
    "aim_timing_reset": ([vp], i32),
    "aim_last_call_stats": ([vp, ctypes.POINTER(CallStats)], i32),
    "aim_autotune": ([vp, ctypes.POINTER(Batch), i32, Penalties, i32, ctypes.POINTER(Results), vp, i32,
                      ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], i32),
    "aim_tune_get": ([vp, i32, i32, ctypes.POINTER(i32)], i32),
    "aim_tune_set": ([vp, i32, i32, ctypes.POINTER(i32)], i32),
    "aim_tune_save": ([vp, ctypes.c_char_p], i32),
    "aim_tune_entries": ([vp, i32, vp, vp, vp, ctypes.POINTER(i32)], i32),
    "aim_tune_load": ([vp, ctypes.c_char_p], i32),
    "aim_graph_capture": ([vp, ctypes.POINTER(Batch), i32, Penalties, i32, ctypes.POINTER(Results), vp,
                           ctypes.POINTER(vp)], i32),
    "aim_graph_launch": ([vp, vp], i32),
    "aim_graph_destroy": ([vp], None),
    "aim_server_create": ([i32, ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)], i32),
    "aim_server_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(i64)], i32),
    "aim_server_poll": ([vp, i64, ctypes.POINTER(RequestResult)], i32),
    "aim_server_wait": ([vp, i64, i32, ctypes.POINTER(RequestResult)], i32),
    "aim_server_release": ([vp, i64], i32),
    "aim_server_stats_get": ([vp, ctypes.POINTER(ServerStats)], i32),
    "aim_server_reset_stats": ([vp], i32),
    "aim_server_last_error": ([], ctypes.c_char_p),
    "aim_server_destroy": ([vp], None),
    "aim_last_error": ([], ctypes.c_char_p),
    "aim_version": ([], ctypes.c_char_p),
}

_lib = None


def lib():
    """Load libaim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libaim.so is not built; run __graft_entry__.build() "
                              "(or python paper_2208_01243_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise AimError(code, lib().aim_last_error().decode())


def _ptr(t):
    return None if t is None else vp(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return vp(stream)
    return vp(stream.cuda_stream)


class Context:
    """An aim_context on one HIP device."""

    def __init__(self, device: int = 0, kernel: str = "auto", scratch_limit: int = 0,
                 timing: bool = False, static_scratch: bool = False, prefilter: bool = True,
                 hard_limit: bool = False):
        opt = Options(KERNEL_PLAIN if kernel == "plain" else KERNEL_AUTO,
                      (FLAG_TIMING if timing else 0) | (FLAG_STATIC_SCRATCH if static_scratch else 0)
                      | (0 if prefilter else FLAG_NO_PREFILTER) | (FLAG_HARD_LIMIT if hard_limit else 0),
                      scratch_limit)
        h = vp()
        _check(lib().aim_create(ctypes.byref(h), device, ctypes.byref(opt)))
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            lib().aim_destroy(self._h)
            self._h = vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @staticmethod
    def _args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg, score,
              status, cigar, cigar_off, want_cigar):
        n = pat_len.numel()
        b = Batch(n, enc, max_len, _ptr(pat_seq), _ptr(pat_off), _ptr(pat_len),
                  _ptr(txt_seq), _ptr(txt_off), _ptr(txt_len))
        r = Results(_ptr(score), _ptr(status), _ptr(cigar), _ptr(cigar_off),
                    cigar.numel() if cigar is not None else 0, int(bool(want_cigar)))
        a = ALGORITHMS[alg] if isinstance(alg, str) else int(alg)
        return b, r, a

    def align_batch(self, pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, *, enc: int,
                    max_len: int, alg, pen, max_score: int, score, status, cigar=None,
                    cigar_off=None, want_cigar: bool = True, stream=None):
        """aim_align_batch on device tensors; outputs are written in place."""
        b, r, a = self._args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg,
                             score, status, cigar, cigar_off, want_cigar)
        _check(lib().aim_align_batch(self._h, ctypes.byref(b), a, Penalties(*pen), max_score,
                                     ctypes.byref(r), _stream(stream)))

    def align_batch_static(self, pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, *, enc: int,
                           max_len: int, alg, pen, max_score: int, score, status, cigar=None,
                           cigar_off=None, want_cigar: bool = True, stream=None):
        """aim_align_batch_static (no device allocation) on device tensors."""
        b, r, a = self._args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg,
                             score, status, cigar, cigar_off, want_cigar)
        _check(lib().aim_align_batch_static(self._h, ctypes.byref(b), a, Penalties(*pen), max_score,
                                            ctypes.byref(r), _stream(stream)))

    def wfa_adaptive_params(self, min_len: int, max_dist: int):
        """aim_wfa_adaptive_params: the reduction rule of alg "wfa_adaptive"."""
        _check(lib().aim_wfa_adaptive_params(self._h, min_len, max_dist))

    def scratch_usage(self):
        """aim_scratch_usage: (current, peak) device bytes of the context's scratch."""
        cur, peak = i64(), i64()
        _check(lib().aim_scratch_usage(self._h, ctypes.byref(cur), ctypes.byref(peak)))
        return cur.value, peak.value

    def prefilter(self, pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, *, enc: int, max_len: int,
                  alg, pen, max_score: int, lower, passed, stream=None):
        """aim_prefilter on device tensors: lower (int32) and passed (int8) per pair, in place."""
        b, _, a = self._args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg,
                             None, None, None, None, False)
        _check(lib().aim_prefilter(self._h, ctypes.byref(b), a, Penalties(*pen), max_score, _ptr(lower),
                                   _ptr(passed), _stream(stream)))

    def autotune(self, pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, *, enc, max_len, alg,
                 pen, max_score, score, status, cigar=None, cigar_off=None, want_cigar=True,
                 stream=None, reps=2):
        """aim_autotune; returns (params list of 13, best ms)."""
        b, r, a = self._args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg,
                             score, status, cigar, cigar_off, want_cigar)
        params = (i32 * 13)()
        ms = ctypes.c_double()
        _check(lib().aim_autotune(self._h, ctypes.byref(b), a, Penalties(*pen), max_score,
                                  ctypes.byref(r), _stream(stream), reps, params, ctypes.byref(ms)))
        return list(params), ms.value

    def tune_entries(self):
        """aim_tune_entries: [(kind, alg, bucket)], kind 0 batch tune, 1 WFA class tune."""
        cnt = i32()
        _check(lib().aim_tune_entries(self._h, 0, None, None, None, ctypes.byref(cnt)))
        k = (i32 * max(cnt.value, 1))()
        a = (i32 * max(cnt.value, 1))()
        b = (i32 * max(cnt.value, 1))()
        _check(lib().aim_tune_entries(self._h, cnt.value, k, a, b, ctypes.byref(cnt)))
        return [(k[i], a[i], b[i]) for i in range(cnt.value)]

    def tune_get(self, alg, max_len):
        params = (i32 * 13)()
        _check(lib().aim_tune_get(self._h, ALGORITHMS[alg] if isinstance(alg, str) else alg, max_len, params))
        return list(params)

    def tune_set(self, alg, max_len, params):
        arr = (i32 * 13)(*params)
        _check(lib().aim_tune_set(self._h, ALGORITHMS[alg] if isinstance(alg, str) else alg, max_len, arr))

    def tune_save(self, path):
        _check(lib().aim_tune_save(self._h, path.encode()))

    def tune_load(self, path):
        _check(lib().aim_tune_load(self._h, path.encode()))

    def graph_capture(self, pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, *, enc, max_len,
                      alg, pen, max_score, score, status, cigar=None, cigar_off=None, want_cigar=True,
                      stream=None):
        """aim_graph_capture; returns a Graph."""
        b, r, a = self._args(pat_seq, pat_off, pat_len, txt_seq, txt_off, txt_len, enc, max_len, alg,
                             score, status, cigar, cigar_off, want_cigar)
        h = vp()
        _check(lib().aim_graph_capture(self._h, ctypes.byref(b), a, Penalties(*pen), max_score,
                                       ctypes.byref(r), _stream(stream), ctypes.byref(h)))
        return Graph(h)

    def timing(self):
        """{phase: (total_ms, launches)} since the last reset (AIM_FLAG_TIMING)."""
        out = {}
        k = 0
        while True:
            name, ms, cnt = ctypes.c_char_p(), ctypes.c_double(), i64()
            rc = lib().aim_timing(self._h, k, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
            if rc == -6:
                return out
            _check(rc)
            out[name.value.decode()] = (ms.value, cnt.value)
            k += 1

    def last_call_stats(self) -> dict:
        """aim_last_call_stats as a dict (waits for the last call)."""
        st = CallStats()
        _check(lib().aim_last_call_stats(self._h, ctypes.byref(st)))
        out = {k: getattr(st, k) for k, _ in CallStats._fields_}
        out["full_store"] = list(st.full_store)
        out["wfa_class_pairs"] = list(st.wfa_class_pairs)
        out["wfa_class_window"] = list(st.wfa_class_window)
        return out

    def timing_reset(self):
        _check(lib().aim_timing_reset(self._h))

    def pack_2bit(self, enc: int, seq, off, length, out_words, out_off, seq_flags=None, stream=None):
        """aim_pack_2bit on device tensors."""
        _check(lib().aim_pack_2bit(self._h, length.numel(), enc, _ptr(seq), _ptr(off), _ptr(length),
                                   _ptr(out_words), out_words.numel(), _ptr(out_off), _ptr(seq_flags),
                                   _stream(stream)))


class Graph:
    """A captured aim_align_batch call (aim_graph)."""

    def __init__(self, h):
        self._h = h

    def launch(self, stream=None):
        _check(lib().aim_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().aim_graph_destroy(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(code):
    if code != 0:
        raise AimError(code, lib().aim_server_last_error().decode())


class Server:
    """aim_server: continuous batching of alignment requests (host arrays in,
    host arrays out)."""

    def __init__(self, device: int = 0, n_streams: int = 4, budget_bytes: int = 0,
                 max_batch_pairs: int = 0):
        h = vp()
        _scheck(lib().aim_server_create(device, ctypes.byref(ServerOptions(n_streams, 0, budget_bytes,
                                                                          max_batch_pairs)),
                                        ctypes.byref(h)))
        self._h = h

    def submit(self, alg, pen, max_score, pat, pat_off, pat_len, txt, txt_off, txt_len, *,
               enc=ENC_CODE, want_cigar=True) -> int:
        """Numpy arrays (uint8 bytes, int64 byte offsets, int32 lengths); copied at submit."""
        import numpy as np
        arrs = [np.ascontiguousarray(a) for a in (pat, pat_off, pat_len, txt, txt_off, txt_len)]
        ptr = lambda a: vp(a.ctypes.data) if a.size else None  # noqa: E731
        q = Request(ALGORITHMS[alg] if isinstance(alg, str) else alg, Penalties(*pen), max_score,
                    int(bool(want_cigar)), enc, len(arrs[2]), *[ptr(a) for a in arrs])
        rid = i64()
        _scheck(lib().aim_server_submit(self._h, ctypes.byref(q), ctypes.byref(rid)))
        return rid.value

    @staticmethod
    def _copy(res):
        import numpy as np
        n = res.n_pairs

        def arr(p, ct, cnt):
            if cnt == 0 or not p:
                return np.zeros(cnt, dtype=np.ctypeslib.as_array((ct * 1)()).dtype)
            return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ct)), shape=(cnt,)).copy()
        off = arr(res.cigar_off, ctypes.c_int64, n + 1)
        return (arr(res.score, ctypes.c_int32, n), arr(res.status, ctypes.c_int8, n),
                arr(res.cigar, ctypes.c_uint32, int(off[-1]) if n >= 0 and len(off) else 0), off,
                res.latency_us)

    def wait(self, rid: int, timeout_ms: int = -1, release: bool = True):
        """(score, status, cigar, cigar_off, latency_us) as numpy copies."""
        res = RequestResult()
        _scheck(lib().aim_server_wait(self._h, rid, timeout_ms, ctypes.byref(res)))
        out = self._copy(res)
        if release:
            _scheck(lib().aim_server_release(self._h, rid))
        return out

    def poll(self, rid: int):
        """None while running, else the wait() tuple (results released)."""
        res = RequestResult()
        rc = lib().aim_server_poll(self._h, rid, ctypes.byref(res))
        if rc == -5:
            return None
        _scheck(rc)
        out = self._copy(res)
        _scheck(lib().aim_server_release(self._h, rid))
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _scheck(lib().aim_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        _scheck(lib().aim_server_reset_stats(self._h))

    def close(self):
        if self._h:
            lib().aim_server_destroy(self._h)
            self._h = vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def version() -> str:
    return lib().aim_version().decode()
