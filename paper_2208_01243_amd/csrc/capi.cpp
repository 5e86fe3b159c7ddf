// C ABI of libaim.so: context, scratch management, validation and the
// orchestration of the alignment kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <mutex>
#include <string>
#include <vector>

#include "aim.h"
#include "aim_internal.h"

namespace {

thread_local std::string g_err;

aim_status fail(aim_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
aim_status fail(aim_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(AIM_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
  bool pooled = false;  // from the stream-ordered pool (hipMallocAsync)
};

}  // namespace

// Optional per-phase timing with events recorded on the launch stream.
struct PhaseTimer {
  struct Pending {
    const char *name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<const char *, std::pair<double, int64_t>>> totals;  // in first-seen order

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void flush() {
    for (auto &p : pending) {
      float ms = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        bool found = false;
        for (auto &t : totals)
          if (!strcmp(t.first, p.name)) { t.second.first += ms; t.second.second += 1; found = true; }
        if (!found) totals.push_back({p.name, {(double)ms, 1}});
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~PhaseTimer() {
    flush();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Launch parameters chosen per (algorithm, length bucket) by aim_autotune.
struct Tune {
  int32_t band_w0 = 32;       // first band width (32: 32 then 64; 64: 64 only)
  int32_t band_wpc = 16;      // resident wavefronts per CU for the first band tier
  int32_t sort = -1;          // length-sort the pairs first (-1: auto)
  int32_t wfa_ring_kb = 32;   // LDS per workgroup for the WFA score ring
  int32_t wfa_trace_kb = 16;  // LDS per workgroup for the WFA full store
  int32_t wfa_long_threads = 256;  // workgroup size for long WFA pairs
  int32_t band16 = 3;         // packed 16-bit band kernel when the value bound allows
                              // (1: the fill walks its pairs, 2: a separate walk kernel,
                              // 3: 2 for batches of at least SPLIT_MIN_PAIRS pairs, else 1)
  int32_t wfa_classes = 1;    // WFA pairs wider than the one-wavefront window: LDS-window
                              // classes (1) or straight to the HBM-ring pass (0)
  int32_t wfa_cls_threads[3] = {64, 128, 128};  // workgroup size of each window class
  int32_t wfa_cls_global = 7;  // bit c: class c + 1 keeps its ring in a global buffer, not LDS
  int32_t wfa_c16 = 0;         // one-wavefront window in units of 64 diagonals (0: from the batch)
};

// Launch parameters of one WFA window class, keyed by the class's length
// bucket (its extent bound, or the batch's max_len for the last class), so
// that one mixed batch runs each class with its own tuned configuration.
struct ClassTune {
  int32_t threads = 0;  // workgroup size (0: the batch tune's)
  int32_t global = -1;  // ring in a global slot (1) or LDS (0); -1: the batch tune's
};

// Every scratch buffer of one call.
struct Scratch {
  Buf order, hist;
  Buf flags, pflag, tflag, pat2, txt2, pat2off, txt2off, nruns, slot, tb32, tb64, full, list2,
      list3, counters, scan_tmp, spill, total, wring, warena1, warena2, warena3, wneed, wlists, pool, pooloff,
      wbits, wwalk, wlds, wgring, flist, genasm, wlong;
};

struct aim_graph {
  aim_context *c = nullptr;  // nullptr once the context is destroyed
  int32_t device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t generation = 0;
};

struct aim_context {
  int32_t device = 0;
  std::string arch;
  aim_options opt{};
  int32_t cus = 256;
  PhaseTimer timer;
  std::map<std::pair<int32_t, int32_t>, Tune> tunes;  // (alg, length bucket) -> tune
  std::map<std::pair<int32_t, int32_t>, ClassTune> class_tunes;  // (alg, class length bucket)
  std::set<aim_graph *> graphs;  // captured graphs still alive (detached when the context goes)
  const Tune *force = nullptr;  // set while the autotuner tries a candidate
  bool capturing = false;       // inside a hipGraph capture: no timing events
  // second stream (default priority) for the escalation tiers, which run
  // beside the first tier's traceback; fork / join through the two events
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Scratch grows in stream order on the running call's stream (astream):
  // the old buffer is freed and the new one allocated there, so a growing
  // context does not synchronise the device (and stall the other contexts'
  // streams).  ev_done marks the end of the last call's work; a call on
  // another stream waits for it first.
  hipStream_t astream = nullptr, done_stream = nullptr;
  hipEvent_t ev_done = nullptr;
  bool has_done = false;
  int64_t generation = 0;       // bumped whenever scratch is reallocated
  // Scratch of the running call: the context's own (grown on demand), or,
  // inside aim_align_batch_static, buffers carved from the static array.
  Scratch own;
  Scratch *sc = &own;
  // device bytes held by the context's own scratch, now and at most
  int64_t dev_bytes = 0, dev_peak = 0;
  // carving state of aim_align_batch_static (arena == nullptr otherwise)
  uint8_t *arena = nullptr;
  size_t arena_cap = 0, arena_top = 0;
  // the scratch budget the launch plans are sized for in this call
  // (a hard limit leaves the rest to the arrays that grow with the batch and
  // to the plans' own margins and minimum sizes: half, or 5/8 of a limit
  // under 1 GiB, where those minimums weigh more)
  int64_t limit() const {
    if (arena) return aim::STATIC_PLAN_BUDGET;
    if (!strict()) return opt.scratch_limit;
    return opt.scratch_limit >= ((int64_t)1 << 30) ? opt.scratch_limit / 2 : opt.scratch_limit / 8 * 3;
  }
  bool strict() const { return !arena && (opt.flags & AIM_FLAG_HARD_LIMIT); }
  // the last call's work counters (device) and size, for aim_last_call_stats
  const int32_t *last_cnt = nullptr;
  int64_t last_n = 0;
  int32_t last_window = 0;  // diagonals of the one-wavefront WFA window (0: not run)
  int32_t last_class_window[4] = {0, 0, 0, 0};  // windows of the LDS classes (0: none)
  int32_t last_class_bucket[4] = {-1, -1, -1, -1};  // their class-tune buckets
  // WFA-adaptive reduction parameters (aim_wfa_adaptive_params)
  int32_t ad_min = 10, ad_max = 50;
};

namespace {

aim_status ensure(aim_context *c, Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return AIM_OK;
  if (c->arena) {
    // static-array mode: carve, 256-byte aligned; never allocate or free
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (c->arena_top + need > c->arena_cap)
      return fail(AIM_ERR_INVALID_ARG,
                  "this batch needs more scratch than the static array holds (%zu bytes): "
                  "split it, or call aim_align_batch", c->arena_cap);
    b.p = c->arena + c->arena_top;
    b.bytes = need;
    b.pooled = false;
    c->arena_top += need;
    return AIM_OK;
  }
  if (c->capturing) return fail(AIM_ERR_INVALID_ARG, "scratch would grow during graph capture");
  hipStream_t as = c->astream;
  if (b.p) {
    // previously enqueued work may still use the old buffer: free it behind
    // that work on the call's stream, or after a device synchronisation
    if (b.pooled && as) {
      HIP_TRY(hipFreeAsync(b.p, as));
    } else {
      HIP_TRY(hipDeviceSynchronize());
      if (b.pooled)
        HIP_TRY(hipFreeAsync(b.p, nullptr));
      else
        HIP_TRY(hipFree(b.p));
    }
    c->dev_bytes -= (int64_t)b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;
  if (c->opt.flags & AIM_FLAG_HARD_LIMIT) {
    const int64_t room = c->opt.scratch_limit - c->dev_bytes;
    if ((int64_t)bytes > room)
      return fail(AIM_ERR_OOM, "scratch limit of %lld bytes reached (%lld held, %zu more needed)",
                  (long long)c->opt.scratch_limit, (long long)c->dev_bytes, bytes);
    want = std::min<size_t>(want, (size_t)room);
  }
  c->generation += 1;
  auto alloc = [&](size_t sz) { return as ? hipMallocAsync(&b.p, sz, as) : hipMalloc(&b.p, sz); };
  b.pooled = as != nullptr;
  hipError_t e = alloc(want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = alloc(bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(AIM_ERR_OOM, "cannot allocate %zu bytes of device scratch", bytes);
    }
    want = bytes;
  }
  b.bytes = want;
  c->dev_bytes += (int64_t)want;
  c->dev_peak = std::max(c->dev_peak, c->dev_bytes);
  return AIM_OK;
}

template <class T>
T *as(Buf &b) {
  return (T *)b.p;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

enum Counter {
  C_T1 = 0, C_T2, C_T3, C_L2, C_L3, C_SPILL, C_SPILL_W,
  C_W1, C_W1G, C_RL, C_FAIL, C_N0, C_N1, C_N2, C_N3, C_P0, C_P1, C_P2, C_P3, C_TB, C_DTB,
  C_M0, C_M1, C_M2, C_M3, C_WF, C_WS, C_FL, C_FR, C_LL, C_LW, C_LF,
  C_CL = 32,  // WFA window classes 1..4: list lengths, then their work counters (C_CL + 4)
  C_N = 48
};

// Smallest batch for which the packed band tier's traceback is walked by a
// separate kernel beside the escalation tiers by default.
constexpr int64_t SPLIT_MIN_PAIRS = 65536;
// Below this many pairs of reads of at most SMALL_BATCH_LEN bases the first
// tier is, by default, the 32-bit band (one pair per lane) rather than the
// packed band (two pairs per lane): 10,000 x 100 bp, 0.285 ms against 0.357 ms
// (longer reads, as the serving loop's merged batches of 100-1,000 bases,
// are better off on the packed band).
constexpr int64_t SMALL_BATCH_PAIRS = 16384;
constexpr int32_t SMALL_BATCH_LEN = 128;

// WFA requires a bounded ring of past wavefronts: max(x, o + e) <= this.
constexpr int32_t WFA_MAX_STEP = 1024;
// WFA-adaptive runs on 16-bit offsets over a window of every diagonal
constexpr int32_t WFA_ADAPTIVE_MAX_LEN = 16000;

aim_status check_pen(int32_t alg, const aim_penalties &pen) {
  if (alg < AIM_NW_LINEAR || alg > AIM_GENASM) return fail(AIM_ERR_INVALID_ARG, "unknown algorithm %d", alg);
  if (pen.match != 0) return fail(AIM_ERR_UNSUPPORTED, "match cost must be 0 (got %d)", pen.match);
  if (pen.mismatch <= 0 || pen.gap_extend <= 0 || pen.gap_open < 0)
    return fail(AIM_ERR_INVALID_ARG, "penalties need mismatch > 0, gap_extend > 0, gap_open >= 0");
  if (pen.mismatch > 65535 || pen.gap_extend > 65535 || pen.gap_open > 65535)
    return fail(AIM_ERR_INVALID_ARG, "penalties must not exceed 65535");
  if (alg == AIM_NW_LINEAR && pen.gap_open != 0)
    return fail(AIM_ERR_INVALID_ARG, "linear NW takes gap_open 0 (one gap base costs gap_extend)");
  if ((alg == AIM_WFA_AFFINE || alg == AIM_WFA_ADAPTIVE) &&
      (pen.mismatch > WFA_MAX_STEP || pen.gap_open + pen.gap_extend > WFA_MAX_STEP))
    return fail(AIM_ERR_UNSUPPORTED, "WFA needs mismatch and gap_open + gap_extend <= %d", WFA_MAX_STEP);
  return AIM_OK;
}

// Brackets one launch with timing events when AIM_FLAG_TIMING is set.
struct Phase {
  aim_context *c;
  hipStream_t s;
  const char *name;
  hipEvent_t a = nullptr;
  Phase(aim_context *c_, hipStream_t s_, const char *n) : c(c_), s(s_), name(n) {
    if ((c->opt.flags & AIM_FLAG_TIMING) && !c->capturing && !c->arena) {
      a = c->timer.get();
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~Phase() {
    if (!a) return;
    hipEvent_t b = c->timer.get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->timer.pending.push_back({name, a, b});
    if (c->timer.pending.size() > 8192) c->timer.flush();
  }
};

constexpr int32_t MAX_LEN_LIMIT = 1 << 20;
constexpr int32_t SLOT_CAP = 128;  // at most this many runs per pair held before compaction



int32_t len_bucket_host(int32_t L) {
  int32_t b = 0;
  while ((1 << b) < L + 1 && b < 30) ++b;
  return b;
}

// Built-in defaults where no tune is kept, from the autotuner on MI355X:
// - WFA, reads of 4,096 bases or more (500,000 pairs of 100-10,000 bases at
//   0.5-10 % error: 489 ms per call against 518 ms): a one-wavefront window
//   of 64 diagonals (pairs that are going to be wide leave it early, rather
//   than after filling a wider window) and 256-thread workgroups for the
//   widest window class;
// - GenASM: no length sort below 512 bases (1,000,000 x 150 bp: 2.17 ms
//   against 2.28 ms; fixed-length reads gain nothing from it).
Tune default_tune(int32_t alg, int32_t L) {
  Tune t;
  if (alg == AIM_WFA_AFFINE && L >= 4096) {
    t.wfa_c16 = 1;
    t.wfa_cls_threads[2] = 256;
  }
  if (alg == AIM_GENASM) t.sort = L >= 512 ? 1 : 0;
  return t;
}

Tune tune_for(aim_context *c, int32_t alg, int32_t L) {
  if (c->force) return *c->force;
  auto it = c->tunes.find({alg, len_bucket_host(L)});
  return it == c->tunes.end() ? default_tune(alg, L) : it->second;
}

// The penalties the wavefront kernels run on: x, o, e and the threshold
// divided by g = gcd(x, o, e).  Every alignment costs a multiple of g, so the
// optimum, the CIGAR (each comparison of the canonical order scales by g) and
// the threshold test (g s' > S_max exactly when s' > floor(S_max / g)) are
// unchanged, while the score loop takes 1/g of the steps (with 4/6/2, every
// odd score was an empty wavefront) and the ring holds max(x, o + e) / g + 1
// scores.  Scores go out as g s'.
aim::Scoring wfa_scoring(const aim::Scoring &P) {
  const int32_t g = std::gcd(P.x, std::gcd(P.o, P.e));
  if (g <= 1) return P;
  aim::Scoring R = P;
  R.x /= g;
  R.o /= g;
  R.e /= g;
  R.max_score = P.max_score >= 0 ? P.max_score / g : -1;
  R.unit = g;
  return R;
}

// WFA: the one-wavefront score pass (16-bit LDS ring, fused walk) when the
// batch allows it, else the score pass with the ring in LDS; then the score
// pass with the ring in HBM for pairs too wide for either (fused walk too);
// then the fallback pass (full store + walk) by store-size class for pairs
// whose origin codes did not fit.
// `order` lists the pairs to align (nullptr: all n), `order_count` its length
// on the device (nullptr: n).
// WFA-adaptive: every pair through the packed wavefront kernel with its
// ring in a global slot and a window of every diagonal the batch can reach,
// plus the reduction step.  Wk lists the pairs (a re-run when Wk.direct).
aim_status run_wfa_adaptive(aim_context *c, const aim::Seqs &S, const aim::Outs &O, const aim::Scoring &Pin,
                            int64_t n, int32_t L, int32_t *cnt, const aim::Work &Wk, const Tune &tu,
                            hipStream_t s) {
  aim_status st;
  const aim::Scoring P = wfa_scoring(Pin);
  aim::WfaLds D{};
  D.R = std::max(P.x, P.o + P.e) + 1;
  D.MG = 2 * D.R + 4;
  D.W = (2 * L + 2 + 3) / 4 * 4 + 4;
  D.seq_words = (L + 31) / 32;
  D.s_cap = 16000;
  D.my_class = 1;
  D.ad_min = c->ad_min;
  D.ad_max = c->ad_max;
  D.ad_dropped = reinterpret_cast<unsigned long long *>(cnt + C_N);
  D.walk_fail = cnt + C_WF;
  D.walk_skip = cnt + C_WS;
  const int32_t threads = tu.wfa_cls_threads[0];
  // the ring in LDS when a window of every diagonal is small (short reads:
  // no global round trips per score, and the walk's tokens in LDS too),
  // else in a global slot
  const bool lds_ring = aim::wfa_lds_bytes(D.W, D.MG, D.R, P.e, D.seq_words, false) <= 24 * 1024;
  const size_t lds = aim::wfa_lds_bytes(D.W, D.MG, D.R, P.e, D.seq_words, !lds_ring);
  if (lds > 160 * 1024) return fail(AIM_ERR_UNSUPPORTED, "WFA-adaptive: sequences too long to stage");
  const int32_t per_cu = (int32_t)std::max<size_t>(1, std::min<size_t>(160 * 1024 / lds, 2048 / threads));
  int32_t nslots = (int32_t)std::min<int64_t>(n, (int64_t)c->cus * per_cu);
  // per workgroup slot: the ring (with its guard word) and, with CIGARs, the
  // score table and the origin codes of every kept score, within a third of
  // the budget each way (fewer workgroups when they do not fit)
  D.gring_slot = lds_ring ? 0 : (aim::wfa_ring_words(D.W, D.MG, D.R, P.e) + 1 + 63) / 64 * 64;
  const int64_t share = c->limit() / 3;
  if (!lds_ring) nslots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nslots, share / (D.gring_slot * 4)));
  // scores kept: up to what any alignment of the batch can cost (2 L ops at
  // the dearest step), at most s_cap; codes: up to the widest row at every
  // kept score, at most 4 MiB per slot (a pair needing more gets no CIGAR)
  const int64_t steps = std::min<int64_t>(D.s_cap, 2 * (int64_t)L * std::max(P.x, P.o + P.e) + 1) + 1;
  D.steps_cap = P.want_cigar ? (int32_t)steps : 0;
  if (P.want_cigar) {
    const int64_t fixed = (int64_t)D.steps_cap * 12;
    nslots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nslots, share / (fixed + (256 << 10))));
    const int64_t most = std::min<int64_t>(steps * (D.W / 2 + 1), (int64_t)4 << 20);
    D.code_cap = std::max<int64_t>(std::min<int64_t>(share / nslots - fixed, most), 256 << 10);
  }
  D.code_slot = ((int64_t)D.steps_cap * 12 + D.code_cap + 255) / 256 * 256;
  if (!lds_ring && (st = ensure(c, c->sc->wgring, (size_t)D.gring_slot * 4 * nslots))) return st;
  if ((st = ensure(c, c->sc->wlds, std::max<size_t>((size_t)D.code_slot * nslots, 256)))) return st;
  D.gring = lds_ring ? nullptr : as<uint32_t>(c->sc->wgring);
  D.codes = as<uint8_t>(c->sc->wlds);
  c->last_class_window[0] = D.W;
  Phase ph(c, s, Wk.direct ? "wfa_adaptive_rerun" : "wfa_adaptive");
  HIP_TRY(aim::launch_wfa_lds(S, O, P, Wk, D, threads, nslots, s));
  return AIM_OK;
}

// GenASM: one launch over the listed pairs, each wavefront with a slot of
// every edit level a window can need (k + 1, at most 65, in whole sweeps).  The tune's
// wavefronts per CU (in 256-thread blocks), fewer when the slots would pass a
// quarter of the budget.
aim_status run_genasm(aim_context *c, const aim::Seqs &S, const aim::Outs &O, const aim::Scoring &P, int64_t n,
                      const aim::Work &Wk, const Tune &tu, hipStream_t s) {
  const int32_t levels = aim::genasm_levels(P.max_score);
  const int64_t block_bytes = aim::genasm_block_words(levels) * 8;
  const int64_t per_cu = std::max<int64_t>(1, tu.band_wpc / 4);
  int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)c->cus * per_cu);
  blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, c->limit() / 4 / block_bytes));
  aim_status st = ensure(c, c->sc->genasm, (size_t)(blocks * block_bytes));
  if (st) return st;
  Phase ph(c, s, Wk.direct ? "genasm_rerun" : "genasm");
  HIP_TRY(aim::launch_genasm(S, O, P, Wk, as<uint64_t>(c->sc->genasm), levels, (int32_t)blocks, s));
  return AIM_OK;
}

// The memory-bounded long pass of a WFA call (CIGARs wanted): up to 8
// workgroups, each with a slot of 16 ring checkpoints, a width per score, a
// code window of 1/64 of the budget (1 to 16 MiB) and the walk tokens,
// within 1/16 of the budget; none (nslots 0) when one slot does not fit.
aim_status wfa_long_plan(aim_context *c, int32_t L, const aim::Scoring &P, const aim::WfaPlan &pl, bool i16,
                         aim::WfaLong &LG, int32_t &nslots) {
  LG = aim::WfaLong{};
  nslots = 0;
  LG.R = pl.R;
  LG.wcap = 2 * L + 1;
  LG.seq_words = pl.seq_words;
  LG.ck_cap = 16;
  LG.sw_cap = (int32_t)std::min<int64_t>(1 << 20, (int64_t)std::max(P.x, P.o + P.e) * (2 * (int64_t)L + 1) + 2);
  LG.wt_cap = std::min(LG.sw_cap, 1 << 16);
  LG.tok_cap = 2 * (2 * L + 1) + 8;
  LG.code_cap = std::max<int64_t>(1 << 20, std::min<int64_t>(16 << 20, c->limit() / 64)) / 16 * 16;
  LG.slot_words = aim::wfa_long_slot_words(LG, i16);
  const int64_t fit = c->limit() / 16 / (LG.slot_words * 4);
  if (fit < 1) return AIM_OK;
  nslots = (int32_t)std::min<int64_t>(8, fit);
  aim_status st = ensure(c, c->sc->wlong, (size_t)LG.slot_words * 4 * nslots);
  if (st) return st;
  LG.slots = as<int32_t>(c->sc->wlong);
  return AIM_OK;
}

aim_status run_wfa(aim_context *c, const aim::Seqs &S, const aim::Outs &O, const aim::Scoring &Pin,
                   int64_t n, int32_t L, bool plain, int32_t *cnt, const int32_t *order,
                   const int32_t *order_count, const Tune &tu, hipStream_t s) {
  aim_status st;
  const aim::Scoring P = wfa_scoring(Pin);
  const aim::WfaPlan pl = aim::wfa_plan(L, P, c->limit(), c->cus, plain, tu.wfa_ring_kb,
                                        tu.wfa_trace_kb, tu.wfa_long_threads, c->strict());
  if ((st = ensure(c, c->sc->wneed, (size_t)n * 8))) return st;
  // lists: [0] the HBM-ring pass, [1-4] full-store classes, [5] unused,
  // [6-9] LDS-window classes, [10] predicted extents
  if ((st = ensure(c, c->sc->wlists, (size_t)n * 4 * 12))) return st;
  int32_t *lists = as<int32_t>(c->sc->wlists);
  aim::WfaLaunch WL{};
  WL.R = pl.R;
  WL.seq_words = pl.seq_words;
  WL.ring_list = lists;
  WL.ring_count = cnt + C_RL;
  for (int k = 0; k < 4; ++k) {
    WL.need_list[k] = lists + (int64_t)n * (k + 1);
    WL.need_count[k] = cnt + C_N0 + k;
    WL.need_cap[k] = pl.need_cap[k];
    WL.need_max[k] = cnt + C_M0 + k;
  }
  WL.need = as<int64_t>(c->sc->wneed);
  WL.walk_fail = cnt + C_WF;
  WL.walk_skip = cnt + C_WS;
  // long pairs: the memory-bounded pass, when its slots fit the budget
  aim::WfaLong LG{};
  int32_t long_slots = 0;
  const bool long_i16 = L <= aim::WFA16_MAX_LEN;
  if (P.want_cigar && !plain) {
    if ((st = wfa_long_plan(c, L, P, pl, long_i16, LG, long_slots))) return st;
    if (long_slots > 0) {
      WL.long_list = lists + (int64_t)n * 11;
      WL.long_count = cnt + C_LL;
      LG.failed = cnt + C_LF;
    }
  }
  const int32_t slots = (int32_t)std::min<int64_t>(n, (int64_t)c->cus * 8);
  // one wavefront per pair with 16-bit offsets over a window of 64 C diagonals
  int32_t C16 = (int32_t)std::min<int64_t>(4, std::max<int64_t>(1, (pl.wcap + 63) / 64));
  if (tu.wfa_c16 > 0) C16 = std::min(C16, tu.wfa_c16);
  const bool w16 = !plain && L <= aim::WFA16_MAX_LEN && pl.R <= 32 && pl.seq_words > 0 &&
                   aim::wfa_score16_lds(WL, P.e, C16) <= 48 * 1024;
  WL.store16 = w16;  // the full store of the fallback pass holds 16-bit offsets
  // Window classes for the pairs that leave the one-wavefront window: LDS
  // windows of growing width, each pair routed to the first that holds its
  // predicted extent, then the HBM-ring pass for the rest.
  struct LdsClass {
    int32_t W, threads, nslots;
    bool global;
    int32_t half;  // routing bound: pairs predicted to span at most this many diagonals each side
  };
  std::vector<LdsClass> cls;
  const int32_t MG = 2 * pl.R + 4;
  if (w16 && tu.wfa_classes) {
    const size_t lds_cap = 160 * 1024;
    int32_t wmax = 0;
    for (int32_t w = 512; w <= 16384; w += 512)
      if (aim::wfa_lds_bytes(w, MG, pl.R, P.e, pl.seq_words, false) <= lds_cap) wmax = w;
    // classes by predicted extent: up to 512, 1536, then the rest.  An LDS
    // class holds a window of twice its bound (the widest that fits LDS for
    // the last); a global-ring class holds every diagonal of the batch's
    // pairs (its window costs memory only), so no pair leaves it and the
    // bound only picks the workgroup size.
    const int32_t full = (int32_t)std::min<int64_t>(32768, (2 * (int64_t)L + 2 + 3) / 4 * 4 + 4);
    const int32_t bound[3] = {512, 1536, INT32_MAX};
    int32_t prev_half = 32 * C16;
    for (int k = 0; k < 3; ++k) {
      // this class's own tune, if one is kept for its length bucket
      const int32_t cb = len_bucket_host(k < 2 ? bound[k] : L);
      const auto ct = c->class_tunes.find({AIM_WFA_AFFINE, cb});
      const ClassTune *ctp = ct == c->class_tunes.end() ? nullptr : &ct->second;
      const bool glob = (ctp && ctp->global >= 0) ? ctp->global != 0 : ((tu.wfa_cls_global >> k) & 1) != 0;
      const int32_t w = glob ? full : std::min<int64_t>((int64_t)2 * std::min(bound[k], wmax / 2), wmax);
      const int32_t half = glob ? bound[k] : w / 2;
      if (std::min(half, w / 2) <= prev_half) continue;
      const size_t lds = aim::wfa_lds_bytes(w, MG, pl.R, P.e, pl.seq_words, glob);
      if (lds > lds_cap) continue;
      const int32_t th = (ctp && ctp->threads > 0) ? ctp->threads : tu.wfa_cls_threads[k];
      c->last_class_bucket[cls.size()] = cb;
      const int32_t per_cu = (int32_t)std::max<size_t>(1, std::min<size_t>(lds_cap / lds, 2048 / th));
      cls.push_back({w, th, (int32_t)std::min<int64_t>(n, (int64_t)c->cus * per_cu), glob, half});
      prev_half = std::min(half, w / 2);
      if (prev_half > L) break;  // every pair fits: no wider class needed
    }
    // a last class whose window holds every pair takes whatever the earlier
    // ones do not
    if (!cls.empty() && cls.back().W >= 2 * L + 2) cls.back().half = INT32_MAX;
  }
  aim::WfaRoute route{};
  if (!plain && w16) {
    route.nclass = (int32_t)cls.size() + 1;
    for (size_t k = 0; k < cls.size(); ++k) {
      route.half[k + 1] = cls[k].half;
      route.list[k + 1] = lists + (int64_t)n * (6 + k);
      route.count[k + 1] = cnt + C_CL + (int32_t)k;
    }
    route.half[route.nclass] = INT32_MAX;
    route.list[route.nclass] = lists;  // the HBM-ring pass
    route.count[route.nclass] = cnt + C_RL;
    route.pred = lists + (int64_t)n * 10;
  }
  if (w16) {
    const int32_t nslots16 = (int32_t)std::min<int64_t>(n, (int64_t)c->cus * 28);
    aim::WfaLaunch A = WL;
    if (P.want_cigar) {
      // origin codes for the fused walk: every score up to the threshold, at
      // most WFA16_WALK_STEPS (pairs above go to the full-store pass)
      // and within an eighth of the scratch budget
      A.bits_steps = P.max_score >= 0 ? std::min(P.max_score + 1, aim::WFA16_WALK_STEPS)
                                      : aim::WFA16_WALK_STEPS;
      A.bits_steps = (int32_t)std::max<int64_t>(
          1, std::min<int64_t>(A.bits_steps, c->limit() / 8 / ((int64_t)nslots16 * (C16 * 32 + 32))));
      // rows of C16 x 32 bytes plus 32 bytes of padding
      if ((st = ensure(c, c->sc->wbits, (size_t)nslots16 * A.bits_steps * (C16 * 32 + 32)))) return st;
      A.bits = as<uint8_t>(c->sc->wbits);
    }
    A.route = route;
    aim::Work W{order, order_count, n, cnt + C_W1, nullptr, nullptr, 0};
    {
      Phase ph(c, s, "wfa_score");
      HIP_TRY(aim::launch_wfa_score16(S, O, P, W, A, C16, nslots16, s));
    }
    c->last_window = 64 * C16;
    // the LDS-window classes, narrowest first; origin codes in one buffer
    // the classes share (they run one after the other on this stream)
    std::vector<aim::WfaLds> LL(cls.size());
    size_t code_bytes = 0, ring_bytes = 0;
    for (size_t k = 0; k < cls.size(); ++k) {
      aim::WfaLds &D = LL[k];
      D.W = cls[k].W;
      D.MG = MG;
      D.R = pl.R;
      D.seq_words = pl.seq_words;
      D.s_cap = 16000;
      D.my_class = (int32_t)k + 1;
      D.route = route;
      // scores and widest row a pair of this class is expected to need (a
      // pair that needs more leaves its codes to the full-store pass)
      const int32_t bnd = cls[k].half == INT32_MAX ? D.W / 2 : std::min(cls[k].half, D.W / 2);
      D.steps_cap = P.want_cigar ? (int32_t)std::min<int64_t>(2 * (int64_t)D.W + 64, 8 * (int64_t)bnd + 64) : 0;
      // Per workgroup slot: the score table, the ring when it is global, and
      // the origin codes (at most every score's widest row).  The classes run
      // in turn and share one code buffer and one ring buffer, each within a
      // third of the scratch budget: fewer workgroups when the slots would
      // not fit (at least one, with at least 64 KB of codes).
      // (plus the guard word before the rows)
      D.gring_slot = cls[k].global ? (aim::wfa_ring_words(D.W, MG, pl.R, P.e) + 1 + 63) / 64 * 64 : 0;
      const int64_t share = c->limit() / 3;
      const int64_t fixed = (int64_t)D.steps_cap * 12 + D.gring_slot * 4;
      cls[k].nslots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cls[k].nslots, share / (fixed + (64 << 10))));
      D.code_cap = P.want_cigar ? std::max<int64_t>(std::min<int64_t>((int64_t)D.steps_cap * (bnd / 2 + 1),
                                                                      share / cls[k].nslots - fixed),
                                                    64 << 10)
                                : 0;
      D.code_slot = ((int64_t)D.steps_cap * 12 + D.code_cap + 255) / 256 * 256;
      ring_bytes = std::max(ring_bytes, (size_t)D.gring_slot * 4 * cls[k].nslots);
      for (int q = 0; q < 4; ++q) {
        D.need_cap[q] = WL.need_cap[q];
        D.need_list[q] = WL.need_list[q];
        D.need_count[q] = WL.need_count[q];
        D.need_max[q] = WL.need_max[q];
      }
      D.need = WL.need;
      D.long_list = WL.long_list;
      D.long_count = WL.long_count;
      D.walk_fail = WL.walk_fail;
      D.walk_skip = WL.walk_skip;
      code_bytes = std::max(code_bytes, (size_t)D.code_slot * cls[k].nslots);
    }
    for (size_t k = 0; k < cls.size() && k < 4; ++k) c->last_class_window[k] = cls[k].W;
    if (!cls.empty()) {
      if ((st = ensure(c, c->sc->wlds, std::max<size_t>(code_bytes, 256)))) return st;
      if (ring_bytes && (st = ensure(c, c->sc->wgring, ring_bytes))) return st;
      for (size_t k = 0; k < cls.size(); ++k) {
        LL[k].codes = as<uint8_t>(c->sc->wlds);
        LL[k].gring = cls[k].global ? as<uint32_t>(c->sc->wgring) : nullptr;
        aim::Work WC{route.list[k + 1], route.count[k + 1], n, cnt + C_CL + 4 + (int32_t)k, nullptr, nullptr, 0};
        static const char *cls_names[4] = {"wfa_lds1", "wfa_lds2", "wfa_lds3", "wfa_lds4"};
        Phase ph(c, s, cls_names[k]);
        HIP_TRY(aim::launch_wfa_lds(S, O, P, WC, LL[k], cls[k].threads, cls[k].nslots, s));
      }
    }
  } else if (!plain && pl.wcap_lds > 0) {
    aim::WfaLaunch A = WL;
    A.wcap = pl.wcap_lds;
    aim::Work W{order, order_count, n, cnt + C_W1, nullptr, nullptr, 0};
    Phase ph(c, s, "wfa_score");
    HIP_TRY(aim::launch_wfa_score(S, O, P, W, A, nullptr, true, slots, 64, false, s));
  }
  {
    // pairs whose wavefronts outgrew the LDS ring (all pairs for the plain path)
    const int64_t pad = aim::wfa_ring_pad(pl.wcap);  // read margin at both ends
    if ((st = ensure(c, c->sc->wring, (size_t)(pl.ring_slot_words * pl.ring_slots + 2 * pad) * 4))) return st;
    aim::WfaLaunch B = WL;
    B.wcap = pl.wcap;
    B.slot_words = pl.ring_slot_words;
    B.ring_list = lists + (int64_t)n * 5;  // never reached: wcap bounds every width
    B.ring_count = cnt + C_FAIL;
    const bool all = plain || (!w16 && pl.wcap_lds == 0);
    int32_t grid = all ? std::min<int32_t>(slots, pl.ring_slots) : pl.ring_slots;
    if (P.want_cigar && !plain) {
      // origin codes for the fused walk: 1/4 of the budget over the workgroups
      B.walk_steps = P.max_score >= 0 ? std::min(P.max_score + 1, aim::WFA_WALK_STEPS) : aim::WFA_WALK_STEPS;
      B.walk_tok = 2 * (2 * L + 1) + 8;
      // (no more than every kept score at the widest wavefront needs)
      const int64_t most = (int64_t)B.walk_steps * ((pl.wcap + 1) / 2) + 16;
      B.walk_codes = std::min<int64_t>(
          most, std::max<int64_t>(256 << 10, std::min<int64_t>(16 << 20, c->limit() / 4 / grid)));
      B.walk_codes = (B.walk_codes + 15) / 16 * 16;
      B.walk_slot = ((int64_t)B.walk_steps * 16 + B.walk_codes + (int64_t)B.walk_tok * 4 + 255) / 256 * 256;
      // the slots (each at least 256 KB of codes) within a quarter of the
      // budget: fewer workgroups rather than more memory
      grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(grid, c->limit() / 4 / B.walk_slot));
      if ((st = ensure(c, c->sc->wwalk, (size_t)B.walk_slot * grid))) return st;
      B.walk = as<uint8_t>(c->sc->wwalk);
    }
    aim::Work W{all ? order : lists, all ? order_count : cnt + C_RL, n, cnt + C_W1G, nullptr, nullptr, 0};
    Phase ph(c, s, "wfa_score_hbm");
    HIP_TRY(aim::launch_wfa_score(S, O, P, W, B, as<int32_t>(c->sc->wring) + pad, false, grid,
                                  plain ? 64 : pl.ring_threads, !plain && L <= aim::WFA16_MAX_LEN, s));
  }
  if (!P.want_cigar) return AIM_OK;
  // fallback pass by class: 0 LDS arena, 1-3 HBM slots of growing size
  Buf *arena[4] = {nullptr, &c->sc->warena1, &c->sc->warena2, &c->sc->warena3};
  static const char *names[4] = {"wfa_trace_lds", "wfa_trace_1m", "wfa_trace_16m", "wfa_trace_192m"};
  for (int k = 0; k < 4; ++k) {
    if (k == 0 && (plain || pl.lds_arena_words <= 0)) continue;
    aim::WfaLaunch T = WL;
    T.full_in_lds = k == 0;
    T.slot_words = k == 0 ? pl.lds_arena_words : pl.need_cap[k];
    int32_t *hbm = nullptr;
    if (k > 0) {
      if ((st = ensure(c, *arena[k], (size_t)pl.pool_words[k] * 4))) return st;
      hbm = as<int32_t>(*arena[k]);
      T.slot_need_max = WL.need_max[k];
      T.pool_words = pl.pool_words[k];
    }
    aim::Work W{WL.need_list[k], WL.need_count[k], n, cnt + C_P0 + k, nullptr, nullptr, 0};
    Phase ph(c, s, names[k]);
    // the LDS class: as many workgroups as the LDS of a CU holds (up to 20)
    const int32_t lds_slots = (int32_t)std::min<int64_t>(
        n, (int64_t)c->cus * std::max(1, std::min(20, 160 / std::max(1, tu.wfa_trace_kb))));
    HIP_TRY(aim::launch_wfa_trace(S, O, P, W, T, hbm, k == 0 ? lds_slots : pl.arena_slots[k],
                                  plain ? 64 : pl.threads[k], w16, s));
  }
  if (long_slots > 0) {
    aim::Work W{WL.long_list, cnt + C_LL, n, cnt + C_LW, nullptr, nullptr, 0};
    Phase ph(c, s, "wfa_long");
    HIP_TRY(aim::launch_wfa_long(S, O, P, W, LG, long_slots, aim::WGMAX_THREADS, long_i16, s));
  }
  return AIM_OK;
}

}  // namespace

extern "C" {

const char *aim_last_error(void) { return g_err.c_str(); }

const char *aim_version(void) { return "aim-mi355x 0.1 (gfx950)"; }

aim_status aim_timing(aim_context *c, int32_t idx, const char **name, double *total_ms,
                      int64_t *launches) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(c->device);
  c->timer.flush();
  if (idx < 0 || idx >= (int32_t)c->timer.totals.size()) return fail(AIM_ERR_NOT_FOUND, "no phase %d", idx);
  const auto &t = c->timer.totals[(size_t)idx];
  if (name) *name = t.first;
  if (total_ms) *total_ms = t.second.first;
  if (launches) *launches = t.second.second;
  return AIM_OK;
}

aim_status aim_timing_reset(aim_context *c) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard g(c->device);
  c->timer.flush();
  c->timer.totals.clear();
  return AIM_OK;
}

aim_status aim_create(aim_context **ctx, int32_t device, const aim_options *opt) {
  g_err.clear();
  if (!ctx) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  *ctx = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AIM_ERR_INVALID_ARG, "device %d out of range (have %d)", device, ndev);
  aim_options o{};
  if (opt) o = *opt;
  if (o.kernel != AIM_KERNEL_AUTO && o.kernel != AIM_KERNEL_PLAIN)
    return fail(AIM_ERR_INVALID_ARG, "unknown kernel option %d", o.kernel);
  if (o.scratch_limit < 0) return fail(AIM_ERR_INVALID_ARG, "scratch_limit < 0");
  if (o.scratch_limit == 0) o.scratch_limit = (int64_t)64 << 30;
  if (o.flags & ~(AIM_FLAG_TIMING | AIM_FLAG_STATIC_SCRATCH | AIM_FLAG_NO_PREFILTER | AIM_FLAG_HARD_LIMIT))
    return fail(AIM_ERR_INVALID_ARG, "unknown option flags 0x%x", o.flags);
  auto *c = new aim_context();
  c->device = device;
  c->opt = o;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    if (prop.multiProcessorCount > 0) c->cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
  }
  {
    DeviceGuard g(device);
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess) {
      if (c->aux) (void)hipStreamDestroy(c->aux);
      if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
      if (c->ev_join) (void)hipEventDestroy(c->ev_join);
      delete c;
      return fail(AIM_ERR_HIP, "could not create the context's stream and events");
    }
    if (o.flags & AIM_FLAG_STATIC_SCRATCH) {
      // set-up of aim_align_batch_static on this device
      void *base = nullptr;
      const hipError_t e = aim::static_scratch_address(device, &base);
      if (e != hipSuccess) {
        (void)hipEventDestroy(c->ev_done);
        (void)hipEventDestroy(c->ev_join);
        (void)hipEventDestroy(c->ev_fork);
        (void)hipStreamDestroy(c->aux);
        delete c;
        return fail(AIM_ERR_HIP, "static scratch array: %s", hipGetErrorString(e));
      }
    }
  }
  *ctx = c;
  return AIM_OK;
}

void aim_destroy(aim_context *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  for (aim_graph *gr : c->graphs) gr->c = nullptr;  // their launches now fail; destroy still frees them
  c->graphs.clear();
  (void)hipDeviceSynchronize();
  Buf *all[] = {&c->own.order, &c->own.hist, &c->own.flags, &c->own.pflag, &c->own.tflag, &c->own.pat2, &c->own.txt2, &c->own.pat2off, &c->own.txt2off,
                &c->own.nruns, &c->own.slot, &c->own.tb32, &c->own.tb64, &c->own.full, &c->own.list2, &c->own.list3,
                &c->own.counters, &c->own.scan_tmp, &c->own.spill, &c->own.total, &c->own.wring, &c->own.warena1,
                &c->own.warena2, &c->own.warena3, &c->own.wneed, &c->own.wlists, &c->own.pool, &c->own.pooloff, &c->own.wbits, &c->own.wwalk, &c->own.wlds, &c->own.wgring, &c->own.flist,
                &c->own.genasm, &c->own.wlong};
  for (Buf *b : all)
    if (b->p) (void)(b->pooled ? hipFreeAsync(b->p, nullptr) : hipFree(b->p));
  (void)hipDeviceSynchronize();
  if (c->ev_done) (void)hipEventDestroy(c->ev_done);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
}

aim_status aim_pack_2bit(aim_context *c, int64_t n, int32_t enc, const uint8_t *seq,
                         const int64_t *off, const int32_t *len, uint64_t *out_words,
                         int64_t words_cap, int64_t *out_off, int8_t *seq_flags, void *stream) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 0) return fail(AIM_ERR_INVALID_ARG, "n_seqs < 0");
  if (enc != AIM_ENC_ASCII && enc != AIM_ENC_CODE) return fail(AIM_ERR_INVALID_ARG, "enc must be ASCII or CODE");
  if (!out_off || (n > 0 && (!seq || !off || !len || (!out_words && words_cap > 0))) || words_cap < 0)
    return fail(AIM_ERR_INVALID_ARG, "NULL buffer or negative capacity");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t tmp = aim::scan_tmp_elems(n) + (size_t)n + 2;
  aim_status st = ensure(c, c->sc->scan_tmp, tmp * sizeof(int64_t));
  if (st) return st;
  HIP_TRY(aim::launch_pack(n, enc, seq, off, len, INT32_MAX, out_words, words_cap, out_off, seq_flags,
                           as<int64_t>(c->sc->scan_tmp), s));
  return AIM_OK;
}

// Validation shared by the calls that take a batch (no device work).
static aim_status check_batch(const aim_batch *B) {
  if (!B) return fail(AIM_ERR_INVALID_ARG, "NULL batch");
  const int64_t n = B->n_pairs;
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(AIM_ERR_INVALID_ARG, "n_pairs out of range");
  if (B->max_len < 0 || B->max_len > MAX_LEN_LIMIT)
    return fail(AIM_ERR_INVALID_ARG, "max_len must be in [0, %d]", MAX_LEN_LIMIT);
  if (B->enc < AIM_ENC_ASCII || B->enc > AIM_ENC_2BIT) return fail(AIM_ERR_INVALID_ARG, "unknown encoding %d", B->enc);
  if (n > 0 && (!B->pat_seq || !B->pat_off || !B->pat_len || !B->txt_seq || !B->txt_off || !B->txt_len))
    return fail(AIM_ERR_INVALID_ARG, "NULL sequence array");
  return AIM_OK;
}

// The batch as 2-bit words (packed into scratch unless it already is) and
// the per-pair validity flags in c->sc->flags.
static aim_status prep_inputs(aim_context *c, const aim_batch *B, hipStream_t s, aim::Seqs &S) {
  aim_status st;
  const int64_t n = B->n_pairs;
  const int32_t L = B->max_len;
  if ((st = ensure(c, c->sc->flags, (size_t)n))) return st;
  const int8_t *pf = nullptr, *tf = nullptr;
  Phase ph_prep(c, s, "prep");
  if (B->enc == AIM_ENC_2BIT) {
    S = {(const uint64_t *)B->pat_seq, B->pat_off, B->pat_len,
         (const uint64_t *)B->txt_seq, B->txt_off, B->txt_len};
  } else {
    const size_t words = (size_t)n * ((L + 31) / 32) + 1;
    if ((st = ensure(c, c->sc->pat2, words * 8))) return st;
    if ((st = ensure(c, c->sc->txt2, words * 8))) return st;
    if ((st = ensure(c, c->sc->pat2off, (n + 1) * 8))) return st;
    if ((st = ensure(c, c->sc->txt2off, (n + 1) * 8))) return st;
    if ((st = ensure(c, c->sc->pflag, n))) return st;
    if ((st = ensure(c, c->sc->tflag, n))) return st;
    // lengths above max_len are flagged invalid below; one slot of
    // ceil(max_len / 32) words per sequence (the buffers hold n of them):
    // one launch per side, no offset scan
    HIP_TRY(aim::launch_pack_strided(n, B->enc, (const uint8_t *)B->pat_seq, B->pat_off, B->pat_len, L,
                                     as<uint64_t>(c->sc->pat2), (int64_t)words, as<int64_t>(c->sc->pat2off),
                                     as<int8_t>(c->sc->pflag), s));
    HIP_TRY(aim::launch_pack_strided(n, B->enc, (const uint8_t *)B->txt_seq, B->txt_off, B->txt_len, L,
                                     as<uint64_t>(c->sc->txt2), (int64_t)words, as<int64_t>(c->sc->txt2off),
                                     as<int8_t>(c->sc->tflag), s));
    S = {as<uint64_t>(c->sc->pat2), as<int64_t>(c->sc->pat2off), B->pat_len,
         as<uint64_t>(c->sc->txt2), as<int64_t>(c->sc->txt2off), B->txt_len};
    pf = as<int8_t>(c->sc->pflag);
    tf = as<int8_t>(c->sc->tflag);
  }
  HIP_TRY(aim::launch_pair_flags(n, L, B->pat_len, B->txt_len, pf, tf, as<int8_t>(c->sc->flags), s));
  return AIM_OK;
}

static aim_status align_batch(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen,
                              int32_t max_score, aim_results *R, void *stream) {
  g_err.clear();
  // validation needs no device and happens before anything is enqueued
  if (!B || !R) return fail(AIM_ERR_INVALID_ARG, "NULL batch or results");
  aim_status st = check_pen(alg, pen);
  if (st) return st;
  if ((st = check_batch(B))) return st;
  const int64_t n = B->n_pairs;
  if (n > 0 && (!R->score || !R->status)) return fail(AIM_ERR_INVALID_ARG, "NULL score/status");
  if (R->want_cigar && (!R->cigar_off || R->cigar_cap < 0 || (R->cigar_cap > 0 && !R->cigar)))
    return fail(AIM_ERR_INVALID_ARG, "want_cigar needs cigar_off and a cigar buffer of cigar_cap >= 0");
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (alg == AIM_WFA_ADAPTIVE && B->max_len > WFA_ADAPTIVE_MAX_LEN)
    return fail(AIM_ERR_UNSUPPORTED, "WFA-adaptive takes max_len <= %d", WFA_ADAPTIVE_MAX_LEN);
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;

  if (n == 0) {
    c->last_cnt = nullptr;
    c->last_n = 0;
    if (R->cigar_off) HIP_TRY(aim::launch_zero_offsets(0, R->cigar_off, s));
    return AIM_OK;
  }
  const int32_t L = B->max_len;
  const bool affine = alg != AIM_NW_LINEAR;
  aim::Scoring P{pen.mismatch, alg == AIM_NW_LINEAR ? 0 : pen.gap_open, pen.gap_extend, max_score,
                 R->want_cigar ? 1 : 0};

  // ---- common scratch ----
  const size_t tmp = aim::scan_tmp_elems(n) + (size_t)n + 2;
  if ((st = ensure(c, c->sc->scan_tmp, tmp * sizeof(int64_t)))) return st;
  if ((st = ensure(c, c->sc->counters, C_N * sizeof(int32_t) + 64))) return st;
  if ((st = ensure(c, c->sc->total, 64))) return st;
  if ((st = ensure(c, c->sc->nruns, (size_t)n * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->sc->spill, (size_t)n * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->sc->list2, (size_t)n * sizeof(int32_t)))) return st;
  if ((st = ensure(c, c->sc->list3, (size_t)n * sizeof(int32_t)))) return st;
  // runs held per pair before compaction: with a threshold S an optimal
  // alignment has at most S / min(x, o + e) non-match runs, so at most twice
  // that plus one runs in all; pairs with more are re-run in place
  int64_t run_bound = 2 * (int64_t)L + 1;
  const int32_t cmin = alg == AIM_GENASM ? 1 : std::min(pen.mismatch, (alg == AIM_NW_LINEAR ? 0 : pen.gap_open) + pen.gap_extend);
  if (max_score >= 0) run_bound = std::min<int64_t>(run_bound, 2 * (int64_t)(max_score / cmin) + 1);
  // a multiple of 4 words, so the compaction reads slots with 16-byte loads
  const int32_t slot_cap =
      (int32_t)((std::max<int64_t>(1, std::min<int64_t>(run_bound, SLOT_CAP)) + 3) & ~int64_t(3));
  if (R->want_cigar && (st = ensure(c, c->sc->slot, (size_t)n * slot_cap * sizeof(uint32_t)))) return st;
  int32_t *cnt = as<int32_t>(c->sc->counters);
  c->last_cnt = cnt;
  c->last_n = n;
  c->last_window = 0;
  for (int k = 0; k < 4; ++k) {
    c->last_class_window[k] = 0;
    c->last_class_bucket[k] = -1;
  }
  HIP_TRY(aim::launch_fill_i32(cnt, 0, C_N + 2, s));  // + the 64-bit adaptive drop count

  // ---- input encoding ----
  aim::Seqs S;
  if ((st = prep_inputs(c, B, s, S))) return st;

  // pool for runs beyond the per-pair slot (reset every call)
  // sized from the batch (a quarter of the worst-case run count per pair),
  // between 4 MiB and 1/64 of the scratch budget; exhaustion falls back to
  // the exact in-place re-run
  const int64_t pool_cap =
      R->want_cigar ? std::max<int64_t>(c->strict() ? 1 << 14 : 1 << 20,
                                        std::min<int64_t>(c->limit() / 64 / 4,
                                                          n * std::min<int64_t>(2 * (int64_t)L + 1, 8192) / 4))
                    : 1;
  if ((st = ensure(c, c->sc->pool, (size_t)pool_cap * 4))) return st;
  if ((st = ensure(c, c->sc->pooloff, (size_t)n * 8))) return st;
  HIP_TRY(aim::launch_fill_i32(as<int32_t>(c->sc->total) + 2, 0, 2, s));
  // a2: length buckets, longest first (LPT order for the persistent queues)
  const Tune tu = tune_for(c, alg, L);
  const bool do_sort = tu.sort >= 0 ? tu.sort != 0 : (alg != AIM_NW_LINEAR && alg != AIM_SWG_AFFINE) || L >= 512;
  const int32_t *order = nullptr;
  if (do_sort && c->opt.kernel != AIM_KERNEL_PLAIN) {
    if ((st = ensure(c, c->sc->order, (size_t)n * 4))) return st;
    if ((st = ensure(c, c->sc->hist, aim::LEN_BUCKETS * 4))) return st;
    Phase ph(c, s, "sort");
    HIP_TRY(aim::launch_length_sort(n, B->pat_len, B->txt_len, as<int32_t>(c->sc->hist),
                                    as<int32_t>(c->sc->order), s));
    order = as<int32_t>(c->sc->order);
  }
  aim::Outs O{R->score, R->status, as<int32_t>(c->sc->nruns), as<uint32_t>(c->sc->slot), slot_cap,
              as<int8_t>(c->sc->flags), R->cigar, R->cigar_off, R->cigar_cap, as<uint32_t>(c->sc->pool),
              pool_cap, (unsigned long long *)(as<int64_t>(c->sc->total) + 1), as<int64_t>(c->sc->pooloff)};
  const int64_t budget = c->limit() / 4;
  const bool plain = c->opt.kernel == AIM_KERNEL_PLAIN;

  // exact pre-alignment filter: with a threshold, pairs whose lower bound
  // already exceeds it are finished here and the aligners take the rest (in
  // `order`, counted on the device)
  const int32_t *order_count = nullptr;
  // (the band tiers reject short pairs about as fast as the filter would:
  // for NW/SWG it runs on reads over 256 bases, where a hopeless pair would
  // otherwise escalate to the wider tiers)
  // (GenASM rejects a hopeless pair in its first window)
  const bool filter_pays = alg != AIM_GENASM && (alg == AIM_WFA_AFFINE || alg == AIM_WFA_ADAPTIVE || L > 256);
  if (max_score >= 0 && !plain && filter_pays && !(c->opt.flags & AIM_FLAG_NO_PREFILTER)) {
    if ((st = ensure(c, c->sc->flist, (size_t)n * 4))) return st;
    Phase ph(c, s, "prefilter");
    HIP_TRY(aim::launch_prefilter(n, S, as<int8_t>(c->sc->flags), L, P.x, P.o, P.e, max_score, order, nullptr,
                                  nullptr, &O, as<int32_t>(c->sc->flist), cnt + C_FL, cnt + C_FR, s));
    order = as<int32_t>(c->sc->flist);
    order_count = cnt + C_FL;
  }

  auto run_full = [&](const aim::Work &Wk, int64_t max_items, hipStream_t s) -> aim_status {
    const int64_t sw = aim::full_slot_words(L);
    int64_t slots = std::min<int64_t>(max_items, (int64_t)c->cus * 8);
    slots = std::min<int64_t>(slots, std::max<int64_t>(1, budget / (sw * 4)));
    slots = std::max<int64_t>(slots, 1);
    aim_status e = ensure(c, c->sc->full, (size_t)(slots * sw * 4));
    if (e) return e;
    Phase ph(c, s, Wk.direct ? "full_rerun" : "full");
    HIP_TRY(aim::launch_full(affine, S, O, P, Wk, as<uint32_t>(c->sc->full), sw, L, (int32_t)slots, s));
    return AIM_OK;
  };

  if (alg == AIM_GENASM) {
    aim::Work WG{order, order_count, n, cnt + C_W1, nullptr, nullptr, 0};
    if ((st = run_genasm(c, S, O, P, n, WG, tu, s))) return st;
  } else if (alg == AIM_WFA_ADAPTIVE) {
    aim::Work WA{order, order_count, n, cnt + C_W1, nullptr, nullptr, 0};
    if ((st = run_wfa_adaptive(c, S, O, P, n, L, cnt, WA, tu, s))) return st;
  } else if (alg == AIM_WFA_AFFINE) {
    if ((st = run_wfa(c, S, O, P, n, L, plain, cnt, order, order_count, tu, s))) return st;
  } else if (plain) {
    aim::Work W1{nullptr, nullptr, n, cnt + C_T1, nullptr, nullptr, 0};
    if ((st = run_full(W1, n, s))) return st;
  } else {
    // tier 1: 32-diagonal band, one pair per lane (64 when tuned so)
    const int32_t rows_cap = L + 1;
    const int64_t chunks = (n + 63) / 64;
    const int32_t w0 = tu.band_w0 == 64 ? 64 : 32;
    // 32 diagonals in packed 16-bit arithmetic (two pairs per lane) when the
    // value bound allows, else 32-bit
    // (auto: not for small batches of short reads, which the one pair per
    // lane of the 32-bit band spreads over twice the wavefronts)
    const bool b16 = w0 == 32 && tu.band16 &&
                     !(tu.band16 == 3 && n < SMALL_BATCH_PAIRS && L <= SMALL_BATCH_LEN) &&
                     aim::band16_fits(L, P, affine);
    Buf &tbA = w0 == 32 ? c->sc->tb32 : c->sc->tb64;
    const int64_t swA = aim::band_tb_slot_words(b16 ? 64 : w0, affine, rows_cap);
    const int64_t chunksA = b16 ? (n + 127) / 128 : chunks;
    int64_t slots = std::min<int64_t>(chunksA, (int64_t)c->cus * std::max(1, tu.band_wpc));
    slots = std::max<int64_t>(1, std::min<int64_t>(slots, budget / (swA * 4)));
    // split fill / traceback when every chunk can keep its own bits
    // (the separate walk pays a second stream and two more launches, which
    // only large batches repay)
    const bool split = b16 && (tu.band16 == 2 || (tu.band16 == 3 && n >= SPLIT_MIN_PAIRS)) &&
                       R->want_cigar && chunksA * swA * 4 <= budget;
    if ((st = ensure(c, tbA, (size_t)((split ? chunksA : slots) * swA * 4)))) return st;
    aim::Work W1{order, order_count, n, cnt + C_T1, as<int32_t>(c->sc->list2), cnt + C_L2, 0};
    {
      Phase ph(c, s, b16 ? "band16" : (w0 == 32 ? "band32" : "band64"));
      if (b16)
        HIP_TRY(aim::launch_band16(affine, split, S, O, P, W1, as<uint32_t>(tbA), swA, rows_cap,
                                   (int32_t)slots, s));
      else
        HIP_TRY(aim::launch_band(w0, affine, S, O, P, W1, as<uint32_t>(tbA), swA, rows_cap,
                                 (int32_t)slots, s));
    }
    // Tier 1's traceback and tiers 2 and 3 work on disjoint pairs, so the
    // traceback runs on the second stream beside them.  Tiers 2 and 3 stay on
    // `s` right behind the fill: their few long-running wavefronts are then
    // dispatched first and hold their slots while the traceback takes the rest.
    hipStream_t s2 = c->aux;
    if (split) {
      HIP_TRY(hipEventRecord(c->ev_fork, s));
      HIP_TRY(hipStreamWaitEvent(s2, c->ev_fork, 0));
    }
    int32_t *full_list = as<int32_t>(c->sc->list2);
    int32_t *full_count = cnt + C_L2;
    if (w0 == 32) {
      // tier 2: 64-diagonal band for the pairs tier 1 could not decide, one
      // pair per 32 lanes along the anti-diagonal, then a walk per lane
      const int64_t cw = aim::diag_chunk_words(affine, L);
      const int64_t need = (n + 1) / 2;
      int64_t cap2 = std::min<int64_t>(need, std::max<int64_t>(1024, ((int64_t)512 << 20) / (cw * 4)));
      cap2 = std::max<int64_t>(1, std::min<int64_t>(cap2, budget / (cw * 4)));
      if (!R->want_cigar) cap2 = 1;
      if ((st = ensure(c, c->sc->tb64, (size_t)(cap2 * cw * 4)))) return st;
      aim::Work W2{as<int32_t>(c->sc->list2), cnt + C_L2, n, cnt + C_T2, as<int32_t>(c->sc->list3),
                   cnt + C_L3, 0};
      {
        Phase ph2(c, s, "diag");
        HIP_TRY(aim::launch_diag(affine, S, O, P, W2, as<uint32_t>(c->sc->tb64), cw, cap2,
                                 (int32_t)std::min<int64_t>(need, (int64_t)c->cus * 16), s));
      }
      if (R->want_cigar) {
        aim::Work W2t{as<int32_t>(c->sc->list2), cnt + C_L2, n, cnt + C_DTB, nullptr, nullptr, 0};
        Phase ph2(c, s, "diag_tb");
        HIP_TRY(aim::launch_diag_tb(affine, S, O, W2t, as<uint32_t>(c->sc->tb64), cw,
                                    (int32_t)std::min<int64_t>((n + 15) / 16, (int64_t)c->cus * 8), s));
      }
      full_list = as<int32_t>(c->sc->list3);
      full_count = cnt + C_L3;
    }
    if (split) {
      aim::Work WT{order, order_count, n, cnt + C_TB, nullptr, nullptr, 0};
      Phase ph(c, s2, "band16_tb");
      // six of the eight workgroups a CU could hold: the persistent traceback
      // must leave slots for the second tier's kernels beside it
      HIP_TRY(aim::launch_band16_tb(affine, S, O, WT, as<uint32_t>(tbA), swA,
                                    (int32_t)std::min<int64_t>(chunksA, (int64_t)c->cus * 6), s2));
    }
    // tier 3, the pairs no band certified: for reads over 256 bases the
    // wavefront algorithm, which reaches the same optimum and (with the same
    // tie order) the same CIGAR in time growing with the score rather than
    // with m x n; the full matrix for short reads (one launch instead of the
    // wavefront passes' six, which small batches notice) and for penalties
    // beyond the wavefront ring's reach
    if (L > 256 && P.x <= WFA_MAX_STEP && P.o + P.e <= WFA_MAX_STEP) {
      if ((st = run_wfa(c, S, O, P, n, L, false, cnt, full_list, full_count,
                        tune_for(c, AIM_WFA_AFFINE, L), s)))
        return st;
    } else {
      aim::Work W3{full_list, full_count, n, cnt + C_T3, nullptr, nullptr, 0};
      if ((st = run_full(W3, n, s))) return st;
    }
    if (split) {
      HIP_TRY(hipEventRecord(c->ev_join, s2));
      HIP_TRY(hipStreamWaitEvent(s, c->ev_join, 0));
    }
  }

  if (!R->want_cigar) {
    if (R->cigar_off) HIP_TRY(aim::launch_zero_offsets(n, R->cigar_off, s));
    return AIM_OK;
  }
  {
  Phase ph(c, s, "compact");
  HIP_TRY(aim::launch_compact(n, O, R->cigar_off, R->cigar, R->cigar_cap, as<int64_t>(c->sc->scan_tmp),
                              as<int64_t>(c->sc->total), as<int32_t>(c->sc->spill), cnt + C_SPILL,
                              R->status, s));
  }
  // pairs whose runs exceeded the slot: recompute and write in place
  aim::Work WS{as<int32_t>(c->sc->spill), cnt + C_SPILL, n, cnt + C_SPILL_W, nullptr, nullptr, 1};
  if (alg == AIM_GENASM) {
    if ((st = run_genasm(c, S, O, P, n, WS, tu, s))) return st;
  } else if (alg == AIM_WFA_ADAPTIVE) {
    if ((st = run_wfa_adaptive(c, S, O, P, n, L, cnt, WS, tu, s))) return st;
  } else if (alg == AIM_WFA_AFFINE) {
    const aim::Scoring PW = wfa_scoring(P);
    aim::WfaPlan pl = aim::wfa_plan(L, PW, c->limit(), c->cus, plain, tu.wfa_ring_kb,
                                    tu.wfa_trace_kb, tu.wfa_long_threads, c->strict());
    aim::WfaLaunch WL{};
    WL.R = pl.R;
    WL.seq_words = pl.seq_words;
    WL.full_in_lds = 0;
    WL.slot_words = pl.need_cap[3];
    WL.need = as<int64_t>(c->sc->wneed);
    // the memory-bounded pass re-runs any pair, whatever its full store
    aim::WfaLong LG{};
    int32_t long_slots = 0;
    if (!plain && (st = wfa_long_plan(c, L, PW, pl, L <= aim::WFA16_MAX_LEN, LG, long_slots))) return st;
    if (long_slots > 0) {
      LG.failed = cnt + C_LF;
      Phase ph(c, s, "wfa_rerun");
      HIP_TRY(aim::launch_wfa_long(S, O, PW, WS, LG, long_slots, aim::WGMAX_THREADS, L <= aim::WFA16_MAX_LEN, s));
      return AIM_OK;
    }
    if ((st = ensure(c, c->sc->warena3, (size_t)pl.pool_words[3] * 4))) return st;
    const int32_t rslots = (int32_t)std::max<int64_t>(1, pl.pool_words[3] / pl.need_cap[3]);
    Phase ph(c, s, "wfa_rerun");
    HIP_TRY(aim::launch_wfa_trace(S, O, PW, WS, WL, as<int32_t>(c->sc->warena3), rslots,
                                  pl.threads[3], L <= aim::WFA16_MAX_LEN && !plain, s));
  } else {
    if ((st = run_full(WS, n, s))) return st;
  }
  return AIM_OK;
}

aim_status aim_align_batch(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen,
                           int32_t max_score, aim_results *R, void *stream) {
  if (!c || c->capturing) return align_batch(c, B, alg, pen, max_score, R, stream);
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  // the previous call's work (on another stream) before this call's, so that
  // scratch freed or reused in stream order on `s` is no longer in use
  if (c->has_done && c->done_stream != s) HIP_TRY(hipStreamWaitEvent(s, c->ev_done, 0));
  c->astream = s;
  const aim_status st = align_batch(c, B, alg, pen, max_score, R, stream);
  c->astream = nullptr;
  HIP_TRY(hipEventRecord(c->ev_done, s));
  c->has_done = true;
  c->done_stream = s;
  return st;
}

aim_status aim_last_call_stats(aim_context *c, aim_call_stats *out) {
  g_err.clear();
  if (!c || !out) return fail(AIM_ERR_INVALID_ARG, "NULL argument");
  memset(out, 0, sizeof *out);
  if (!c->has_done || !c->last_cnt) return AIM_OK;
  DeviceGuard g(c->device);
  HIP_TRY(hipEventSynchronize(c->ev_done));
  int32_t v[C_N];
  HIP_TRY(hipMemcpy(v, c->last_cnt, sizeof v, hipMemcpyDeviceToHost));
  out->n_pairs = c->last_n;
  out->band_escalated = v[C_L2];
  out->band_escalated2 = v[C_L3];
  out->wfa_wide = v[C_RL];
  out->wfa_walk_failed = v[C_WF];
  out->wfa_walk_skipped = v[C_WS];
  for (int k = 0; k < 4; ++k) out->full_store[k] = v[C_N0 + k];
  out->cigar_reruns = v[C_SPILL];
  out->wfa_window = c->last_window;
  for (int k = 0; k < 4; ++k) {
    out->wfa_class_pairs[k] = v[C_CL + k];
    out->wfa_class_window[k] = c->last_class_window[k];
  }
  out->prefilter_rejected = v[C_FR];
  unsigned long long dropped = 0;
  HIP_TRY(hipMemcpy(&dropped, c->last_cnt + C_N, sizeof dropped, hipMemcpyDeviceToHost));
  out->wfa_adaptive_dropped = (int64_t)dropped;
  out->wfa_long_pairs = v[C_LL];
  out->wfa_long_failed = v[C_LF];
  return AIM_OK;
}

aim_status aim_align_batch_static(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen,
                                  int32_t max_score, aim_results *R, void *stream) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (c->capturing) return fail(AIM_ERR_INVALID_ARG, "aim_align_batch_static inside aim_graph_capture");
  DeviceGuard g(c->device);
  void *base = nullptr;
  const hipError_t e = aim::static_scratch_address(c->device, &base);
  if (e != hipSuccess) return fail(AIM_ERR_HIP, "static scratch array: %s", hipGetErrorString(e));
  hipStream_t s = (hipStream_t)stream;
  if (c->has_done && c->done_stream != s) HIP_TRY(hipStreamWaitEvent(s, c->ev_done, 0));
  // this call's buffers, carved from the array from its start
  Scratch carved;
  c->sc = &carved;
  c->arena = static_cast<uint8_t *>(base);
  c->arena_cap = aim::STATIC_SCRATCH_BYTES;
  c->arena_top = 0;
  c->astream = s;
  const aim_status st = align_batch(c, B, alg, pen, max_score, R, stream);
  c->astream = nullptr;
  c->arena = nullptr;
  c->arena_cap = c->arena_top = 0;
  c->sc = &c->own;
  HIP_TRY(hipEventRecord(c->ev_done, s));
  c->has_done = true;
  c->done_stream = s;
  return st;
}

aim_status aim_wfa_adaptive_params(aim_context *c, int32_t min_len, int32_t max_dist) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (min_len < 1 || max_dist < 0) return fail(AIM_ERR_INVALID_ARG, "need min_len >= 1 and max_dist >= 0");
  c->ad_min = min_len;
  c->ad_max = max_dist;
  return AIM_OK;
}

aim_status aim_scratch_usage(aim_context *c, int64_t *current, int64_t *peak) {
  g_err.clear();
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (current) *current = c->dev_bytes;
  if (peak) *peak = c->dev_peak;
  return AIM_OK;
}

aim_status aim_prefilter(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen, int32_t max_score,
                         int32_t *lower, int8_t *pass, void *stream) {
  g_err.clear();
  aim_status st = check_pen(alg, pen);
  if (st) return st;
  if ((st = check_batch(B))) return st;
  const int64_t n = B->n_pairs;
  if (n > 0 && (!lower || !pass)) return fail(AIM_ERR_INVALID_ARG, "NULL lower or pass");
  if (!c) return fail(AIM_ERR_INVALID_ARG, "ctx is NULL");
  if (n == 0) return AIM_OK;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  // ordered after the context's previous call like aim_align_batch
  if (c->has_done && c->done_stream != s) HIP_TRY(hipStreamWaitEvent(s, c->ev_done, 0));
  c->astream = s;
  aim::Seqs S;
  st = prep_inputs(c, B, s, S);
  if (!st) {
    // GenASM counts edits: its result is at least the unit-cost bound
    const bool unit = alg == AIM_GENASM;
    const hipError_t e = aim::launch_prefilter(n, S, as<int8_t>(c->sc->flags), B->max_len, unit ? 1 : pen.mismatch,
                                               (alg == AIM_NW_LINEAR || unit) ? 0 : pen.gap_open,
                                               unit ? 1 : pen.gap_extend, max_score,
                                               nullptr, lower, pass, nullptr, nullptr, nullptr, nullptr, s);
    if (e != hipSuccess) st = fail(AIM_ERR_HIP, "prefilter launch: %s", hipGetErrorString(e));
  }
  c->astream = nullptr;
  HIP_TRY(hipEventRecord(c->ev_done, s));
  c->has_done = true;
  c->done_stream = s;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
namespace {
const int32_t TUNE_FIELDS = 13;
void tune_to(const Tune &t, int32_t *v) {
  v[0] = t.band_w0; v[1] = t.band_wpc; v[2] = t.sort;
  v[3] = t.wfa_ring_kb; v[4] = t.wfa_trace_kb; v[5] = t.wfa_long_threads; v[6] = t.band16;
  v[7] = t.wfa_classes;
  for (int k = 0; k < 3; ++k) v[8 + k] = t.wfa_cls_threads[k];
  v[11] = t.wfa_cls_global;
  v[12] = t.wfa_c16;
}
Tune tune_from(const int32_t *v) {
  Tune t;
  t.band_w0 = v[0]; t.band_wpc = v[1]; t.sort = v[2];
  t.wfa_ring_kb = v[3]; t.wfa_trace_kb = v[4]; t.wfa_long_threads = v[5]; t.band16 = v[6];
  t.wfa_classes = v[7];
  for (int k = 0; k < 3; ++k) t.wfa_cls_threads[k] = v[8 + k];
  t.wfa_cls_global = v[11];
  t.wfa_c16 = v[12];
  return t;
}
bool tune_valid(const Tune &t) {
  return (t.band_w0 == 32 || t.band_w0 == 64) && t.band_wpc >= 1 && t.band_wpc <= 64 &&
         t.sort >= -1 && t.sort <= 1 && t.wfa_ring_kb >= 8 && t.wfa_ring_kb <= 60 &&
         t.wfa_trace_kb >= 8 && t.wfa_trace_kb <= 60 &&
         (t.wfa_long_threads == 64 || t.wfa_long_threads == 128 || t.wfa_long_threads == 256) &&
         (t.band16 >= 0 && t.band16 <= 3) && (t.wfa_classes == 0 || t.wfa_classes == 1) && t.wfa_cls_global >= 0 && t.wfa_cls_global <= 7 &&
         t.wfa_c16 >= 0 && t.wfa_c16 <= 4 &&
         [&] {
           for (int k = 0; k < 3; ++k) {
             const int32_t th = t.wfa_cls_threads[k];
             if (th != 64 && th != 128 && th != 256 && th != 512) return false;
           }
           return true;
         }();
}
std::string tune_key() {
  int v = 0;
  (void)hipRuntimeGetVersion(&v);
  return std::to_string(v);
}
}  // namespace

extern "C" {

aim_status aim_autotune(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen,
                        int32_t max_score, aim_results *R, void *stream, int32_t reps,
                        int32_t *best_params, double *best_ms) {
  g_err.clear();
  if (!c || !B || !R) return fail(AIM_ERR_INVALID_ARG, "NULL context, batch or results");
  if (reps < 1 || reps > 100) return fail(AIM_ERR_INVALID_ARG, "reps must be in [1, 100]");
  std::vector<Tune> cand;
  if (alg == AIM_WFA_AFFINE || alg == AIM_WFA_ADAPTIVE) {
    // the batch-level choices: the order of the pairs, the one-wavefront
    // window (64, 128 or 256 diagonals) and the workgroup of the pairs no
    // window class takes; the classes' own configurations follow
    for (int so : {0, 1})
      for (int c16 : {1, 2, 4})
        for (int th : {128, 256}) {
          if (alg == AIM_WFA_ADAPTIVE && (c16 != 1 || th != 128)) continue;
          Tune t;
          t.sort = so;
          t.wfa_c16 = c16;
          t.wfa_long_threads = th;
          if (alg == AIM_WFA_ADAPTIVE)
            for (int w : {64, 128}) {
              t.wfa_cls_threads[0] = w;
              cand.push_back(t);
            }
          else
            cand.push_back(t);
        }
  } else if (alg == AIM_GENASM) {
    // wavefronts per CU (the slots scale with them) and the order
    for (int wpc : {4, 8, 12, 16})
      for (int so : {0, 1}) {
        Tune t;
        t.band_wpc = wpc;
        t.sort = so;
        cand.push_back(t);
      }
  } else {
    for (int w0 : {32, 64})
      for (int wpc : {8, 16, 32})
        for (int so : {0, 1})
          for (int b16 : {0, 1, 2}) {
            if (w0 == 64 && b16) continue;
            Tune t;
            t.band_w0 = w0;
            t.band_wpc = wpc;
            t.sort = so;
            t.band16 = b16;
            cand.push_back(t);
          }
  }
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = 1e300;
  size_t bi = 0;
  aim_status st = AIM_OK;
  for (size_t k = 0; k < cand.size() && st == AIM_OK; ++k) {
    c->force = &cand[k];
    st = aim_align_batch(c, B, alg, pen, max_score, R, stream);  // warm-up, sizes scratch
    std::vector<double> ms;
    for (int r = 0; r < reps && st == AIM_OK; ++r) {
      (void)hipEventRecord(e0, s);
      st = aim_align_batch(c, B, alg, pen, max_score, R, stream);
      (void)hipEventRecord(e1, s);
      float t = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        st = fail(AIM_ERR_HIP, "timing the candidate failed");
        break;
      }
      ms.push_back(t);
    }
    if (st == AIM_OK) {
      std::sort(ms.begin(), ms.end());
      const double med = ms[ms.size() / 2];
      if (med < best) { best = med; bi = k; }
    }
  }
  // WFA: then each window class of this batch in turn, with the batch tune
  // chosen: workgroup size {64, 128, 256} x ring in a global slot or LDS,
  // kept per class length bucket
  if (st == AIM_OK && alg == AIM_WFA_AFFINE) {
    c->force = &cand[bi];
    st = aim_align_batch(c, B, alg, pen, max_score, R, stream);
    int32_t buckets[4];
    for (int k = 0; k < 4; ++k) buckets[k] = c->last_class_bucket[k];
    for (int k = 0; k < 4 && st == AIM_OK; ++k) {
      if (buckets[k] < 0) continue;
      const std::pair<int32_t, int32_t> key{AIM_WFA_AFFINE, buckets[k]};
      const auto had = c->class_tunes.find(key);
      const bool had_entry = had != c->class_tunes.end();
      const ClassTune prev = had_entry ? had->second : ClassTune{};
      ClassTune bestc{};
      double bestk = 1e300;
      for (int th : {64, 128, 256})
        for (int gl : {1, 0}) {
          c->class_tunes[key] = ClassTune{th, gl};
          st = aim_align_batch(c, B, alg, pen, max_score, R, stream);
          std::vector<double> ms;
          for (int r = 0; r < reps && st == AIM_OK; ++r) {
            (void)hipEventRecord(e0, s);
            st = aim_align_batch(c, B, alg, pen, max_score, R, stream);
            (void)hipEventRecord(e1, s);
            float t = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
              st = fail(AIM_ERR_HIP, "timing the candidate failed");
              break;
            }
            ms.push_back(t);
          }
          if (st != AIM_OK) break;
          std::sort(ms.begin(), ms.end());
          if (ms[ms.size() / 2] < bestk) {
            bestk = ms[ms.size() / 2];
            bestc = ClassTune{th, gl};
          }
        }
      if (st == AIM_OK) {
        c->class_tunes[key] = bestc;
        best = std::min(best, bestk);
      } else if (had_entry) {
        c->class_tunes[key] = prev;
      } else {
        c->class_tunes.erase(key);
      }
    }
  }
  c->force = nullptr;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AIM_OK) return st;
  c->tunes[{alg, len_bucket_host(B->max_len)}] = cand[bi];
  if (best_params) tune_to(cand[bi], best_params);
  if (best_ms) *best_ms = best;
  // leave the outputs of the chosen configuration in `out`
  return aim_align_batch(c, B, alg, pen, max_score, R, stream);
}

aim_status aim_tune_get(aim_context *c, int32_t alg, int32_t max_len, int32_t *params) {
  g_err.clear();
  if (!c || !params) return fail(AIM_ERR_INVALID_ARG, "NULL argument");
  tune_to(tune_for(c, alg, max_len), params);
  return AIM_OK;
}

aim_status aim_tune_set(aim_context *c, int32_t alg, int32_t max_len, const int32_t *params) {
  g_err.clear();
  if (!c || !params) return fail(AIM_ERR_INVALID_ARG, "NULL argument");
  Tune t = tune_from(params);
  if (!tune_valid(t)) return fail(AIM_ERR_INVALID_ARG, "tune parameters out of range");
  c->tunes[{alg, len_bucket_host(max_len)}] = t;
  return AIM_OK;
}

aim_status aim_tune_entries(aim_context *c, int32_t cap, int32_t *kind, int32_t *alg, int32_t *bucket,
                            int32_t *count) {
  g_err.clear();
  if (!c || !count || cap < 0 || (cap > 0 && (!kind || !alg || !bucket)))
    return fail(AIM_ERR_INVALID_ARG, "NULL argument or negative cap");
  int32_t k = 0;
  for (auto &kv : c->tunes) {
    if (k < cap) { kind[k] = 0; alg[k] = kv.first.first; bucket[k] = kv.first.second; }
    ++k;
  }
  for (auto &kv : c->class_tunes) {
    if (k < cap) { kind[k] = 1; alg[k] = kv.first.first; bucket[k] = kv.first.second; }
    ++k;
  }
  *count = k;
  return AIM_OK;
}

aim_status aim_tune_save(aim_context *c, const char *path) {
  g_err.clear();
  if (!c || !path) return fail(AIM_ERR_INVALID_ARG, "NULL argument");
  std::ofstream f(path);
  if (!f) return fail(AIM_ERR_INVALID_ARG, "cannot write %s", path);
  f << "aim-tune 3 " << c->arch << " " << tune_key() << "\n";
  for (auto &kv : c->tunes) {
    int32_t v[TUNE_FIELDS];
    tune_to(kv.second, v);
    f << "T " << kv.first.first << " " << kv.first.second;
    for (int k = 0; k < TUNE_FIELDS; ++k) f << " " << v[k];
    f << "\n";
  }
  for (auto &kv : c->class_tunes)
    f << "C " << kv.first.first << " " << kv.first.second << " " << kv.second.threads << " " << kv.second.global
      << "\n";
  return f ? AIM_OK : fail(AIM_ERR_INVALID_ARG, "write failed: %s", path);
}

aim_status aim_tune_load(aim_context *c, const char *path) {
  g_err.clear();
  if (!c || !path) return fail(AIM_ERR_INVALID_ARG, "NULL argument");
  std::ifstream f(path);
  if (!f) return fail(AIM_ERR_NOT_FOUND, "cannot read %s", path);
  std::string magic, ver, arch, key;
  f >> magic >> ver >> arch >> key;
  if (magic != "aim-tune" || ver != "3") return fail(AIM_ERR_INVALID_ARG, "not a tune file: %s", path);
  if (arch != c->arch || key != tune_key())
    return fail(AIM_ERR_NOT_FOUND, "tune file is for %s / runtime %s", arch.c_str(), key.c_str());
  std::map<std::pair<int32_t, int32_t>, Tune> loaded;
  std::map<std::pair<int32_t, int32_t>, ClassTune> loaded_cls;
  std::string kind;
  int32_t alg, bucket, v[TUNE_FIELDS];
  while (f >> kind >> alg >> bucket) {
    if (kind == "T") {
      for (int k = 0; k < TUNE_FIELDS; ++k) f >> v[k];
      if (!f) return fail(AIM_ERR_INVALID_ARG, "truncated tune file");
      Tune t = tune_from(v);
      if (!tune_valid(t)) return fail(AIM_ERR_INVALID_ARG, "bad tune entry in %s", path);
      loaded[{alg, bucket}] = t;
    } else if (kind == "C") {
      ClassTune ct;
      f >> ct.threads >> ct.global;
      if (!f) return fail(AIM_ERR_INVALID_ARG, "truncated tune file");
      if ((ct.threads != 0 && ct.threads != 64 && ct.threads != 128 && ct.threads != 256 && ct.threads != 512) ||
          ct.global < -1 || ct.global > 1)
        return fail(AIM_ERR_INVALID_ARG, "bad class entry in %s", path);
      loaded_cls[{alg, bucket}] = ct;
    } else {
      return fail(AIM_ERR_INVALID_ARG, "bad tune line in %s", path);
    }
  }
  for (auto &kv : loaded) c->tunes[kv.first] = kv.second;
  for (auto &kv : loaded_cls) c->class_tunes[kv.first] = kv.second;
  return AIM_OK;
}

// ---------------------------------------------------------------- graphs
aim_status aim_graph_capture(aim_context *c, const aim_batch *B, int32_t alg, aim_penalties pen,
                             int32_t max_score, aim_results *R, void *stream, aim_graph **out) {
  g_err.clear();
  if (!c || !out) return fail(AIM_ERR_INVALID_ARG, "NULL context or graph handle");
  if (!stream) return fail(AIM_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  *out = nullptr;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  aim_status st = aim_align_batch(c, B, alg, pen, max_score, R, stream);  // sizes scratch
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t gen = c->generation;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  st = aim_align_batch(c, B, alg, pen, max_score, R, stream);
  c->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(s, &graph);
  if (st != AIM_OK || ee != hipSuccess || c->generation != gen) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st != AIM_OK) return st;
    if (ee != hipSuccess) return fail(AIM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    return fail(AIM_ERR_HIP, "scratch changed during capture");
  }
  hipGraphExec_t exec = nullptr;
  hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(AIM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  auto *gr = new aim_graph();
  gr->c = c;
  gr->device = c->device;
  c->graphs.insert(gr);
  gr->graph = graph;
  gr->exec = exec;
  gr->generation = gen;
  *out = gr;
  return AIM_OK;
}

aim_status aim_graph_launch(aim_graph *gr, void *stream) {
  g_err.clear();
  if (!gr) return fail(AIM_ERR_INVALID_ARG, "NULL graph");
  if (!gr->c) return fail(AIM_ERR_INVALID_ARG, "the graph's context was destroyed");
  if (gr->c->generation != gr->generation)
    return fail(AIM_ERR_INVALID_ARG, "the context's scratch was reallocated since capture; capture again");
  aim_context *c = gr->c;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  // the same ordering as aim_align_batch: a replay shares the context's
  // scratch with its eager calls, so it waits for the last of them (or of
  // the replays) issued on another stream, and the next call waits for it
  if (c->has_done && c->done_stream != s) HIP_TRY(hipStreamWaitEvent(s, c->ev_done, 0));
  HIP_TRY(hipGraphLaunch(gr->exec, s));
  HIP_TRY(hipEventRecord(c->ev_done, s));
  c->has_done = true;
  c->done_stream = s;
  return AIM_OK;
}

void aim_graph_destroy(aim_graph *gr) {
  if (!gr) return;
  if (gr->c) gr->c->graphs.erase(gr);
  DeviceGuard g(gr->device);
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
}

}  // extern "C"
