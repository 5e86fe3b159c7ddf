// Internal declarations shared by the HIP translation units of libaim.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aim {

// "Infinity" for int32 DP cells.  Finite costs stay far below it for the
// supported lengths (<= 2^20) and penalties (<= 65535), and it plus the
// largest per-row growth stays below 2^31.
constexpr int32_t DP_INF = 1 << 28;

constexpr int OP_EQ = 0, OP_X = 1, OP_I = 2, OP_D = 3;
constexpr int8_t ST_ALIGNED = 0, ST_REJECTED = 1, ST_OVERFLOW = 2, ST_INVALID = 3;

// Pairs as 2-bit packed CSR (base t of a sequence at bits 2*(t%32) of word
// t/32, sequences word aligned).
struct Seqs {
  const uint64_t *pat;
  const int64_t *pat_off;
  const int32_t *pat_len;
  const uint64_t *txt;
  const int64_t *txt_off;
  const int32_t *txt_len;
};

// Per-pair results plus the run slots the align kernels write before the
// CIGAR compaction (runs stored last-op-first, up to slot_cap per pair; the
// true run count is always recorded in nruns).
struct Outs {
  int32_t *score;
  int8_t *status;
  int32_t *nruns;
  uint32_t *slot;      // [n_pairs * slot_cap]
  int32_t slot_cap;
  const int8_t *flags; // per pair: nonzero = invalid input
  // Direct mode (re-run of pairs whose runs exceeded slot_cap): runs are
  // written last-op-first ending at cigar[cigar_off[p] + nruns[p] - 1].
  uint32_t *cigar;
  const int64_t *cigar_off;
  int64_t cigar_cap;
  // Runs beyond slot_cap go to a shared pool: the first overflowing run of a
  // pair reserves `bound` words with one atomic add; pool_off[p] is that
  // offset (-1: none, -2: pool exhausted, the pair is re-run in place).
  uint32_t *pool;
  int64_t pool_cap;
  unsigned long long *pool_top;
  int64_t *pool_off;
};

// Appends runs of one pair (last op first) to its slot, then to the pool.
struct RunSink {
  uint32_t *slot;
  int32_t cap;
  uint32_t *pool;
  int64_t pool_cap;
  unsigned long long *pool_top;
  int64_t *pool_off;  // &Outs::pool_off[p]
  int64_t pbase;      // reserved pool offset, -1 none, -2 failed
  __device__ void begin(const Outs &O, int64_t p) {
    slot = O.slot + p * (int64_t)O.slot_cap;
    cap = O.slot_cap;
    pool = O.pool;
    pool_cap = O.pool_cap;
    pool_top = O.pool_top;
    pool_off = O.pool_off + p;
    pbase = -1;
  }
  // nr: index of this run; more: upper bound on the runs still to come
  // (this one included) when the pool is first needed.
  __device__ void put(int32_t nr, uint32_t run, int64_t more) {
    if (nr < cap) {
      slot[nr] = run;
      return;
    }
    if (pbase == -1) {
      const unsigned long long need = (unsigned long long)(more > 0 ? more : 1);
      const unsigned long long at = atomicAdd(pool_top, need);
      pbase = (at + need <= (unsigned long long)pool_cap) ? (int64_t)at : -2;
      *pool_off = pbase;
    }
    if (pbase >= 0) pool[pbase + (nr - cap)] = run;
  }
  __device__ void finish() {
    if (pbase == -1) *pool_off = -1;
  }
};

struct Scoring {
  int32_t x, o, e;     // linear NW: o == 0 and e == gap cost
  int32_t max_score;   // < 0: none
  int32_t want_cigar;
  // The wavefront kernels run on penalties divided by their common divisor
  // (every alignment cost is a multiple of it, so the optimum and the tie
  // order are the same and no score step is empty); a score s of theirs is
  // unit * s in O.score.  1 everywhere else.
  int32_t unit = 1;
};

// A list of pair indices to work on, consumed through an atomic counter;
// `count` (device) overrides `n` when non-null.
struct Work {
  const int32_t *idx;   // nullptr: identity
  const int32_t *count; // nullptr: n
  int64_t n;
  int32_t *counter;     // work counter, zeroed before the launch
  int32_t *next_idx;    // escalation list (may be nullptr)
  int32_t *next_count;
  int32_t direct;       // 1: write runs straight into Outs::cigar
};

// ---- host-side launchers (each enqueues on `stream`) ----------------------
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_pair_flags(int64_t n, int32_t max_len, const int32_t *pl, const int32_t *tl,
                             const int8_t *pf, const int8_t *tf, int8_t *flags, hipStream_t s);
hipError_t launch_pack(int64_t n, int32_t enc, const uint8_t *seq, const int64_t *off,
                       const int32_t *len, int32_t max_len, uint64_t *words, int64_t words_cap,
                       int64_t *out_off, int8_t *flags, int64_t *scan_tmp, hipStream_t s);
// The same packing with sequence s at word s * ceil(max_len / 32) (one
// launch, no scan); words_cap must cover n such strides.
hipError_t launch_pack_strided(int64_t n, int32_t enc, const uint8_t *seq, const int64_t *off,
                               const int32_t *len, int32_t max_len, uint64_t *words,
                               int64_t words_cap, int64_t *out_off, int8_t *flags, hipStream_t s);
size_t scan_tmp_elems(int64_t n);
// exclusive scan of int32 counts into int64 out[n+1]
hipError_t launch_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *tmp, hipStream_t s);

// Banded DP (one pair per lane).  W in {32, 64}.
hipError_t launch_band(int W, bool affine, const Seqs &S, const Outs &O, const Scoring &P,
                       const Work &Wk, uint32_t *tb, int64_t tb_slot_words, int32_t rows_cap,
                       int32_t nslots, hipStream_t s);
int64_t band_tb_slot_words(int W, bool affine, int32_t rows_cap);

// Banded DP with packed 16-bit cells, two pairs per lane, 32 diagonals
// (traceback slot layout of the 64-diagonal kernel).  band16_fits: whether
// pairs of length <= max_len provably stay within 16 bits.
bool band16_fits(int32_t max_len, const Scoring &P, bool affine);
// split: traceback bits kept per chunk of 128 pairs (tb_slot_words per
// chunk) and walked afterwards by launch_band16_tb; else per workgroup slot,
// walked in the fill kernel.
hipError_t launch_band16(bool affine, bool split, const Seqs &S, const Outs &O, const Scoring &P,
                         const Work &Wk, uint32_t *tb, int64_t tb_slot_words, int32_t rows_cap,
                         int32_t nslots, hipStream_t s);
// One workgroup of 128 threads per chunk at a time (persistent, nslots).
hipError_t launch_band16_tb(bool affine, const Seqs &S, const Outs &O, const Work &Wk, const uint32_t *tb,
                            int64_t tb_chunk_words, int32_t nslots, hipStream_t s);

// Banded DP with 64 diagonals, one pair per 32 lanes along the anti-diagonal
// (two pairs per wavefront).  Traceback bits of chunk c (the two pairs of
// list positions 2c, 2c+1) in chunk_words words at tb + c * chunk_words, for
// c < chunks_cap; pairs of later chunks are escalated when CIGARs are wanted.
// Accepted pairs get nruns = -2 until launch_diag_tb walks them (the first
// tier's split walk, which may run at the same time, waits for -1).
int64_t diag_chunk_words(bool affine, int32_t max_len);
hipError_t launch_diag(bool affine, const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                       uint32_t *tb, int64_t chunk_words, int64_t chunks_cap, int32_t nslots,
                       hipStream_t s);
// Walk of the pairs of the same list (same Work idx / count) with nruns == -2,
// diag_tb_pairs_per_wave() list positions per wavefront.
int32_t diag_tb_pairs_per_wave();
hipError_t launch_diag_tb(bool affine, const Seqs &S, const Outs &O, const Work &Wk, const uint32_t *tb,
                          int64_t chunk_words, int32_t nslots, hipStream_t s);

// Full-matrix DP, one pair per workgroup.
hipError_t launch_full(bool affine, const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                       uint32_t *scratch, int64_t slot_words, int32_t max_len, int32_t nslots,
                       hipStream_t s);
int64_t full_slot_words(int32_t max_len);

// Where a pair whose wavefronts leave a pass's window goes next: classes
// 1..nclass, each with a wider window (half-width half[c] diagonals around
// diagonal 0; the last class, the HBM-ring pass, has no bound); the pair
// joins the first later class whose window holds its predicted extent.
constexpr int WFA_MAX_CLASSES = 6;
struct WfaRoute {
  int32_t nclass;
  int32_t half[WFA_MAX_CLASSES];
  int32_t *list[WFA_MAX_CLASSES];
  int32_t *count[WFA_MAX_CLASSES];
  int32_t *pred;  // per pair: the extent predicted when it left its last window
};

// Wavefront algorithm, one pair per 64-lane wavefront, two passes.
struct WfaLaunch {
  int32_t R;            // ring slots (score passes): max(x, o+e) + 1
  int32_t wcap;         // ring width capacity of this launch (score passes)
  int32_t seq_words;    // words of LDS per staged sequence (0: read from HBM)
  int32_t full_in_lds;  // fallback pass: arena in LDS
  int64_t slot_words;   // HBM slot per workgroup (score ring / fallback arena), or LDS arena words
  int32_t *ring_list;   // score pass: pairs whose width passed wcap
  int32_t *ring_count;
  int32_t *need_list[4];  // score -> fallback pass: accepted pairs by full-store class
  int32_t *need_count[4];
  int64_t need_cap[4];    // class capacities in words
  int32_t *need_max[4];   // score -> fallback pass: largest full store per class (words)
  int64_t *need;          // per pair: words of the full store
  int32_t store16;        // score passes count the full store in 16-bit entries
  // fallback pass, HBM arena: when set, each workgroup's slot is the class's largest
  // full store (rounded up), and only pool_words / slot workgroups take pairs
  const int32_t *slot_need_max;
  int64_t pool_words;
  // one-wavefront score pass with a CIGAR wanted: per workgroup, room for the
  // origin codes of bits_steps scores (0: none); pairs that need more go to
  // the fallback pass
  uint8_t *bits;
  int32_t bits_steps;
  // HBM-ring score pass with a CIGAR wanted: per workgroup, a table of
  // walk_steps scores, walk_codes bytes of origin codes and walk_tok walk
  // tokens, walk_slot bytes in all (walk_steps == 0: none)
  uint8_t *walk;
  int32_t walk_steps, walk_tok;
  int64_t walk_codes, walk_slot;
  // one-wavefront pass: where pairs that leave its window go (route.nclass
  // == 0: to ring_list)
  WfaRoute route;
  // score passes with a CIGAR wanted: counters of accepted pairs left to the
  // full-store pass, because their fused walk failed (walk_fail; it cannot,
  // for codes that were kept and read back intact) or because their codes
  // were not kept (walk_skip: more scores than the code slot holds)
  int32_t *walk_fail, *walk_skip;
  // accepted pairs whose full store passes the largest class: appended here
  // for the memory-bounded pass (nullptr: they get CIGAR_OVERFLOW)
  int32_t *long_list, *long_count;
};

// The memory-bounded pass for long pairs (a CIGAR for pairs whose origin codes
// and full store fit no slot), one workgroup per pair with a slot of
// slot_words int32 words: the score pass again from s = 0 to the pair's known
// score, keeping its ring of the last R wavefronts every K scores as a
// checkpoint (at most ck_cap, K = ceil((score + 1) / ck_cap)) and each score's
// width; then the walk from the end cell back, recomputing from the
// checkpoint below the walk's score the origin codes of as many scores as
// code_cap bytes (and wt_cap table entries) hold, walking them, and again
// until the start.  Memory per pair: ck_cap rings, one code window and a
// width per score, instead of every score's codes.
struct WfaLong {
  int32_t R;
  int32_t wcap;       // widest wavefront (2 max_len + 1 bounds every pair)
  int32_t seq_words;  // LDS staging per sequence (0: read in place)
  int32_t ck_cap;     // checkpoints per pair
  int32_t sw_cap;     // scores (width table); a pair with a higher score gets CIGAR_OVERFLOW
  int32_t wt_cap;     // scores one recompute keeps the codes of
  int32_t tok_cap;    // walk tokens
  int64_t code_cap;   // bytes of origin codes per recompute (a multiple of 16)
  int64_t slot_words;
  int32_t *slots;
  int32_t *failed;    // pairs left CIGAR_OVERFLOW (a score or a code row past the caps)
};
int64_t wfa_long_slot_words(const WfaLong &L, bool i16);
constexpr int32_t WGMAX_THREADS = 256;  // workgroup of the long pass
// nslots workgroups of `threads`; i16: 16-bit ring entries (max_len <=
// WFA16_MAX_LEN).  Wk.direct: re-run, runs straight into the CIGAR output.
hipError_t launch_wfa_long(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, const WfaLong &L,
                           int32_t nslots, int32_t threads, bool i16, hipStream_t s);

// One LDS-window class of wide pairs (k_wfa_lds): the last R scores of M and
// the last e + 1 of I and D are LDS rows of packed 16-bit offsets indexed by
// absolute diagonal over the window [-W/2, W/2) plus MG entries of margin on
// each side.  Origin codes and a per-score table go to a per-workgroup HBM
// slot for the fused walk.
struct WfaLds {
  int32_t W, MG, R, seq_words;
  int32_t s_cap;          // scores a pair may take in this class (16-bit absent marks)
  int32_t my_class;       // this class's index in the route
  WfaRoute route;
  uint8_t *codes;         // per workgroup: steps_cap table entries (3 int32) + code_cap bytes
  int64_t code_slot;      // bytes per workgroup slot
  int32_t steps_cap;
  int64_t code_cap;
  // the full-store fallback, as in WfaLaunch
  int64_t need_cap[4];
  int32_t *need_list[4];
  int32_t *need_count[4];
  int32_t *need_max[4];
  int64_t *need;
  int32_t *walk_fail, *walk_skip;
  // non-null: the ring rows live in a global buffer, gring_slot words per
  // workgroup (wfa_ring_words), instead of LDS
  uint32_t *gring;
  int64_t gring_slot;
  // WFA-adaptive (ad_min > 0): after each score, trim outer diagonals whose
  // distance to the end lags the best by more than ad_max once the range
  // spans ad_min diagonals; ad_dropped counts them.  A pair whose codes do
  // not fit, or that passes s_cap, gets no fallback (the exact passes would
  // compute another alignment).
  int32_t ad_min, ad_max;
  unsigned long long *ad_dropped;
  int32_t *long_list, *long_count;  // as in WfaLaunch
};
int64_t wfa_ring_words(int32_t W, int32_t MG, int32_t R, int32_t e);
size_t wfa_lds_bytes(int32_t W, int32_t MG, int32_t R, int32_t e, int32_t seq_words, bool gring);
// threads: 64, 128, 256 or 512
hipError_t launch_wfa_lds(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, const WfaLds &L,
                          int32_t threads, int32_t nslots, hipStream_t s);

struct WfaPlan {
  int32_t R, wcap, wcap_lds, seq_words, lds_score_bytes, ring_slots, ring_threads, lds_arena_words;
  int64_t ring_slot_words;
  int64_t need_cap[4];
  int64_t pool_words[4];  // HBM arena per class (words)
  int32_t arena_slots[4];  // workgroups launched per class
  int32_t threads[4];
};

// strict: every pool (one slot of its class included) stays within its share
// of budget_bytes, shrinking the store classes if need be
WfaPlan wfa_plan(int32_t max_len, const Scoring &P, int64_t budget_bytes, int32_t cus, bool plain,
                 int32_t ring_kb, int32_t trace_kb, int32_t long_threads, bool strict = false);
// ring16 (HBM ring only): 16-bit ring entries, for batches with max_len <=
// WFA16_MAX_LEN.  The HBM ring must be readable for wfa_ring_pad(wcap) words
// before hbm and after its last slot (its steps read without clamping).
hipError_t launch_wfa_score(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                            const WfaLaunch &L, int32_t *hbm, bool ring_in_lds, int32_t nslots,
                            int32_t threads, bool ring16, hipStream_t s);
// Pass 1 by one wavefront per pair with 16-bit offsets in LDS over a window of
// 64 C diagonals (C <= 4); needs max_len <= WFA16_MAX_LEN and L.seq_words > 0
// (sequences staged in LDS).  Pairs that leave the window go to L.ring_list.
constexpr int32_t WFA16_MAX_LEN = 32000;
// Scores whose origin codes the one-wavefront pass keeps for its fused walk
// (32 bytes per 64 diagonals per score and workgroup).
constexpr int32_t WFA16_WALK_STEPS = 2048;
// Scores whose origin codes the HBM-ring score pass keeps for its fused walk.
constexpr int32_t WFA_WALK_STEPS = 16384;
size_t wfa_score16_lds(const WfaLaunch &L, int32_t e, int32_t C);
inline int64_t wfa_ring_pad(int32_t wcap) { return 4 * (int64_t)wcap + 1024; }
hipError_t launch_wfa_score16(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                              const WfaLaunch &L, int32_t C, int32_t nslots, hipStream_t s);
// i16: wavefronts stored as 16-bit offsets (max_len <= WFA16_MAX_LEN); the
// full-store sizes counted by the score passes then over-cover the store.
hipError_t launch_wfa_trace(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                            const WfaLaunch &L, int32_t *hbm, int32_t nslots, int32_t threads,
                            bool i16, hipStream_t s);

// CIGAR compaction: cigar_off from nruns (with the cap cut), copy slot and
// pool runs, collect pairs whose runs could not be held into the spill list.
hipError_t launch_compact(int64_t n, const Outs &O, int64_t *cigar_off, uint32_t *cigar,
                          int64_t cigar_cap, int64_t *scan_tmp, int64_t *total_written,
                          int32_t *spill_idx, int32_t *spill_count, int8_t *status,
                          hipStream_t s);
hipError_t launch_zero_offsets(int64_t n, int64_t *cigar_off, hipStream_t s);

// Length buckets: order[] = pair indices sorted by max(m, n), longest first
// (128 buckets, 8 per octave; order within a bucket unspecified).  hist needs
// 128 int32.
constexpr int LEN_BUCKETS = 128;
hipError_t launch_length_sort(int64_t n, const int32_t *pl, const int32_t *tl, int32_t *hist,
                              int32_t *order, hipStream_t s);

// Exact pre-alignment filter (filter.hip).  Lower bound of each pair's
// optimal cost from its Levenshtein distance (shorter side at most
// FILTER_REACH bases) and its length difference.  O == nullptr: writes
// lower[p] / pass[p] for every pair.  Otherwise, for the pairs of `idx`
// (nullptr: all n): finishes the rejected and invalid ones in O, appends the
// rest to list / count and counts the rejected in `rejected`.
constexpr int32_t FILTER_REACH = 1024;
hipError_t launch_prefilter(int64_t n, const Seqs &S, const int8_t *flags, int32_t max_len, int32_t x, int32_t o,
                            int32_t e, int32_t max_score, const int32_t *idx, int32_t *lower, int8_t *pass,
                            const Outs *O, int32_t *list, int32_t *count, int32_t *rejected, hipStream_t s);

// GenASM (windowed bitap with traceback, unit edits, threshold max_score),
// one pair per lane, 64 pairs per wavefront from Wk's counter.  Each
// wavefront keeps `levels` edit levels of 64 x 64 status words in its slot of
// `store`: genasm_block_words(levels) words per 256-thread block, nblocks
// blocks.  levels = genasm_levels(max_score).
int32_t genasm_levels(int32_t max_score);
int64_t genasm_block_words(int32_t levels);
hipError_t launch_genasm(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, uint64_t *store,
                         int32_t levels, int32_t nblocks, hipStream_t s);

// ---- allocation-free entry point ------------------------------------------
// Size of the static device array (one per GPU) that aim_align_batch_static
// carves its scratch from, and the scratch budget its launch plans are sized
// for (well below the array, since the plans' shares of a budget add up to
// more than half of it and some buffers have fixed minimum sizes).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)256 << 20;
constexpr int64_t STATIC_PLAN_BUDGET = (int64_t)96 << 20;
// The array's address on `device`, which must be the current device; looked
// up once per device (hipGetSymbolAddress) and kept.
hipError_t static_scratch_address(int device, void **out);

}  // namespace aim
