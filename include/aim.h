/*
 * aim.h -- C ABI of libaim.so: batched global pairwise alignment on AMD
 * MI355X (gfx950).
 *
 * The operation follows the problem statement of the Alignment-in-Memory
 * paper (System and Methods, "Overall Workflow" and "Supported Alignment
 * Algorithms"): a batch of read pairs goes in, every pair is aligned on its
 * own by the chosen algorithm with the chosen scoring parameters, and the
 * alignment score plus the alignment operations (a CIGAR) come out per pair.
 * An edit-distance threshold (abstract; GenASM's k) bounds the work: pairs
 * whose optimum exceeds it are reported as rejected.
 *
 * Alignment model (all algorithms):
 *   global (end to end) alignment of a pattern P (m bases) against a text T
 *   (n bases); costs are minimised; match costs 0, a mismatch costs x, a run
 *   of L gap bases costs gap_open + L * gap_extend (linear NW: gap_open 0).
 *   Ops: '=' match, 'X' mismatch, 'I' a base of P only, 'D' a base of T only.
 *   Among co-optimal alignments the library returns the canonical one: walking
 *   back from the end it takes, at each cell, the first feasible op of
 *   X, I, D, '=' and closes a gap run as early (towards the start) as the
 *   optimum allows.  NW, SWG and WFA return identical CIGARs for identical
 *   costs (SWG with gap_open 0 equals NW).
 *
 * Conventions:
 *   - Every call returns aim_status: AIM_OK (0) or a negative error code;
 *     aim_last_error() then describes it.  Nothing throws across the ABI.
 *   - Device pointers are HIP device (or managed) memory of the context's
 *     device.  The caller owns every buffer it passes; the library owns its
 *     scratch, which lives in the context and grows on demand, in stream
 *     order on the call's stream (hipFreeAsync / hipMallocAsync), so growing
 *     one context does not synchronise the device.  A call on a different
 *     stream than the context's previous call first waits for that call.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *     null stream); outputs are valid once the stream is synchronised.  Calls
 *     that share a context must not run concurrently from several host
 *     threads.
 *   - Per-pair outcomes are statuses, not errors (AIM_PAIR_*).
 */
#ifndef AIM_H
#define AIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t aim_status;
#define AIM_OK 0
#define AIM_ERR_INVALID_ARG (-1) /* bad pointer, size, penalty or option */
#define AIM_ERR_UNSUPPORTED (-2) /* valid but not supported (e.g. match != 0) */
#define AIM_ERR_OOM (-3)         /* device scratch allocation failed */
#define AIM_ERR_HIP (-4)         /* a HIP runtime call failed */
#define AIM_ERR_BUSY (-5)        /* serving: queue full / request still running */
#define AIM_ERR_NOT_FOUND (-6)   /* serving: unknown request id */

typedef enum {
  AIM_NW_LINEAR = 0,
  AIM_SWG_AFFINE = 1,
  AIM_WFA_AFFINE = 2,
  AIM_WFA_ADAPTIVE = 3,
  AIM_GENASM = 4
} aim_algorithm;

/* Sequence encodings.  ASCII: bytes 'A','C','G','T' (upper case only).
 * CODE: bytes 0..3 for A, C, G, T.  2BIT: 32 bases per uint64 word, base t of
 * a sequence at bits 2*(t % 32) of word t / 32; each sequence starts on a
 * word boundary.  Anything outside the alphabet makes that pair
 * AIM_PAIR_INVALID. */
typedef enum { AIM_ENC_ASCII = 0, AIM_ENC_CODE = 1, AIM_ENC_2BIT = 2 } aim_encoding;

/* Per-pair status values written to aim_results.status. */
#define AIM_PAIR_ALIGNED 0
#define AIM_PAIR_REJECTED 1       /* optimum > max_score: score -1, empty CIGAR */
#define AIM_PAIR_CIGAR_OVERFLOW 2 /* score valid, no CIGAR: it did not fit cigar_cap, or
                                     (WFA) its full store passes the largest class
                                     and the memory-bounded long pass cannot take
                                     it either (scratch too small for one of its
                                     slots, a score past 2^20, or one score's
                                     origin codes past its code window; see
                                     aim_call_stats.wfa_long_failed), or (WFA-
                                     adaptive) its origin codes outgrew the slot */
#define AIM_PAIR_INVALID 3        /* non-ACGT base or length beyond max_len */

/* CIGAR run encoding: (run_length << 4) | op. */
#define AIM_OP_MATCH 0
#define AIM_OP_MISMATCH 1
#define AIM_OP_INS 2 /* consumes the pattern only */
#define AIM_OP_DEL 3 /* consumes the text only */

/* Scoring parameters, as costs (paper: NW uses a match cost a, mismatch cost
 * x and gap cost e; SWG and WFA add a gap-opening cost o).  Requirements:
 * match == 0, mismatch > 0, gap_extend > 0, gap_open >= 0, each <= 65535;
 * AIM_NW_LINEAR requires gap_open == 0 (one gap base costs gap_extend).
 * Violations return AIM_ERR_UNSUPPORTED (match != 0) or AIM_ERR_INVALID_ARG. */
typedef struct {
  int32_t match, mismatch, gap_open, gap_extend;
} aim_penalties;

/* A batch of pairs in CSR form (all arrays are device pointers).
 *   pat_seq / txt_seq: concatenated sequences in encoding `enc`
 *     (uint8 for ASCII/CODE, uint64 words for 2BIT);
 *   pat_off / txt_off: int64 [n_pairs] start of each sequence, in bytes for
 *     ASCII/CODE and in uint64 words for 2BIT;
 *   pat_len / txt_len: int32 [n_pairs] lengths in bases.
 * max_len is a host-side upper bound on every length (it sizes scratch);
 * a pair whose length exceeds it, or is negative, is AIM_PAIR_INVALID.
 * 0 <= max_len <= 1048576. */
typedef struct {
  int64_t n_pairs;
  int32_t enc;
  int32_t max_len;
  const void *pat_seq;
  const int64_t *pat_off;
  const int32_t *pat_len;
  const void *txt_seq;
  const int64_t *txt_off;
  const int32_t *txt_len;
} aim_batch;

/* Outputs (device pointers, caller-owned).
 *   score:     int32 [n_pairs], the optimal cost, -1 when rejected/invalid;
 *   status:    int8  [n_pairs], AIM_PAIR_*;
 *   cigar:     uint32 [cigar_cap] RLE runs of all pairs, CSR by cigar_off;
 *   cigar_off: int64 [n_pairs + 1]; pair p owns cigar[cigar_off[p] ..
 *              cigar_off[p+1]).  Pairs are laid out in order; the first pair
 *              whose runs would pass cigar_cap and every later pair get
 *              AIM_PAIR_CIGAR_OVERFLOW and an empty range.
 *   want_cigar: 0 = score only (cigar may be NULL, cigar_off all zero). */
typedef struct {
  int32_t *score;
  int8_t *status;
  uint32_t *cigar;
  int64_t *cigar_off;
  int64_t cigar_cap;
  int32_t want_cigar;
} aim_results;

/* Kernel family.
 *   AIM_KERNEL_AUTO  -- the production path: NW/SWG run a banded DP with one
 *     pair per GPU lane whose band is proven exact per pair (or widened), WFA
 *     runs the wavefront kernel over length-bucketed work queues.
 *   AIM_KERNEL_PLAIN -- the baseline: one pair per workgroup over the full
 *     DP matrix (NW/SWG) or one pair per workgroup WFA without bucketing.
 * Both return identical results. */
typedef enum { AIM_KERNEL_AUTO = 0, AIM_KERNEL_PLAIN = 1 } aim_kernel;

/* aim_options.flags bits */
#define AIM_FLAG_TIMING 1 /* time every kernel launch with HIP events (aim_timing) */
#define AIM_FLAG_STATIC_SCRATCH 2 /* set up aim_align_batch_static's array at create */
#define AIM_FLAG_NO_PREFILTER 4   /* aligning calls skip the pre-alignment filter */
#define AIM_FLAG_HARD_LIMIT 8     /* scratch_limit is a hard cap (see aim_options) */

typedef struct {
  int32_t kernel;        /* aim_kernel */
  int32_t flags;         /* AIM_FLAG_* */
  /* Library scratch budget in bytes (0: 64 GiB).  Launch plans are sized
   * for it.  Without AIM_FLAG_HARD_LIMIT it is soft: buffers that grow with
   * the batch (per-pair arrays) may pass it.  With the flag the device
   * memory the context's scratch holds never exceeds it (launch plans are
   * then sized for half of it, 3/8 below 1 GiB, the rest holding the arrays
   * that grow with the batch): a call that would need more fails with
   * AIM_ERR_OOM (its outputs
   * are then unspecified), and a smaller batch can be retried on the same
   * context. */
  int64_t scratch_limit;
} aim_options;

typedef struct aim_context aim_context;

/* Create a context on HIP device `device`.  opt may be NULL (defaults).
 * Paper: Data Management, dynamic memory allocation -- the framework gives
 * each worker its own allocator instead of a shared one; a context is that
 * owner here: its scratch (grown on demand, kept across calls) serves only
 * the calls made with it.
 * Returns AIM_ERR_INVALID_ARG for a bad device or options, AIM_ERR_HIP if the
 * runtime refuses the device. */
aim_status aim_create(aim_context **ctx, int32_t device, const aim_options *opt);

/* Release the context and all its scratch (paper: Data Management, the
 * per-worker allocator frees everything at once).  Waits for its work to
 * finish.  NULL is ignored. */
void aim_destroy(aim_context *ctx);

/* Align every pair of `pairs` (paper: workflow steps 3-5 for all pairs,
 * "Supported Alignment Algorithms" for `alg`), writing `out`.
 *   alg: AIM_NW_LINEAR (NW subsection), AIM_SWG_AFFINE (SWG subsection, global
 *        form), AIM_WFA_AFFINE (WFA subsection, exact gap-affine WFA),
 *        AIM_WFA_ADAPTIVE (WFA subsection, the heuristic variant that drops
 *        outer diagonals; see aim_wfa_adaptive_params for the rule -- the
 *        result is a valid alignment whose cost is at least the optimum and
 *        at most the reported score, and is the same as exact WFA whenever
 *        no diagonal is dropped; max_len <= 16,000, else
 *        AIM_ERR_UNSUPPORTED; a pair whose score passes 16,000 times the
 *        penalties' common divisor is AIM_PAIR_INVALID),
 *        AIM_GENASM (GenASM subsection: bitap with a traceback under a bound
 *        k on the edits; the library's reading, unit edits in windows of 64
 *        bases overlapping by 24, is spelled out below);
 *   pen: scoring parameters (see aim_penalties; validated but unused by
 *        AIM_GENASM, which counts edits);
 *   max_score: threshold in penalty units (AIM_GENASM: k, in edits); a pair
 *        whose optimum (AIM_GENASM, WFA-adaptive: whose result) exceeds it is
 *        AIM_PAIR_REJECTED; < 0 means no threshold.  Results of accepted pairs
 *        do not depend on it.
 * AIM_GENASM aligns a pair from its end towards its start in windows of at
 * most 64 pattern and 64 text bases taken from the end of what is still to
 * align.  The last window (64 bases or fewer of each left) must reach the
 * start of both sequences; the others may begin anywhere on their first row
 * or column.  In each window the bitap distance calculation finds the fewest
 * edits d (status bit i of text position j at level d says whether the
 * window's first i pattern and j text bases align within d edits), and a
 * traceback from the window's end spends that budget taking, at each cell,
 * the first available of: the previous op again if it was 'I' or 'D'; '=';
 * 'X'; 'I'; 'D'.  A window other than the last commits ops until 40 bases of
 * either sequence are consumed or its first row or column is reached; when
 * either sequence runs out the rest of the other is one gap.  The score is
 * the number of edits (at least the Levenshtein distance; equal to it when
 * both sequences fit one window), and a window that needs more edits than k
 * still allows, or a total above k, rejects the pair.
 * Asynchronous on `stream`.  Errors: AIM_ERR_INVALID_ARG (NULL pointers,
 * n_pairs < 0, max_len out of range, cigar_cap < 0 with want_cigar),
 * AIM_ERR_UNSUPPORTED (penalties), AIM_ERR_OOM, AIM_ERR_HIP. */
aim_status aim_align_batch(aim_context *ctx, const aim_batch *pairs, int32_t alg,
                           aim_penalties pen, int32_t max_score, aim_results *out, void *stream);

/* aim_align_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * this call allocates and frees nothing.  Its scratch is carved from one
 * static device array of 256 MiB per GPU, which that GPU holds from the first
 * such call on it (or from aim_create with AIM_FLAG_STATIC_SCRATCH, which does
 * the set-up there) until the process ends.  Launch plans are sized for a
 * 96 MiB scratch budget.  A batch whose scratch would pass the 256 MiB returns
 * AIM_ERR_INVALID_ARG; kernels enqueued before the check found it may have
 * written parts of `out`, which is then unspecified -- split such a batch, or
 * use aim_align_batch.  The caller owns inputs and outputs as for
 * aim_align_batch; arguments, errors, asynchrony and results (bit for bit) are
 * those of aim_align_batch, and calls on one context are ordered the same way.
 * Every call on one GPU, from any context, shares that GPU's array, which
 * keeps the last call's contents (each call clears what it needs zeroed):
 * calls that overlap in time on one GPU race. */
aim_status aim_align_batch_static(aim_context *ctx, const aim_batch *pairs, int32_t alg,
                                  aim_penalties pen, int32_t max_score, aim_results *out,
                                  void *stream);

/* Parameters of AIM_WFA_ADAPTIVE on this context (defaults 10 and 50).
 * Paper: WFA subsection -- WFA-adaptive removes the outer diagonals unlikely
 * to lead to the optimum; the rule (a reading, the paper gives none): after
 * each score's wavefront is computed and extended, if it spans at least
 * min_len diagonals, each diagonal k whose M offset f reaches text position
 * f and pattern position f - k gets the distance max(m - (f - k), n - f) to
 * the end, and diagonals are removed from both ends of the range, inwards,
 * while their M is absent or their distance exceeds the smallest by more
 * than max_dist; removed cells no longer feed later scores.  The score is
 * the first wavefront score that reaches the end cell.  min_len >= 1,
 * max_dist >= 0, else AIM_ERR_INVALID_ARG. */
aim_status aim_wfa_adaptive_params(aim_context *ctx, int32_t min_len, int32_t max_dist);

/* Device bytes the context's scratch holds now (`current`) and the most it
 * has held at any time since aim_create (`peak`), from the context's own
 * allocation accounting (buffers of aim_align_batch_static's static array
 * excluded).  Either pointer may be NULL.  Paper: Data Management (the
 * host decides what each processing unit's memory holds); this is the figure
 * a caller budgets device memory with. */
aim_status aim_scratch_usage(aim_context *ctx, int64_t *current, int64_t *peak);

/* Exact pre-alignment filter (paper: Introduction, the third way to speed
 * up alignment -- drop, before aligning them, the pairs that are too
 * dissimilar, without losing any pair that meets the threshold).
 * For each pair writes a lower bound of its optimal cost under (alg, pen):
 *   lower[p] = max(A, B), where, for a pattern of m and a text of n bases,
 *     B = gap_open + gap_extend * |m - n| if m != n, else 0  (a length
 *         difference needs one gap run; gap_open counts as 0 for NW), and
 *     A = min(mismatch, gap_extend) * lev + gap_open * [m != n], lev being
 *         the Levenshtein distance (every alignment makes at least lev edits,
 *         each costing at least min(mismatch, gap_extend)); A is taken only
 *         when min(m, n) <= 1024, else lower = B;
 *   pass[p]  = 1 if max_score < 0 or lower[p] <= max_score, else 0: a pair
 *         with pass 0 is certain to be AIM_PAIR_REJECTED by aim_align_batch
 *         with the same arguments.
 * For AIM_GENASM the bound is taken with unit edits (mismatch and
 * gap_extend 1, gap_open 0) against max_score = k: GenASM's edits are at
 * least the Levenshtein distance.
 * An invalid pair (see aim_batch) gets lower -1 and pass 0.
 *   pairs: as for aim_align_batch; lower: device int32 [n_pairs];
 *   pass: device int8 [n_pairs] (caller-owned).
 * aim_align_batch runs the same filter in front of its aligners whenever
 * max_score >= 0, for WFA and WFA-adaptive always and for NW and SWG when
 * max_len > 256 (never for GenASM) (unless AIM_FLAG_NO_PREFILTER or AIM_KERNEL_PLAIN); its
 * results do not change, only the work spent on rejected pairs.
 * Asynchronous on `stream`, ordered with the context's other calls like
 * aim_align_batch; errors as for aim_align_batch. */
aim_status aim_prefilter(aim_context *ctx, const aim_batch *pairs, int32_t alg, aim_penalties pen,
                         int32_t max_score, int32_t *lower, int8_t *pass, void *stream);

/* Encode sequences as 2-bit words (the "2BIT" layout above).
 *   enc: AIM_ENC_ASCII or AIM_ENC_CODE; seq/off/len: device CSR (byte offsets);
 *   out_off: device int64 [n_seqs + 1], written: word offset of each output
 *            sequence (ceil(len/32) words each, in order), out_off[n] = total;
 *   out_words: device uint64 [words_cap]; words_cap must be >= the total
 *            (sum of ceil(len/32)), else AIM_ERR_INVALID_ARG is *not*
 *            detectable without a sync, so the kernel writes only words below
 *            words_cap and flags the rest;
 *   seq_flags: device int8 [n_seqs] or NULL; set to 1 for a sequence holding
 *            a byte outside the alphabet (or truncated by words_cap), else 0.
 * Paper: the full pair sits in fast memory during alignment (Data
 * Management); packing 4 bases per byte is how this library keeps it small. */
aim_status aim_pack_2bit(aim_context *ctx, int64_t n_seqs, int32_t enc, const uint8_t *seq,
                         const int64_t *off, const int32_t *len, uint64_t *out_words,
                         int64_t words_cap, int64_t *out_off, int8_t *seq_flags, void *stream);

/* Per-phase GPU time of the launches made since the last aim_timing_reset,
 * measured with HIP events recorded on the launch stream around each kernel
 * (only with AIM_FLAG_TIMING).  Phase `idx` = 0, 1, ...: writes its name
 * (static string, e.g. "band32", "full", "wfa", "compact"), the summed
 * milliseconds and the number of launches.  Waits for the recorded events.
 * Returns AIM_ERR_NOT_FOUND past the last phase. */
aim_status aim_timing(aim_context *ctx, int32_t idx, const char **name, double *total_ms,
                      int64_t *launches);
aim_status aim_timing_reset(aim_context *ctx);

/* Work counters of the context's last aligning call (aim_align_batch, a graph
 * replay, or aim_align_batch_static -- whose counters live in the shared
 * static array, so a later static call on the same GPU overwrites them).
 * Waits for that call to finish.  All zero before the first call or after
 * an empty batch.  These say which paths the pairs took; they are not part of
 * the results, which are the same whatever the path.
 *   band_escalated / band_escalated2: NW/SWG pairs the 32-diagonal band passed
 *     on to the 64-diagonal band, and that band on to the last tier;
 *   wfa_wide: WFA pairs whose wavefronts left the one-wavefront window;
 *   wfa_walk_failed: WFA pairs whose walk over the kept origin codes failed
 *     (0 unless a code was read back wrong; each is re-walked from a full
 *     store, so results stay exact and only time is lost);
 *   wfa_walk_skipped: accepted WFA pairs whose codes were not kept (more
 *     scores than the code slot holds);
 *   full_store[c]: pairs walked by the full-store pass, per store class
 *     (LDS, 1 MB, 16 MB, largest);
 *   cigar_reruns: pairs whose runs outgrew their slot and the run pool,
 *     re-aligned in place by the compaction;
 *   wfa_window: the diagonals the one-wavefront WFA pass keeps, centred on
 *     diagonal 0 (0: that pass did not run); pairs whose wavefronts stay
 *     inside it are aligned there, the others go to wider windows;
 *   wfa_class_pairs[c] / wfa_class_window[c]: pairs routed to the c-th LDS
 *     window class, and its window in diagonals (0: no such class);
 *     wfa_wide counts the pairs that outgrew them all (HBM-ring pass);
 *   prefilter_rejected: pairs rejected by the pre-alignment filter before
 *     any aligner ran (see aim_prefilter);
 *   wfa_adaptive_dropped: diagonals the WFA-adaptive reduction removed;
 *   wfa_long_pairs: accepted WFA pairs whose full store passes the largest
 *     class, walked by the memory-bounded long pass (checkpoints of the
 *     wavefront ring and a window of recomputed origin codes);
 *   wfa_long_failed: of those, pairs left CIGAR_OVERFLOW (a score or one
 *     score's codes past that pass's caps, or no room for its slots). */
typedef struct {
  int64_t n_pairs;
  int32_t band_escalated, band_escalated2;
  int32_t wfa_wide, wfa_walk_failed, wfa_walk_skipped;
  int32_t full_store[4];
  int32_t cigar_reruns;
  int32_t wfa_window;
  int32_t wfa_class_pairs[4];
  int32_t wfa_class_window[4];
  int32_t prefilter_rejected;
  int64_t wfa_adaptive_dropped;
  int32_t wfa_long_pairs, wfa_long_failed;
} aim_call_stats;
aim_status aim_last_call_stats(aim_context *ctx, aim_call_stats *out);

/* ---- batching form: autotuner and captured graphs ---------------------- */

/* Time every candidate launch configuration on this batch and keep the
 * fastest for (alg, length bucket of pairs->max_len); later calls with that
 * key use it.  Candidates: NW/SWG -- first band width {32, 64}, resident
 * wavefronts per CU {8, 16, 32}, length sort {off, on}, packed 16-bit cells
 * {off, on} (32 diagonals only); WFA -- length sort {off, on}, one-wavefront
 * window {64, 128, 256} diagonals, workgroup size for the widest pairs {128,
 * 256}, then, for each window class the batch uses, its workgroup size {64,
 * 128, 256} (pairs per workgroup: one; lanes per pair: the size) and where its
 * ring lives (LDS or a global slot), kept per class length bucket (the
 * class's extent bound, or max_len for the last class), so one mixed batch
 * runs each bucket with its own configuration; WFA-adaptive -- length sort,
 * workgroup size {64, 128}.  Each candidate runs once to warm up and `reps`
 * times timed (median).  Synchronous.  On return `out` holds the results of
 * the chosen configuration; best_params (13 int32, see aim_tune_get) and
 * best_ms (the fastest candidate's time) may be NULL.  Paper: Data
 * Management (the framework picks the number of DPU threads from the
 * algorithm, read length and error rate; WRAM or MRAM per read length). */
aim_status aim_autotune(aim_context *ctx, const aim_batch *pairs, int32_t alg, aim_penalties pen,
                        int32_t max_score, aim_results *out, void *stream, int32_t reps,
                        int32_t *best_params, double *best_ms);

/* Launch parameters for (alg, max_len), 13 int32: params[0] first band width,
 * [1] wavefronts per CU (first band tier; GenASM), [2] length sort (-1 auto, 0 off, 1 on), [3] WFA ring
 * LDS KB, [4] WFA full-store LDS KB, [5] WFA long-pair workgroup size,
 * [6] packed 16-bit band cells when the value bound allows (0 off; 1 on, each
 * wavefront walking its own pairs' tracebacks; 2 on, the tracebacks walked by
 * a second kernel beside the escalation tiers; 3, the default: 2 for batches
 * of at least 65536 pairs, else 1, or 0 for fewer than 16384 pairs of reads
 * of at most 128 bases), [7] WFA pairs wider than the
 * one-wavefront window go through LDS-window classes (1, the default) or
 * straight to the HBM-ring pass (0), [8..10] workgroup size (64, 128, 256 or
 * 512) of the three window classes (narrowest first), [11] bit c set: class
 * c + 1 keeps its recent wavefronts in a global buffer rather than LDS, [12]
 * the one-wavefront window in units of 64 diagonals (0: from the batch; at
 * most 4).  A class tune kept for a class's length bucket (aim_autotune)
 * overrides [8..11] for that class.  Without a kept tune, the built-in
 * defaults apply (aim_tune_get returns them): those above, except [10] 256
 * and [12] 1 for WFA batches with max_len >= 4096, and [2] 0 for GenASM
 * below 512 bases (the autotuner's choices on MI355X);
 * and with [6] at 3, batches of fewer than 16,384 pairs of reads of at most
 * 128 bases use the 32-bit band (one pair per lane, twice the wavefronts of
 * the packed band). */
aim_status aim_tune_get(aim_context *ctx, int32_t alg, int32_t max_len, int32_t *params);
aim_status aim_tune_set(aim_context *ctx, int32_t alg, int32_t max_len, const int32_t *params);
/* The kept tunes: for entry i < min(cap, *count), kind[i] 0 (batch tune) or
 * 1 (WFA class tune), alg[i] and bucket[i] (a length bucket: the smallest b
 * with 2^b > length).  *count is the number of entries. */
aim_status aim_tune_entries(aim_context *ctx, int32_t cap, int32_t *kind, int32_t *alg, int32_t *bucket,
                            int32_t *count);
/* Tune cache as text, keyed by GPU architecture and HIP runtime version; a
 * file for another architecture or runtime is refused (AIM_ERR_NOT_FOUND). */
aim_status aim_tune_save(aim_context *ctx, const char *path);
aim_status aim_tune_load(aim_context *ctx, const char *path);

/* Capture one aim_align_batch call (same arguments) as a HIP graph for
 * repeated batches of the same shape.  Runs the call once eagerly first (so
 * scratch is sized and `out` is valid), then captures it on `stream` (must
 * not be NULL).  The graph keeps the batch and result pointers: replays
 * re-align whatever those buffers hold.  A replay is refused
 * (AIM_ERR_INVALID_ARG) if the context's scratch was reallocated since
 * capture, or if the context was destroyed; aim_graph_destroy may be called
 * before or after aim_destroy of its context.  Not thread-safe with other
 * calls on the same context. */
typedef struct aim_graph aim_graph;
aim_status aim_graph_capture(aim_context *ctx, const aim_batch *pairs, int32_t alg,
                             aim_penalties pen, int32_t max_score, aim_results *out, void *stream,
                             aim_graph **graph);
aim_status aim_graph_launch(aim_graph *graph, void *stream);
void aim_graph_destroy(aim_graph *graph);

/* ---- serving form ---------------------------------------------------------
 * A request server: alignment requests of any size arrive on host threads,
 * wait in one FIFO queue (never dropped, never bypassed by a request of the
 * same kind), and are merged -- in queue order, per (algorithm, penalties,
 * threshold, CIGAR wanted, encoding) -- into device batches by n_streams
 * workers, each with its own context, stream and buffers, so batches
 * overlap on the GPU and requests that arrive while others run join the
 * next batch.  The device-memory budget is split evenly between the
 * workers: of each share, an eighth (at most 1 GiB) holds input staging, as
 * much output staging, and the rest is the hard scratch limit of the worker's context
 * (AIM_FLAG_HARD_LIMIT), so the device memory the server holds never passes
 * the budget; a request is admitted to the device when a worker, with its
 * share, frees up.  A batch that needs more scratch than the share is split
 * in two by request and each half run again; a single request that still
 * does not fit fails with AIM_ERR_OOM.  Paper: Overall Workflow (the host
 * gathers pairs, dispatches them, retrieves score and operations), run
 * continuously. */
typedef struct aim_server aim_server;

typedef struct {
  int32_t n_streams;       /* concurrent device batches, 1..16 (0: 4) */
  int32_t flags;           /* reserved, 0 */
  int64_t budget_bytes;    /* device bytes the server may hold (0: 64 GiB); at least
                              64 MiB per stream */
  int64_t max_batch_pairs; /* pairs merged into one device batch (0: 65,536); a single
                              request larger than this still runs as one batch */
} aim_server_options;

/* One request: host arrays (copied at submit; the caller may reuse them
 * after aim_server_submit returns).  Offsets are in bytes. */
typedef struct {
  int32_t alg;
  aim_penalties pen;
  int32_t max_score;
  int32_t want_cigar;
  int32_t enc; /* AIM_ENC_ASCII or AIM_ENC_CODE */
  int64_t n_pairs;
  const uint8_t *pat;
  const int64_t *pat_off;
  const int32_t *pat_len;
  const uint8_t *txt;
  const int64_t *txt_off;
  const int32_t *txt_len;
} aim_request;

/* Results of a finished request: host arrays owned by the server until
 * aim_server_release; same meaning as aim_results (cigar_off starts at 0). */
typedef struct {
  int64_t n_pairs;
  const int32_t *score;
  const int8_t *status;
  const uint32_t *cigar;
  const int64_t *cigar_off;
  double latency_us; /* completion minus submission */
} aim_request_result;

/* bytes_in_use: device bytes the workers hold now (staging plus their
 * contexts' scratch, from aim_scratch_usage); peak_bytes: the most they have
 * held together since creation or the last reset (the sum of each worker's
 * high-water mark, an upper bound of any instant's total). */
typedef struct {
  int64_t submitted, completed, pairs_completed, batches, queued;
  double p50_us, p99_us, mean_us, max_us; /* latency of completed requests */
  int64_t bytes_in_use, peak_bytes, budget_bytes;
  double elapsed_s; /* since the first submission after the last reset */
} aim_server_stats;

/* Errors of the aim_server_* calls are described by aim_server_last_error. */
aim_status aim_server_create(int32_t device, const aim_server_options *opt, aim_server **srv);
/* Queues a request; returns at once with its id.  AIM_ERR_INVALID_ARG for a
 * request whose staging (sequences, offsets, lengths in; scores, statuses
 * and worst-case CIGAR out) exceeds a worker's staging share. */
aim_status aim_server_submit(aim_server *srv, const aim_request *req, int64_t *id);
/* AIM_ERR_BUSY while the request runs; AIM_ERR_NOT_FOUND for unknown ids. */
aim_status aim_server_poll(aim_server *srv, int64_t id, aim_request_result *res);
/* Blocks until done (timeout_ms < 0: no timeout; AIM_ERR_BUSY on timeout). */
aim_status aim_server_wait(aim_server *srv, int64_t id, int32_t timeout_ms, aim_request_result *res);
/* Frees a finished request's results. */
aim_status aim_server_release(aim_server *srv, int64_t id);
aim_status aim_server_stats_get(aim_server *srv, aim_server_stats *st);
aim_status aim_server_reset_stats(aim_server *srv);
const char *aim_server_last_error(void);
/* Finishes every queued request, then stops the workers and frees all. */
void aim_server_destroy(aim_server *srv);

/* Description of the last error on this host thread ("" if none).  Valid
 * until the next library call on the same thread.  (Not an operation of the
 * paper: the error channel of this C interface.) */
const char *aim_last_error(void);

/* Library version string. */
const char *aim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AIM_H */
