// Exact pre-alignment filter.
//
// Paper, Introduction: besides faster alignment kernels and more parallel
// hardware, work can be saved by filtering out, before alignment, the pairs
// that are too dissimilar -- provided no pair that would meet the threshold
// is lost.  Here a pair is dropped only when a proven lower bound of its
// optimal cost already exceeds the threshold.
//
// The bound, for penalties (0, x, o, e) (linear NW: o = 0) and a pattern of
// m bases against a text of n bases: every alignment makes at least
// lev(P, T) edits (the Levenshtein distance) and each edit costs at least
// min(x, e); a length difference forces a gap run, so one opening o and
// |m - n| extensions.  Hence
//   A = min(x, e) * lev + o * [m != n],  B = [m != n] * (o + e * |m - n|),
//   lower = max(A, B) <= optimum,
// with A taken when the shorter sequence has at most FILTER_REACH bases.
//
// lev is computed with bit-parallel column updates (Myers' bit-vector
// edit-distance recurrence in its block form, global variant): the shorter
// sequence is the bit side, one bit per base, 32 bases per word, and each
// base of the longer sequence advances every word by one column.  The
// vertical deltas of the last column then sum to lev.  One pair per lane,
// no LDS: the two bit planes of the short sequence and the two delta vectors
// of each word stay in registers; the word count is picked per wavefront.
#include "aim_internal.h"
#include "dev_util.h"

namespace aim {
namespace {

using dev::even_bits;
using dev::wave_max;

// Levenshtein distance of the short side s (sl bases, sl <= 32 * NW) against
// the long side t (tl bases).  All lanes of the wavefront call it; `tmax` is
// the wavefront's largest tl, `on` says whether this lane's result is used.
template <int NW>
__device__ __forceinline__ int32_t lev_bits(const uint64_t *s, int32_t sl, const uint64_t *t, int32_t tl, int32_t tmax,
                            bool on) {
  uint32_t p0[NW], p1[NW], pv[NW], mv[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint64_t word = (on && w * 32 < sl) ? s[w] : 0ull;
    p0[w] = even_bits(word);
    p1[w] = even_bits(word >> 1);
    pv[w] = ~0u;  // first column: D[i][0] = i, every vertical delta +1
    mv[w] = 0u;
  }
  uint64_t tw = 0;
  for (int32_t j = 0; j < tmax; ++j) {
    const bool live = on && j < tl;
    if ((j & 31) == 0) tw = live ? t[j >> 5] : 0ull;
    if (live) {
      const uint32_t c = (uint32_t)(tw >> (2 * (j & 31))) & 3u;
      const uint32_t m0 = 0u - (c & 1u), m1 = 0u - (c >> 1);
      // horizontal delta entering the top of the column: row 0 holds
      // D[0][j] = j, so +1 at every column
      uint32_t hp = 1u, hm = 0u;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        uint32_t eq = ~((p0[w] ^ m0) | (p1[w] ^ m1));  // bases equal to t[j]
        const uint32_t xv = eq | mv[w];
        eq |= hm;
        const uint32_t xh = (((eq & pv[w]) + pv[w]) ^ pv[w]) | eq;
        uint32_t ph = mv[w] | ~(xh | pv[w]);
        uint32_t mh = pv[w] & xh;
        const uint32_t hpo = ph >> 31, hmo = mh >> 31;
        ph = (ph << 1) | hp;
        mh = (mh << 1) | hm;
        pv[w] = mh | ~(xv | ph);
        mv[w] = ph & xv;
        hp = hpo;
        hm = hmo;
      }
    }
  }
  // D[sl][tl] = D[0][tl] + the vertical deltas of rows 1..sl in column tl
  int32_t d = tl;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int32_t r = sl - 32 * w;
    const uint32_t mask = r >= 32 ? ~0u : (r > 0 ? (1u << r) - 1u : 0u);
    d += __popc(pv[w] & mask) - __popc(mv[w] & mask);
  }
  return d;
}

template <int NWMAX>
__device__ __forceinline__ int32_t lev_dispatch(int32_t nw, const uint64_t *s, int32_t sl, const uint64_t *t, int32_t tl,
                                int32_t tmax, bool on) {
  if (nw <= 1) return lev_bits<1>(s, sl, t, tl, tmax, on);
  if (nw <= 2) return lev_bits<2>(s, sl, t, tl, tmax, on);
  if (nw <= 4) return lev_bits<4>(s, sl, t, tl, tmax, on);
  if constexpr (NWMAX == 8) {
    return lev_bits<8>(s, sl, t, tl, tmax, on);
  } else if constexpr (NWMAX == 16) {
    if (nw <= 8) return lev_bits<8>(s, sl, t, tl, tmax, on);
    return lev_bits<16>(s, sl, t, tl, tmax, on);
  } else {
    if (nw <= 8) return lev_bits<8>(s, sl, t, tl, tmax, on);
    if (nw <= 16) return lev_bits<16>(s, sl, t, tl, tmax, on);
    return lev_bits<32>(s, sl, t, tl, tmax, on);
  }
}

// LIST = false: write lower[p] and pass[p] for every pair (lower -1 and pass
// 0 for an invalid pair).  LIST = true: in front of the aligners -- a
// rejected pair gets its final outputs here (score -1, REJECTED, no runs), an
// invalid one likewise (INVALID), and the rest are appended to `list` in
// their order within each wavefront.
template <int NWMAX, bool LIST>
__global__ __launch_bounds__(256) void k_prefilter(int64_t n, Seqs S, const int8_t *flags, int32_t x, int32_t o,
                                                   int32_t e, int32_t max_score, const int32_t *idx,
                                                   int32_t *lower, int8_t *pass, Outs O, int32_t *list,
                                                   int32_t *count, int32_t *rejected) {
  const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool has = li < n;
  const int64_t p = has ? (idx ? (int64_t)idx[li] : li) : 0;
  const bool valid = has && !(flags && flags[p]);
  const int32_t m = valid ? S.pat_len[p] : 0, nn = valid ? S.txt_len[p] : 0;
  const bool diff = m != nn;
  const int32_t ad = diff ? (m > nn ? m - nn : nn - m) : 0;
  const int64_t lb_len = diff ? (int64_t)o + (int64_t)e * ad : 0;
  const int32_t ce = min(x, e);
  const int32_t sl = min(m, nn), tl = max(m, nn);
  // A is needed when it can decide something: always for the plain output;
  // in front of the aligners only when the length term does not already
  // reject and A's largest possible value (every base of the longer side an
  // edit) could pass the threshold
  bool need = valid && sl <= FILTER_REACH;
  if (LIST)
    need = need && lb_len <= max_score && (int64_t)ce * tl + (diff ? o : 0) > max_score;
  const int32_t nw = wave_max(need ? (sl + 31) >> 5 : 0);
  int64_t lb = lb_len;
  if (nw > 0) {
    const int32_t tmax = wave_max(need ? tl : 0);
    const bool pat_short = m <= nn;
    const uint64_t *ps = S.pat + (valid ? S.pat_off[p] : 0);
    const uint64_t *ts = S.txt + (valid ? S.txt_off[p] : 0);
    const int32_t lev = lev_dispatch<NWMAX>(nw, pat_short ? ps : ts, sl, pat_short ? ts : ps, tl, tmax, need);
    if (need) lb = max(lb, (int64_t)ce * lev + (diff ? o : 0));
  }
  const int32_t lb32 = (int32_t)min<int64_t>(lb, INT32_MAX);
  const bool ok = valid && (max_score < 0 || lb32 <= max_score);
  if (!LIST) {
    if (has) {
      lower[p] = valid ? lb32 : -1;
      pass[p] = ok ? 1 : 0;
    }
    return;
  }
  if (has && !ok) {
    O.score[p] = -1;
    O.status[p] = valid ? ST_REJECTED : ST_INVALID;
    O.nruns[p] = 0;
  }
  dev::wave_append(ok, (int32_t)p, list, count);
  const uint64_t rj = __ballot(has && valid && !ok);
  if (rj && (threadIdx.x & 63) == 0) atomicAdd(rejected, (int32_t)__popcll(rj));
}

template <int NWMAX>
hipError_t launch_nw(int64_t n, const Seqs &S, const int8_t *flags, int32_t x, int32_t o, int32_t e,
                     int32_t max_score, const int32_t *idx, int32_t *lower, int8_t *pass, const Outs *O,
                     int32_t *list, int32_t *count, int32_t *rejected, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256));
  if (O)
    hipLaunchKernelGGL((k_prefilter<NWMAX, true>), grid, dim3(256), 0, s, n, S, flags, x, o, e, max_score, idx,
                       lower, pass, *O, list, count, rejected);
  else
    hipLaunchKernelGGL((k_prefilter<NWMAX, false>), grid, dim3(256), 0, s, n, S, flags, x, o, e, max_score,
                       idx, lower, pass, Outs{}, list, count, rejected);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prefilter(int64_t n, const Seqs &S, const int8_t *flags, int32_t max_len, int32_t x, int32_t o,
                            int32_t e, int32_t max_score, const int32_t *idx, int32_t *lower, int8_t *pass,
                            const Outs *O, int32_t *list, int32_t *count, int32_t *rejected, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // the widest word count the batch can need picks the register budget: 8
  // words (256 bases) or 16 keep occupancy high for short reads
  if (max_len <= 256)
    return launch_nw<8>(n, S, flags, x, o, e, max_score, idx, lower, pass, O, list, count, rejected, s);
  if (max_len <= 512)
    return launch_nw<16>(n, S, flags, x, o, e, max_score, idx, lower, pass, O, list, count, rejected, s);
  return launch_nw<32>(n, S, flags, x, o, e, max_score, idx, lower, pass, O, list, count, rejected, s);
}

}  // namespace aim
