// Full-matrix DP for NW and SWG/Gotoh, one pair per workgroup: the plain
// baseline kernel, and the exact fallback for pairs no band can certify.
//
// Paper: System and Methods, "Needleman-Wunsch (NW)" and "Smith-Waterman-
// Gotoh (SWG)" -- the whole m x n table is filled and traced back (the
// WRAM+MRAM variant keeps the table off-chip and only the neighbouring cells
// on-chip; here the table of traceback codes lives in an HBM slot of the
// workgroup and the neighbouring cells travel through LDS).
//
// Fill: rows are processed in strips of NT rows, thread t owning row
// s0 + t + 1 and sweeping the columns with a skew of one column per thread, so
// at step tau thread t computes column tau - t + 1.  H and E of the row above
// come from thread t - 1 through a double-buffered LDS array (from the HBM row
// buffer for t = 0); the last row of a strip is written to that buffer for the
// next strip.  Each cell emits a 4-bit traceback code with the same meaning as
// the banded kernel's planes (bit 0: gap op in state H; bit 1: the gap is D;
// bit 2: an I run extends; bit 3: a D run extends).
//
// Traceback: the workgroup stages a 64-row x 64-column tile of codes in LDS
// around the walker, one lane walks inside it, and the tile moves when the
// walker leaves it.
#include "aim_internal.h"

namespace aim {
namespace {

constexpr int NT = 128;
constexpr int TR = 64, TC = 8;  // traceback tile: rows x 32-bit words (8 cells each)

__device__ __forceinline__ uint32_t base_at(const uint64_t *s, int64_t t) {
  return (uint32_t)(s[t >> 5] >> (2 * (t & 31))) & 3u;
}

template <bool AFF>
__global__ __launch_bounds__(NT) void k_full(Seqs S, Outs O, Scoring P, Work Wk,
                                            uint32_t *scratch_all, int64_t slot_words,
                                            int32_t max_len) {
  __shared__ int32_t sH[2][NT], sE[2][NT];
  __shared__ uint32_t tile[TR][TC];
  __shared__ int32_t sh_pair, sh_score;
  __shared__ int32_t sh_i, sh_j, sh_st, sh_nr, sh_done;
  __shared__ uint32_t sh_op, sh_len;

  const int t = threadIdx.x;
  const int32_t x = P.x, o = P.o, e = P.e, oe = P.o + P.e;
  int32_t *rowH = (int32_t *)(scratch_all + (int64_t)blockIdx.x * slot_words);
  int32_t *rowE = rowH + (max_len + 1);
  uint32_t *codes = (uint32_t *)(rowE + (max_len + 1));
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * 1 >= count) return;

  for (;;) {
    __syncthreads();
    if (t == 0) sh_pair = atomicAdd(Wk.counter, 1);
    __syncthreads();
    const int64_t li = sh_pair;
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)Wk.idx[li] : li;
    if (!Wk.direct) {
      if (O.flags && O.flags[p]) {
        if (t == 0) { O.score[p] = -1; O.status[p] = ST_INVALID; O.nruns[p] = 0; }
        continue;
      }
    }
    const int32_t m = S.pat_len[p], n = S.txt_len[p];
    const int32_t d = n - m, ad = d < 0 ? -d : d;
    if (!Wk.direct && P.max_score >= 0 && (ad ? o + ad * e : 0) > P.max_score) {
      if (t == 0) { O.score[p] = -1; O.status[p] = ST_REJECTED; O.nruns[p] = 0; }
      continue;
    }
    const uint64_t *pat = S.pat + S.pat_off[p];
    const uint64_t *txt = S.txt + S.txt_off[p];
    const int64_t stride = (n + 7) >> 3;
    auto border = [&](int32_t k) -> int32_t { return k == 0 ? 0 : (AFF ? o + k * e : k * e); };

    // ---------------- fill ----------------
    for (int32_t j = t; j <= n; j += NT) {
      rowH[j] = border(j);
      rowE[j] = DP_INF;
    }
    if (t == 0) sh_score = (m == 0) ? border(n) : DP_INF;
    if (n == 0 && t == 0) sh_score = border(m);
    __syncthreads();
    for (int32_t s0 = 0; s0 < m && n > 0; s0 += NT) {
      const int32_t r = s0 + t + 1;
      const bool rowok = r <= m;
      const uint32_t pb = rowok ? base_at(pat, r - 1) : 0u;
      int32_t Hl = border(r), Fl = DP_INF, Hd = border(r - 1);
      uint32_t acc = 0;
      int64_t tq = -1;
      uint64_t tw = 0;
      const int32_t steps = n + NT - 1;
      for (int32_t tau = 0; tau < steps; ++tau) {
        const int32_t j = tau - t + 1;
        const int cur = tau & 1, prv = cur ^ 1;
        if (rowok && j >= 1 && j <= n) {
          int32_t Hu, Eu;
          if (t == 0) { Hu = rowH[j]; Eu = rowE[j]; }
          else { Hu = sH[prv][t - 1]; Eu = sE[prv][t - 1]; }
          if (((j - 1) >> 5) != tq) { tq = (j - 1) >> 5; tw = txt[tq]; }
          const uint32_t tbase = (uint32_t)(tw >> (2 * ((j - 1) & 31))) & 3u;
          const int32_t mmb = pb != tbase;
          const int32_t diag = Hd + mmb * x;
          uint32_t code;
          int32_t Hv, Ev, Fv;
          if (AFF) {
            const int32_t aE = Hu + oe, bE = Eu + e;
            Ev = min(aE, bE);
            const int32_t aF = Hl + oe, bF = Fl + e;
            Fv = min(aF, bF);
            const int32_t G = min(Ev, Fv);
            Hv = min(diag, G);
            code = (uint32_t)(G <= Hd + mmb * (x - 1)) | ((uint32_t)(Fv < Ev) << 1) |
                   ((uint32_t)(bE < aE) << 2) | ((uint32_t)(bF < aF) << 3);
          } else {
            const int32_t up = Hu + e, left = Hl + e;
            const int32_t G = min(up, left);
            Hv = min(diag, G);
            Ev = DP_INF;
            Fv = DP_INF;
            code = (uint32_t)(G <= Hd + mmb * (x - 1)) | ((uint32_t)(left < up) << 1);
          }
          sH[cur][t] = Hv;
          sE[cur][t] = Ev;
          if (t == NT - 1) { rowH[j] = Hv; rowE[j] = Ev; }
          if (P.want_cigar) {
            acc |= code << (4 * ((j - 1) & 7));
            if ((j & 7) == 0 || j == n) {
              codes[(int64_t)(r - 1) * stride + ((j - 1) >> 3)] = acc;
              acc = 0;
            }
          }
          if (r == m && j == n) sh_score = Hv;
          Hd = Hu;
          Hl = Hv;
          Fl = Fv;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const int32_t score = sh_score;
    bool accept;
    if (!Wk.direct) {
      accept = !(P.max_score >= 0 && score > P.max_score);
      if (t == 0) {
        O.score[p] = accept ? score : -1;
        O.status[p] = accept ? ST_ALIGNED : ST_REJECTED;
        O.nruns[p] = 0;
      }
    } else {
      accept = true;
    }
    if (!accept || !P.want_cigar) continue;

    // ---------------- traceback ----------------
    const int32_t total = Wk.direct ? O.nruns[p] : 0;
    uint32_t *dst = Wk.direct ? (O.cigar + O.cigar_off[p]) : nullptr;
    __shared__ long long sh_pbase;
    if (t == 0) {
      sh_i = m; sh_j = n; sh_st = 0; sh_nr = 0; sh_done = 0;
      sh_op = 0xffu; sh_len = 0; sh_pbase = -1;
    }
    for (;;) {
      __syncthreads();
      const int32_t i0 = sh_i, j0 = sh_j;
      if (sh_done) break;
      const int32_t r_lo = max(1, i0 - TR + 1);
      const int32_t c_hi = (j0 - 1) >> 3;
      const int32_t c_lo = max(0, c_hi - TC + 1);
      if (i0 >= 1 && j0 >= 1) {
        for (int k = t; k < TR * TC; k += NT) {
          const int32_t rr = r_lo + k / TC, cc = c_lo + k % TC;
          if (rr <= i0 && cc <= c_hi) tile[k / TC][k % TC] = codes[(int64_t)(rr - 1) * stride + cc];
        }
      }
      __syncthreads();
      if (t == 0) {
        int32_t i = i0, j = j0, st = sh_st, nr = sh_nr;
        uint32_t cur_op = sh_op, cur_len = sh_len;
        RunSink sink;
        sink.begin(O, p);
        sink.pbase = sh_pbase;
        auto put = [&](uint32_t op, uint32_t len) {
          if (op == cur_op) {
            cur_len += len;
          } else {
            if (cur_len) {
              const uint32_t run = (cur_len << 4) | cur_op;
              if (Wk.direct) { if (nr < total) dst[total - 1 - nr] = run; }
              else sink.put(nr, run, (int64_t)i + j + 1);
              ++nr;
            }
            cur_op = op;
            cur_len = len;
          }
        };
        int64_t pq = -1, tq = -1;
        uint64_t pw = 0, tw = 0;
        while (i >= 1 && j >= 1 && i >= r_lo && ((j - 1) >> 3) >= c_lo) {
          const uint32_t code = (tile[i - r_lo][((j - 1) >> 3) - c_lo] >> (4 * ((j - 1) & 7))) & 15u;
          if (st == 0) {
            if (!(code & 1u)) {
              if (((i - 1) >> 5) != pq) { pq = (i - 1) >> 5; pw = pat[pq]; }
              if (((j - 1) >> 5) != tq) { tq = (j - 1) >> 5; tw = txt[tq]; }
              const uint32_t a = (uint32_t)(pw >> (2 * ((i - 1) & 31))) & 3u;
              const uint32_t c = (uint32_t)(tw >> (2 * ((j - 1) & 31))) & 3u;
              put(a == c ? OP_EQ : OP_X, 1);
              --i;
              --j;
            } else if (!AFF) {
              if (code & 2u) { put(OP_D, 1); --j; }
              else { put(OP_I, 1); --i; }
            } else {
              st = (code & 2u) ? 2 : 1;
            }
          } else if (st == 1) {
            put(OP_I, 1);
            st = (code & 4u) ? 1 : 0;
            --i;
          } else {
            put(OP_D, 1);
            st = (code & 8u) ? 2 : 0;
            --j;
          }
        }
        if (i == 0 || j == 0) {
          if (i > 0) put(OP_I, (uint32_t)i);
          if (j > 0) put(OP_D, (uint32_t)j);
          put(0xfu, 0);
          i = 0;
          j = 0;
          sh_done = 1;
          if (!Wk.direct) {
            sink.finish();
            O.nruns[p] = nr;
          }
        }
        sh_i = i; sh_j = j; sh_st = st; sh_nr = nr; sh_op = cur_op; sh_len = cur_len;
        sh_pbase = sink.pbase;
      }
    }
  }
}

}  // namespace

int64_t full_slot_words(int32_t max_len) {
  const int64_t L = max_len;
  return 2 * (L + 1) + L * ((L + 7) / 8) + 64;
}

hipError_t launch_full(bool affine, const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                       uint32_t *scratch, int64_t slot_words, int32_t max_len, int32_t nslots,
                       hipStream_t s) {
  const int32_t L = max_len;
  dim3 grid(nslots), block(NT);
  if (affine)
    hipLaunchKernelGGL((k_full<true>), grid, block, 0, s, S, O, P, Wk, scratch, slot_words, L);
  else
    hipLaunchKernelGGL((k_full<false>), grid, block, 0, s, S, O, P, Wk, scratch, slot_words, L);
  return hipGetLastError();
}

}  // namespace aim
