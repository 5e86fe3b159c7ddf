// Banded dynamic programming for NW (linear gaps) and SWG/Gotoh (affine
// gaps), one pair per GPU lane.
//
// Paper: System and Methods, "Needleman-Wunsch (NW)" and "Smith-Waterman-
// Gotoh (SWG)": the DP recurrences over an m x n table, with the traceback
// that turns the table into alignment operations.  On UPMEM each DPU thread
// owns one pair and walks its table in WRAM or MRAM; here each lane of a
// 64-wide wavefront owns one pair and keeps a band of W diagonals of the table
// in registers, row by row.
//
// Band and exactness.  Diagonal k = j - i.  The lane computes the band
// [kmin, kmin + W - 1], chosen to contain diagonals 0 and d = n - m, with every
// cell outside treated as +inf, so it obtains the best cost U over alignments
// that stay inside the band.  Any alignment that touches diagonal kmax + 1 must
// go up from 0 with a D run and come back to d with an I run, so it costs at
// least 2 o + e ((kmax + 1) + (kmax + 1 - d)); symmetrically below the band.
// Call the smaller of the two LB.  If U < LB every optimal alignment lies in
// the band, U is the optimum, and the traceback over the band's cells visits
// exactly the cells and tie decisions of the full-matrix traceback.  If U >= LB
// and the threshold is below LB the pair is rejected; otherwise the pair is
// escalated to a wider band or to the full-matrix kernel.
//
// Registers hold Hs = H + o + e per band cell (linear NW: H + g): that sum is
// both the gap-opening source of E in the next row and of F in the next cell,
// so one add serves both.
//
// Traceback bits per cell, each the sign bit of a difference shifted into a
// 32-bit word with one funnel shift (cell c of a word ends at bit 31 - c):
//   plane 0: the diagonal op (X or '=') is taken in state H, i.e.
//            H(i-1,j-1) + (mismatch ? x - 1 : 0) < min(E, F); this single
//            comparison encodes the canonical order X, I, D, '=' (a gap beats
//            '=' on ties, X beats a gap on ties).
//   plane 1: the gap op is D (F strictly below E), else I.
//   plane 2: (affine) E extends strictly better than it opens, so an I run
//            continues upward; ties close the run (canonical order).
//   plane 3: (affine) the same for F and D runs.
// Linear NW uses planes 0 and 1 with up = H(i-1,j) + g, left = H(i,j-1) + g.
// The rows of bits live in a per-wavefront scratch slot in HBM, lane
// interleaved so each row store is one coalesced 256-byte write.
#include "aim_internal.h"

namespace aim {
namespace {

constexpr uint64_t K55 = 0x5555555555555555ull;

__device__ __forceinline__ uint64_t ld_word(const uint64_t *s, int64_t nw, int64_t q) {
  return (q >= 0 && q < nw) ? s[q] : 0ull;
}

// 32 bases starting at base index s0 (which may lie outside the sequence;
// missing words read as zero -- those cells are never used).
__device__ __forceinline__ uint64_t window32(const uint64_t *s, int64_t nw, int64_t s0) {
  int64_t q = s0 >> 5;
  uint32_t r = (uint32_t)(s0 & 31);
  uint64_t w0 = ld_word(s, nw, q), w1 = ld_word(s, nw, q + 1);
  return r ? ((w0 >> (2 * r)) | (w1 << (64 - 2 * r))) : w0;
}

__device__ __forceinline__ uint32_t base_at(const uint64_t *s, int64_t t) {
  return (uint32_t)(s[t >> 5] >> (2 * (t & 31))) & 3u;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s));
  return v;
}

// Append the calling lanes with `pred` to a device list, one atomic per wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t value, int32_t *list, int32_t *count) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  int lane = threadIdx.x & 63;
  int leader = __ffsll((unsigned long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, (int)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) {
    int rank = __popcll(mask & ((1ull << lane) - 1ull));
    list[base + rank] = value;
  }
}

template <int W, bool AFF>
__global__ __launch_bounds__(64) void k_band(Seqs S, Outs O, Scoring P, Work Wk, uint32_t *tb_all,
                                            int64_t tb_slot_words, int32_t rows_cap) {
  constexpr int NH = W / 32;       // 32-bit words per plane per row
  constexpr int NP = AFF ? 4 : 2;  // planes
  const int lane = threadIdx.x;
  uint32_t *tb = tb_all + (int64_t)blockIdx.x * tb_slot_words;
  const int32_t x = P.x, o = P.o, e = P.e, oe = P.o + P.e;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * 64 >= count) return;

  for (;;) {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(Wk.counter, 1);
    chunk = __shfl(chunk, 0);
    if ((int64_t)chunk * 64 >= count) break;
    const int64_t li = (int64_t)chunk * 64 + lane;
    bool has = li < count;
    int64_t p = has ? (Wk.idx ? (int64_t)Wk.idx[li] : li) : 0;

    int32_t m = 0, n = 0, kmin = 0;
    bool run = false, escalate = false;
    if (has) {
      if (O.flags && O.flags[p]) {
        O.score[p] = -1;
        O.status[p] = ST_INVALID;
        O.nruns[p] = 0;
        has = false;
      } else {
        m = S.pat_len[p];
        n = S.txt_len[p];
        const int32_t d = n - m, ad = d < 0 ? -d : d;
        const int32_t lb_any = ad ? o + ad * e : 0;
        if (P.max_score >= 0 && lb_any > P.max_score) {
          O.score[p] = -1;
          O.status[p] = ST_REJECTED;
          O.nruns[p] = 0;
          has = false;
        } else if (ad > W - 1 || m > rows_cap - 1) {
          escalate = true;
          has = false;
        } else {
          run = true;
          kmin = min(0, d) - (W - 1 - ad) / 2;
        }
      }
    }
    if (Wk.next_idx) wave_append(escalate, (int32_t)p, Wk.next_idx, Wk.next_count);

    const int Mmax = wave_max(run ? m : 0);
    const uint64_t *pat = S.pat + (run ? S.pat_off[p] : 0);
    const uint64_t *txt = S.txt + (run ? S.txt_off[p] : 0);
    const int64_t pnw = run ? (m + 31) >> 5 : 0, tnw = run ? (n + 31) >> 5 : 0;
    const int32_t bstar = n - m - kmin;

    // Hs[b] = H + oe (affine) or H + g (linear) of band cell b in the current row
    const int32_t hoff = AFF ? oe : e;
    int32_t Hs[W], E[W];
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int32_t j = kmin + b;
      Hs[b] = (j < 0 ? DP_INF : (j == 0 ? 0 : (AFF ? o + j * e : j * e))) + hoff;
      E[b] = DP_INF;
    }
    int32_t score = DP_INF;
    if (run && m == 0) {
#pragma unroll
      for (int b = 0; b < W; ++b)
        if (b == bstar) score = Hs[b] - hoff;
    }

    uint64_t pword = 0;
    for (int i = 1; i <= Mmax; ++i) {
      if (((i - 1) & 31) == 0) pword = run ? ld_word(pat, pnw, (i - 1) >> 5) : 0ull;
      const uint64_t prep = (uint64_t)((uint32_t)(pword >> (2 * ((i - 1) & 31))) & 3u) * K55;
      uint32_t mmw[2 * NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const uint64_t X = window32(txt, tnw, (int64_t)i + kmin - 1 + 32 * h) ^ prep;
        const uint64_t mm = (X | (X >> 1)) & K55;
        mmw[2 * h] = (uint32_t)mm;
        mmw[2 * h + 1] = (uint32_t)(mm >> 32);
      }
      uint32_t bits[NP][NH];
#pragma unroll
      for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int h = 0; h < NH; ++h) bits[q][h] = 0u;
      int32_t Hsl = DP_INF + hoff, Fl = DP_INF;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const int32_t Hsd = Hs[b];                              // H(i-1,j-1) + hoff
        const int32_t Hsu = (b + 1 < W) ? Hs[b + 1] : DP_INF;   // H(i-1,j) + hoff
        const uint32_t mmb = (mmw[b >> 4] >> (2 * (b & 15))) & 1u;
        const int h = b >> 5;
        if (AFF) {
          const int32_t Eu = (b + 1 < W) ? E[b + 1] : DP_INF;
          const int32_t bE = Eu + e, Ev = min(Hsu, bE);         // E(i,j)
          const int32_t bF = Fl + e, Fv = min(Hsl, bF);         // F(i,j)
          const int32_t G = min(Ev, Fv);
          const int32_t Gs = G + oe;
          const int32_t Hsv = min((int32_t)__umul24(mmb, (uint32_t)x) + Hsd, Gs);
          const int32_t dg = (int32_t)__umul24(mmb, (uint32_t)(x - 1)) + Hsd;
          bits[0][h] = __builtin_amdgcn_alignbit(bits[0][h], (uint32_t)(dg - Gs), 31);
          bits[1][h] = __builtin_amdgcn_alignbit(bits[1][h], (uint32_t)(Fv - Ev), 31);
          bits[2][h] = __builtin_amdgcn_alignbit(bits[2][h], (uint32_t)(bE - Hsu), 31);
          bits[3][h] = __builtin_amdgcn_alignbit(bits[3][h], (uint32_t)(bF - Hsl), 31);
          Hs[b] = Hsv;
          E[b] = Ev;
          Hsl = Hsv;
          Fl = Fv;
        } else {
          const int32_t G = min(Hsu, Hsl);                      // min(up, left) + g
          const int32_t Gs = G + e;
          const int32_t Hsv = min((int32_t)__umul24(mmb, (uint32_t)x) + Hsd, Gs);
          const int32_t dg = (int32_t)__umul24(mmb, (uint32_t)(x - 1)) + Hsd;
          bits[0][h] = __builtin_amdgcn_alignbit(bits[0][h], (uint32_t)(dg - Gs), 31);
          bits[1][h] = __builtin_amdgcn_alignbit(bits[1][h], (uint32_t)(Hsl - Hsu), 31);
          Hs[b] = Hsv;
          Hsl = Hsv;
        }
        // Materialise this cell's bits now.  Without it the compiler sinks
        // the bit packing towards the row's stores and keeps every cell's
        // intermediates alive across the row.  The empty asm emits nothing.
#pragma unroll
        for (int q = 0; q < NP; ++q) asm volatile("" : "+v"(bits[q][h]));
      }
      if (P.want_cigar) {
        uint32_t *row = tb + ((int64_t)i * NP * NH) * 64 + lane;
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
          for (int h = 0; h < NH; ++h) row[(q * NH + h) * 64] = bits[q][h];
      }
      if (__ballot(run && i == m)) {
        if (run && i == m) {
#pragma unroll
          for (int b = 0; b < W; ++b)
            if (b == bstar) score = Hs[b] - hoff;
        }
      }
    }

    // decide: exact / rejected / escalate
    bool accept = false;
    if (run) {
      const int32_t d = n - m, kmax = kmin + W - 1;
      const int32_t lb_up = kmax + 1 > n ? DP_INF : 2 * o + e * (2 * (kmax + 1) - d);
      const int32_t lb_lo = kmin - 1 < -m ? DP_INF : 2 * o + e * (2 * (1 - kmin) + d);
      const int32_t LB = min(lb_up, lb_lo);
      if (score < LB) {
        if (P.max_score >= 0 && score > P.max_score) {
          O.score[p] = -1;
          O.status[p] = ST_REJECTED;
          O.nruns[p] = 0;
        } else {
          accept = true;
          O.score[p] = score;
          O.status[p] = ST_ALIGNED;
        }
      } else if (P.max_score >= 0 && LB > P.max_score) {
        O.score[p] = -1;
        O.status[p] = ST_REJECTED;
        O.nruns[p] = 0;
      } else {
        escalate = true;
      }
    }
    if (Wk.next_idx) wave_append(run && escalate, (int32_t)p, Wk.next_idx, Wk.next_count);

    if (!P.want_cigar) {
      if (accept) O.nruns[p] = 0;
      continue;
    }
    // ---- traceback (per lane, over this wavefront's scratch rows) ----
    if (accept) {
      int32_t i = m, j = n, b = bstar, st = 0;  // st: 0 H, 1 E (I run), 2 F (D run)
      uint32_t cur_op = 0xffu, cur_len = 0;
      int32_t nr = 0;
      RunSink sink;
      sink.begin(O, p);
      int64_t pq = -1, tq = -1;
      uint64_t pw = 0, tw = 0;
      int32_t rowi = -1;
      uint32_t rw[NP][NH];
      auto put = [&](uint32_t op, uint32_t len) {
        if (op == cur_op) {
          cur_len += len;
        } else {
          if (cur_len) {
            sink.put(nr, (cur_len << 4) | cur_op, (int64_t)i + j + 1);
            ++nr;
          }
          cur_op = op;
          cur_len = len;
        }
      };
      while (i > 0 && j > 0) {
        if (rowi != i) {
          const uint32_t *row = tb + ((int64_t)i * NP * NH) * 64 + lane;
#pragma unroll
          for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int h = 0; h < NH; ++h) rw[q][h] = row[(q * NH + h) * 64];
          rowi = i;
        }
        uint32_t bq[NP];
        const int hsel = b >> 5;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          uint32_t w = rw[q][0];
#pragma unroll
          for (int h = 1; h < NH; ++h) w = hsel == h ? rw[q][h] : w;
          bq[q] = (w >> (31 - (b & 31))) & 1u;
        }
        if (st == 0) {
          if (bq[0]) {
            if (((i - 1) >> 5) != pq) { pq = (i - 1) >> 5; pw = pat[pq]; }
            if (((j - 1) >> 5) != tq) { tq = (j - 1) >> 5; tw = txt[tq]; }
            const uint32_t pb = (uint32_t)(pw >> (2 * ((i - 1) & 31))) & 3u;
            const uint32_t tbase = (uint32_t)(tw >> (2 * ((j - 1) & 31))) & 3u;
            put(pb == tbase ? OP_EQ : OP_X, 1);
            --i;
            --j;
          } else {
            st = bq[1] ? 2 : 1;
            if (!AFF) {
              if (st == 1) { put(OP_I, 1); --i; ++b; }
              else { put(OP_D, 1); --j; --b; }
              st = 0;
            }
          }
        } else if (st == 1) {
          put(OP_I, 1);
          st = bq[2] ? 1 : 0;
          --i;
          ++b;
        } else {
          put(OP_D, 1);
          st = bq[3] ? 2 : 0;
          --j;
          --b;
        }
      }
      if (i > 0) put(OP_I, (uint32_t)i);
      if (j > 0) put(OP_D, (uint32_t)j);
      put(0xfu, 0);  // flush the last run
      sink.finish();
      O.nruns[p] = nr;
    }
  }
}

}  // namespace

int64_t band_tb_slot_words(int W, bool affine, int32_t rows_cap) {
  return (int64_t)rows_cap * (affine ? 4 : 2) * (W / 32) * 64;
}

hipError_t launch_band(int W, bool affine, const Seqs &S, const Outs &O, const Scoring &P,
                       const Work &Wk, uint32_t *tb, int64_t tb_slot_words, int32_t rows_cap,
                       int32_t nslots, hipStream_t s) {
  dim3 grid(nslots), block(64);
  if (W == 32 && affine)
    hipLaunchKernelGGL((k_band<32, true>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else if (W == 32)
    hipLaunchKernelGGL((k_band<32, false>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else if (W == 64 && affine)
    hipLaunchKernelGGL((k_band<64, true>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else if (W == 64)
    hipLaunchKernelGGL((k_band<64, false>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace aim
