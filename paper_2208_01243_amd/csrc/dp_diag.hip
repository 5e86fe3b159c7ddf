// Banded NW / SWG-Gotoh with one pair per 32 lanes, the lanes laid along the
// anti-diagonal (the escalation tier for pairs the 32-diagonal band could not
// decide).
//
// The recurrences, boundary conditions, exactness certificate and traceback
// order are those of the other band kernels (System and Methods: NW and SWG);
// only the order of evaluation differs.  The band holds W = 64 diagonals
// [kmin, kmin + 63] with kmin even.  Lane l of a pair owns diagonals
// k0 = kmin + 2l and k1 = k0 + 1.  A cell (i, j) lies on anti-diagonal
// t = i + j; diagonals of t's parity are computed at step t, so each lane
// computes exactly one cell per step and the whole band advances one
// anti-diagonal per step.  Iteration tau does t = 2 tau (slot 0, cell
// (tau - k0/2, tau + k0/2)) then t = 2 tau + 1 (slot 1, the cell one column
// to the right).  The three predecessors of a cell are the lane's own
// registers or the neighbour lane's value from the step before, moved with
// one DPP wave shift.  A pair therefore takes m + n steps instead of the m
// rows x W cells a lane spends on it in the row-wise kernels, which keeps the
// latency of the few escalated pairs short.
//
// Traceback bits (the four planes of the band kernels: diagonal taken, D over
// I, E extends, F extends; linear NW the first two) are funnel-shifted per
// iteration into one word per (slot, plane) and stored every 32 iterations:
// iteration tau, slot s, plane q of lane l at bit 31 - (tau & 31) of word
// ((tau >> 5) * 2 * planes + s * planes + q) * 64 + lane of the chunk's
// region (a chunk is the two pairs a wavefront takes).  Accepted pairs are
// marked with nruns = DIAG_MARK (-2) and walked by k_diag_tb, one pair per
// lane.  The mark differs from the first tier's (-1): that tier's walk runs on
// another stream at the same time and scans all pairs, so it must never take
// a pair of this tier for one of its own.
#include "aim_internal.h"
#include "dev_util.h"

namespace aim {
namespace {

constexpr int LPP = 32;       // lanes per pair
constexpr int W = 2 * LPP;    // diagonals
constexpr int G = 64 / LPP;   // pairs per wavefront
constexpr int32_t DIAG_MARK = -2;  // nruns of an accepted pair awaiting its walk

__device__ __forceinline__ int32_t shr1(int32_t v, int32_t edge) {  // lane l gets lane l-1
  return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int32_t shl1(int32_t v, int32_t edge) {  // lane l gets lane l+1
  return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xF, 0xF, false);
}

// kmin of the 64-diagonal band: even, <= min(0, d), with kmin + 63 >= max(0, d)
// (needs |d| <= W - 2).
__device__ __forceinline__ int32_t diag_kmin(int32_t m, int32_t n) {
  const int32_t d = n - m, ad = d < 0 ? -d : d;
  const int32_t base = min(0, d) - (W - 1 - ad) / 2;
  return base - (base & 1);
}

template <bool AFF>
__global__ __launch_bounds__(64) void k_diag(Seqs S, Outs O, Scoring P, Work Wk, uint32_t *tb_all,
                                            int64_t chunk_words, int64_t chunks_cap) {
  constexpr int NP = AFF ? 4 : 2;
  constexpr int NS = 2 * NP;  // words per lane per 32 iterations
  const int lane = threadIdx.x, grp = lane / LPP, l = lane % LPP;
  const int32_t x = P.x, o = P.o, e = P.e, oe = P.o + P.e;
  const int32_t hoff = AFF ? oe : e;
  const int32_t INF = DP_INF;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * G >= count) return;

  for (;;) {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(Wk.counter, 1);
    chunk = __shfl(chunk, 0);
    if ((int64_t)chunk * G >= count) break;
    const int64_t li = (int64_t)chunk * G + grp;
    bool has = li < count;
    const int64_t p = has ? (Wk.idx ? (int64_t)Wk.idx[li] : li) : 0;
    int32_t m = 0, n = 0, kmin = 0;
    bool run = false, escalate = false;
    if (has) {
      if (O.flags && O.flags[p]) {
        if (l == 0) {
          O.score[p] = -1;
          O.status[p] = ST_INVALID;
          O.nruns[p] = 0;
        }
      } else {
        m = S.pat_len[p];
        n = S.txt_len[p];
        const int32_t d = n - m, ad = d < 0 ? -d : d;
        const int32_t lb_any = ad ? o + ad * e : 0;
        if (P.max_score >= 0 && lb_any > P.max_score) {
          if (l == 0) {
            O.score[p] = -1;
            O.status[p] = ST_REJECTED;
            O.nruns[p] = 0;
          }
        } else if (ad > W - 2 || (P.want_cigar && chunk >= chunks_cap)) {
          escalate = true;
          if (l == 0) O.nruns[p] = 0;  // the walk must not take a stale mark for its own
        } else {
          run = true;
          kmin = diag_kmin(m, n);
        }
      }
    }
    if (Wk.next_idx) dev::wave_append(escalate && l == 0, (int32_t)p, Wk.next_idx, Wk.next_count);

    const int32_t k0 = kmin + 2 * l, hk = k0 / 2;  // k0 even
    const int32_t T = run ? (m + n + 1) / 2 : 0;   // last iteration needed
    const int32_t Tw = dev::wave_max(T);
    // the cell (m, n): diagonal d, slot (d - kmin) & 1, iteration (m + n - slot) / 2
    const int32_t bd = n - m - kmin;
    const bool own = run && l == (bd >> 1);
    const int32_t sstar = bd & 1, tstar = (m + n - sstar) / 2;
    const uint64_t *pat = S.pat + (run ? S.pat_off[p] : 0);
    const uint64_t *txt = S.txt + (run ? S.txt_off[p] : 0);
    const int64_t pnw = run ? (m + 31) >> 5 : 0, tnw = run ? (n + 31) >> 5 : 0;
    uint32_t *tb = tb_all + (int64_t)chunk * chunk_words + lane;
    // Left / upper band edges (lane 0's left, lane LPP-1's upper neighbour)
    // read as +inf.  The shifts run with every lane active (a DPP read from a
    // lane the EXEC mask switched off yields the edge value, not the lane's
    // data), so the edge is applied to the value a lane sends: with two pairs
    // per wavefront the last lane of a pair sends +inf to the first lane of
    // the next on a right shift, and the first lane sends +inf to the last
    // lane of the previous pair on a left shift.
    const bool first = l == 0, last = l == LPP - 1;

    int32_t H0 = INF, E0 = INF, F0 = INF, H1 = INF, E1 = INF, F1 = INF;  // Hs = H + hoff
    int32_t score = INF;
    // sequence windows: pattern base i-1 at bits 0-1 of pw; text bases j-1,
    // j at bits 0-3 of tw (i = tau - hk, j = tau + hk); both advance one base
    // per iteration and are reloaded every 16 iterations from words fetched
    // one period ahead
    uint64_t pw = dev::window32(pat, pnw, (int64_t)(0 - hk) - 1);
    uint64_t tw = dev::window32(txt, tnw, (int64_t)(0 + hk) - 1);
    uint64_t pw_n = dev::window32(pat, pnw, (int64_t)(16 - hk) - 1);
    uint64_t tw_n = dev::window32(txt, tnw, (int64_t)(16 + hk) - 1);
    uint32_t acc[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = 0u;

    for (int32_t tau = 0; tau <= Tw; ++tau) {
      if (tau > 0 && (tau & 15) == 0) {
        pw = pw_n;
        tw = tw_n;
        pw_n = dev::window32(pat, pnw, (int64_t)(tau + 16 - hk) - 1);
        tw_n = dev::window32(txt, tnw, (int64_t)(tau + 16 + hk) - 1);
      }
      const int32_t i = tau - hk, j = tau + hk;
      const uint32_t pb = (uint32_t)pw & 3u, tb0 = (uint32_t)tw & 3u, tb1 = (uint32_t)(tw >> 2) & 3u;
      pw >>= 2;
      tw >>= 2;
      // ---- slot 0: cell (i, j) on diagonal k0 ----
      {
        const int32_t Hsd = H0, Hsu = H1, Eu = E1;
        const int32_t Hsl = shr1(last ? INF : H1, INF);
        const int32_t Fl = shr1(last ? INF : F1, INF);
        const int32_t mm = pb != tb0;
        int32_t Hsv, Ev, Fv, d0, d1, d2, d3;
        if (AFF) {
          const int32_t bE = Eu + e, bF = Fl + e;
          Ev = min(Hsu, bE);
          Fv = min(Hsl, bF);
          const int32_t Gs = min(Ev, Fv) + oe;
          Hsv = min(Hsd + (mm ? x : 0), Gs);
          d0 = Hsd + (mm ? x - 1 : 0) - Gs;
          d1 = Fv - Ev;
          d2 = bE - Hsu;
          d3 = bF - Hsl;
        } else {
          const int32_t Gs = min(Hsu, Hsl) + e;
          Hsv = min(Hsd + (mm ? x : 0), Gs);
          Ev = Fv = INF;
          d0 = Hsd + (mm ? x - 1 : 0) - Gs;
          d1 = Hsl - Hsu;
          d2 = d3 = 0;
        }
        if (i < 0 || j < 0) {
          Hsv = Ev = Fv = INF;
        } else if (i == 0) {
          Hsv = (j == 0 ? 0 : (AFF ? o + j * e : j * e)) + hoff;
          Ev = Fv = INF;
        }
        H0 = Hsv;
        E0 = Ev;
        F0 = Fv;
        acc[0] = __builtin_amdgcn_alignbit(acc[0], (uint32_t)d0, 31);
        acc[1] = __builtin_amdgcn_alignbit(acc[1], (uint32_t)d1, 31);
        if (AFF) {
          acc[2] = __builtin_amdgcn_alignbit(acc[2], (uint32_t)d2, 31);
          acc[3] = __builtin_amdgcn_alignbit(acc[3], (uint32_t)d3, 31);
        }
      }
      // ---- slot 1: cell (i, j + 1) on diagonal k0 + 1 ----
      {
        const int32_t Hsd = H1, Hsl = H0, Fl = F0;
        const int32_t Hsu = shl1(first ? INF : H0, INF);
        const int32_t Eu = shl1(first ? INF : E0, INF);
        const int32_t mm = pb != tb1;
        const int32_t jj = j + 1;
        int32_t Hsv, Ev, Fv, d0, d1, d2, d3;
        if (AFF) {
          const int32_t bE = Eu + e, bF = Fl + e;
          Ev = min(Hsu, bE);
          Fv = min(Hsl, bF);
          const int32_t Gs = min(Ev, Fv) + oe;
          Hsv = min(Hsd + (mm ? x : 0), Gs);
          d0 = Hsd + (mm ? x - 1 : 0) - Gs;
          d1 = Fv - Ev;
          d2 = bE - Hsu;
          d3 = bF - Hsl;
        } else {
          const int32_t Gs = min(Hsu, Hsl) + e;
          Hsv = min(Hsd + (mm ? x : 0), Gs);
          Ev = Fv = INF;
          d0 = Hsd + (mm ? x - 1 : 0) - Gs;
          d1 = Hsl - Hsu;
          d2 = d3 = 0;
        }
        if (i < 0 || jj < 0) {
          Hsv = Ev = Fv = INF;
        } else if (i == 0) {
          Hsv = (jj == 0 ? 0 : (AFF ? o + jj * e : jj * e)) + hoff;
          Ev = Fv = INF;
        }
        H1 = Hsv;
        E1 = Ev;
        F1 = Fv;
        acc[NP + 0] = __builtin_amdgcn_alignbit(acc[NP + 0], (uint32_t)d0, 31);
        acc[NP + 1] = __builtin_amdgcn_alignbit(acc[NP + 1], (uint32_t)d1, 31);
        if (AFF) {
          acc[NP + 2] = __builtin_amdgcn_alignbit(acc[NP + 2], (uint32_t)d2, 31);
          acc[NP + 3] = __builtin_amdgcn_alignbit(acc[NP + 3], (uint32_t)d3, 31);
        }
      }
      if (own && tau == tstar) score = (sstar ? H1 : H0) - hoff;
      if ((tau & 31) == 31 || tau == Tw) {
        if (P.want_cigar && chunk < chunks_cap) {
          const int sh = 31 - (tau & 31);  // pad a partial last word
          uint32_t *w = tb + (int64_t)(tau >> 5) * NS * 64;
#pragma unroll
          for (int q = 0; q < NS; ++q) w[q * 64] = acc[q] << sh;
        }
      }
    }

    // the lane that owns (m, n) holds the score; share it within the pair
    const int src = grp * LPP + ((run ? bd : 0) >> 1);
    score = __shfl(score, src);
    bool accept = false;
    if (run) {
      const int32_t d = n - m, kmax = kmin + W - 1;
      const int32_t lb_up = kmax + 1 > n ? DP_INF : 2 * o + e * (2 * (kmax + 1) - d);
      const int32_t lb_lo = kmin - 1 < -m ? DP_INF : 2 * o + e * (2 * (1 - kmin) + d);
      const int32_t LB = min(lb_up, lb_lo);
      if (score < LB) {
        if (P.max_score >= 0 && score > P.max_score) {
          if (l == 0) {
            O.score[p] = -1;
            O.status[p] = ST_REJECTED;
            O.nruns[p] = 0;
          }
        } else {
          accept = true;
          if (l == 0) {
            O.score[p] = score;
            O.status[p] = ST_ALIGNED;
            O.nruns[p] = P.want_cigar ? DIAG_MARK : 0;
          }
        }
      } else if (P.max_score >= 0 && LB > P.max_score) {
        if (l == 0) {
          O.score[p] = -1;
          O.status[p] = ST_REJECTED;
          O.nruns[p] = 0;
        }
      } else {
        escalate = true;
        if (l == 0) O.nruns[p] = 0;
      }
    }
    (void)accept;
    if (Wk.next_idx)
      dev::wave_append(run && escalate && l == 0, (int32_t)p, Wk.next_idx, Wk.next_count);
  }
}

// Walk of the pairs k_diag accepted: one pair per lane, TBP pairs per
// wavefront.  The walk visits 32-iteration blocks in decreasing order, so the
// wavefront stages one block of all its pairs' bits in LDS at a time (their
// words of lanes 32g .. 32g+31 of the chunk), with the sequence words the
// block can touch in registers, and every lane walks until its path leaves
// the block.  Each lane thus reads from LDS and registers only, and a global
// round trip is paid once per block rather than whenever some lane changes
// diagonal.
constexpr int TBP = 16;

template <bool AFF>
__global__ __launch_bounds__(64) void k_diag_tb(Seqs S, Outs O, Work Wk, const uint32_t *tb_all,
                                               int64_t chunk_words) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  constexpr int NP = AFF ? 4 : 2;
  constexpr int NS = 2 * NP;
  constexpr int QUADS = TBP * NS * LPP / 4;  // 16-byte pieces of one staged block
  // Each pair's pieces are followed by one quad of padding: a pair's block is
  // NS * LPP words, a multiple of the 32 LDS banks, so without it the pairs'
  // lanes reading the same word of their blocks all hit one bank; with it
  // consecutive pairs are 4 banks apart (at most two lanes share a bank).
  constexpr int PQ = NS * LPP / 4 + 1;  // quads per staged pair, padding included
  __shared__ u32x4 stage[TBP * PQ];
  const uint32_t *lds = reinterpret_cast<const uint32_t *>(stage);
  const int lane = threadIdx.x;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * TBP >= count) return;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(Wk.counter, 1);
    t = __shfl(t, 0);
    if ((int64_t)t * TBP >= count) break;
    const int64_t li = (int64_t)t * TBP + lane;
    bool act = false;
    int64_t p = 0;
    if (lane < TBP && li < count) {
      p = Wk.idx ? (int64_t)Wk.idx[li] : li;
      act = O.nruns[p] == DIAG_MARK;
    }
    // only accepted pairs have bits (their chunk lies below the capacity)
    const uint64_t actmask = __ballot(act);
    int32_t m = 0, n = 0, kmin = 0;
    const uint64_t *pat = S.pat, *txt = S.txt;
    if (act) {
      m = S.pat_len[p];
      n = S.txt_len[p];
      kmin = diag_kmin(m, n);
      pat += S.pat_off[p];
      txt += S.txt_off[p];
    }
    const int64_t pnw = act ? (m + 31) >> 5 : 0, tnw = act ? (n + 31) >> 5 : 0;
    // the walk touches iterations tau <= (m + n) / 2
    const int32_t btop = dev::wave_max(act ? ((m + n) >> 1) >> 5 : -1);

    int32_t i = m, j = n, st = 0;
    uint32_t cur_op = 0xffu, cur_len = 0;
    int32_t nr = 0;
    uint32_t *slot = O.slot + p * (int64_t)O.slot_cap;
    const int32_t cap = O.slot_cap;
    auto put = [&](uint32_t op, uint32_t len) {
      if (op != cur_op) {
        if (cur_len && nr < cap) slot[nr] = (cur_len << 4) | cur_op;
        nr += cur_len ? 1 : 0;
        cur_op = op;
        cur_len = 0;
      }
      cur_len += len;
    };
    // block beta's bits go through registers: the next block's loads are in
    // flight while the lanes walk this one (only active pairs' pieces)
    constexpr int PRE = QUADS / 64;
    u32x4 pre[PRE];
    auto fetch = [&](int32_t beta) {
#pragma unroll
      for (int k = 0; k < PRE; ++k) {
        const int q = lane + 64 * k;
        const int pi = q / (NS * LPP / 4), stream = (q / (LPP / 4)) % NS, quad = q % (LPP / 4);
        if ((actmask >> pi) & 1ull) {
          const int64_t lj = (int64_t)t * TBP + pi;
          const uint32_t *src = tb_all + (lj / G) * chunk_words + ((int64_t)beta * NS + stream) * 64 +
                                (lj % G) * LPP + quad * 4;
          pre[k] = *reinterpret_cast<const u32x4 *>(src);
        }
      }
    };
    if (btop >= 0) fetch(btop);
#pragma unroll 1
    for (int32_t beta = btop; beta >= 0; --beta) {
      // In block beta, i + j lies in [64 beta, 64 beta + 63] and j - i in
      // [kmin, kmin + 63], so base i-1 lies in 32 beta - (kmin + 65) / 2 ..
      // +64 and base j-1 in 32 beta + kmin / 2 - 1 .. +63; four words from
      // one below the first cover either range.  They are loaded before the
      // stage is written, so that the wait for the block's bits covers them
      // and no wait in the walk holds it for the next block's loads.
      const int64_t pq0 = ((int64_t)32 * beta - (kmin + 65) / 2 - 1) >> 5;
      const int64_t tq0 = ((int64_t)32 * beta + kmin / 2 - 2) >> 5;
      uint64_t pw[4], tw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pw[q] = dev::ld_word(pat, pnw, pq0 + q);
        tw[q] = dev::ld_word(txt, tnw, tq0 + q);
      }
      // wait for them here (with the block's bits, loaded before them)
      asm volatile("" ::"v"(pw[0]), "v"(pw[1]), "v"(pw[2]), "v"(pw[3]), "v"(tw[0]), "v"(tw[1]), "v"(tw[2]),
                   "v"(tw[3]));
      __syncthreads();  // the previous block is no longer read
#pragma unroll
      for (int k = 0; k < PRE; ++k)
        if ((actmask >> ((lane + 64 * k) / (NS * LPP / 4))) & 1ull) {
          const int q = lane + 64 * k;
          stage[(q / (NS * LPP / 4)) * PQ + q % (NS * LPP / 4)] = pre[k];
        }
      __syncthreads();
      if (beta > 0) fetch(beta - 1);
      // keeps the compiler from sinking those loads below the walk (it emits
      // nothing and waits for nothing)
      asm volatile("" ::: "memory");
      while (act && i > 0 && j > 0) {
        const int32_t bb = j - i - kmin, ll = (bb >> 1) & (LPP - 1), s = bb & 1;
        const int32_t tau = (i + j - s) >> 1;
        if (tau < 32 * beta) break;
        const uint32_t *w = lds + lane * (PQ * 4) + s * NP * LPP + ll;
        const int sh = 31 - (tau & 31);
        const uint32_t bd = (w[0] >> sh) & 1u, b1 = (w[LPP] >> sh) & 1u;
        uint32_t b2 = 0, b3 = 0;
        if (AFF) {
          b2 = (w[2 * LPP] >> sh) & 1u;
          b3 = (w[3 * LPP] >> sh) & 1u;
        }
        const int32_t g = (st == 0 && !bd) ? (b1 ? 2 : 1) : st;  // 0 diag, 1 I, 2 D
        const int64_t pq = (int64_t)((i - 1) >> 5) - pq0, tq = (int64_t)((j - 1) >> 5) - tq0;
        const uint64_t pwd = pq == 0 ? pw[0] : pq == 1 ? pw[1] : pq == 2 ? pw[2] : pw[3];
        const uint64_t twd = tq == 0 ? tw[0] : tq == 1 ? tw[1] : tq == 2 ? tw[2] : tw[3];
        const uint32_t ca = (uint32_t)(pwd >> (2 * ((i - 1) & 31))) & 3u;
        const uint32_t cb = (uint32_t)(twd >> (2 * ((j - 1) & 31))) & 3u;
        const uint32_t op = g == 0 ? (ca == cb ? OP_EQ : OP_X) : (g == 1 ? OP_I : OP_D);
        put(op, 1);
        st = AFF ? (g == 1 ? (b2 ? 1 : 0) : (g == 2 ? (b3 ? 2 : 0) : 0)) : 0;
        i -= g != 2;
        j -= g != 1;
      }
    }
    if (act) {
      if (i > 0) put(OP_I, (uint32_t)i);
      if (j > 0) put(OP_D, (uint32_t)j);
      put(0xfu, 0);
      if (nr > cap) O.pool_off[p] = -2;  // re-run in place by the compaction
      O.nruns[p] = nr;
    }
  }
}

}  // namespace

int64_t diag_chunk_words(bool affine, int32_t max_len) {
  // iterations 0 .. max_len (T = ceil((m + n) / 2) <= max_len)
  const int64_t blocks = (int64_t)max_len / 32 + 1;
  return blocks * (affine ? 8 : 4) * 64;
}

hipError_t launch_diag(bool affine, const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                       uint32_t *tb, int64_t chunk_words, int64_t chunks_cap, int32_t nslots,
                       hipStream_t s) {
  dim3 grid(nslots), block(64);
  if (affine)
    hipLaunchKernelGGL((k_diag<true>), grid, block, 0, s, S, O, P, Wk, tb, chunk_words, chunks_cap);
  else
    hipLaunchKernelGGL((k_diag<false>), grid, block, 0, s, S, O, P, Wk, tb, chunk_words, chunks_cap);
  return hipGetLastError();
}

int32_t diag_tb_pairs_per_wave() { return TBP; }

hipError_t launch_diag_tb(bool affine, const Seqs &S, const Outs &O, const Work &Wk, const uint32_t *tb,
                          int64_t chunk_words, int32_t nslots, hipStream_t s) {
  dim3 grid(nslots), block(64);
  if (affine)
    hipLaunchKernelGGL((k_diag_tb<true>), grid, block, 0, s, S, O, Wk, tb, chunk_words);
  else
    hipLaunchKernelGGL((k_diag_tb<false>), grid, block, 0, s, S, O, Wk, tb, chunk_words);
  return hipGetLastError();
}

}  // namespace aim
