// Banded NW / SWG-Gotoh with packed 16-bit arithmetic: two pairs per lane.
//
// The same algorithm as the 32-diagonal band kernel (one pair per lane, band
// of W diagonals proven exact per pair, 2-4 traceback bit-planes per cell,
// canonical traceback), but each 32-bit register holds the cell of pair A in
// its low half and of pair B in its high half, so every packed instruction
// (v_pk_add_i16 with clamp, v_pk_min_i16, v_pk_sub_i16) advances two cells.
// Additions saturate at 32767, which plays the role of +infinity.  A pair
// takes this path only when every finite value of its band is provably below
// 32000: any band cell (i,j) is reached by one gap run and a diagonal walk, so
// H(i,j) <= x*max(m,n) + o + e*(m+n), and no register holds more than that
// plus 2 (o + e) + x (E, F and the diagonal candidate on top of H + o + e);
// pairs above the bound go to the 32-bit kernels.  Differences of two values
// in [0, 32767] never wrap, so the sign bit of each 16-bit difference is the
// traceback decision.  One byte permute gathers the sign bytes of two planes'
// differences (four bit streams: plane pair x pair A/B) into one word, and a
// shift plus a bit-field insert appends them to an accumulator, so after a
// group of 8 cells bit c of each byte is cell c of the group.
//
// Traceback words: row i, cell group g (cells 8g..8g+7), plane pair pp
// (planes 2pp and 2pp+1) at ((i * 2 * planes) + g * planes / 2 + pp) * 64 +
// lane; byte (q & 1) * 2 + h holds plane q of pair h (A = 0, B = 1).
#include "aim_internal.h"
#include "dev_util.h"

namespace aim {
namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int W = 32;
constexpr int32_t VMAX = 32000;
constexpr short INF16 = 32767;

__device__ __forceinline__ uint32_t U(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ s16x2 S(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ s16x2 adds(s16x2 a, s16x2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s16x2 mn(s16x2 a, s16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ s16x2 spl(int32_t v) { return (s16x2){(short)v, (short)v}; }
// a * b + c per half, saturated to the int16 range (v_pk_mad_i16 with clamp;
// the compiler does not form it from a multiply and a saturating add)
__device__ __forceinline__ s16x2 mad_sat(s16x2 a, s16x2 b, s16x2 c) {
  uint32_t r;
  asm("v_pk_mad_i16 %0, %1, %2, %3 clamp" : "=v"(r) : "v"(U(a)), "v"(U(b)), "v"(U(c)));
  return S(r);
}
// append the sign bits of the halves of d_lo (plane 2pp) and d_hi (plane
// 2pp+1) at bit 7 of the four bytes of acc, after shifting every byte right
// by one (the bit a byte takes from the byte above is overwritten)
__device__ __forceinline__ uint32_t push_signs(uint32_t acc, s16x2 d_lo, s16x2 d_hi) {
  const uint32_t sg = __builtin_amdgcn_perm(U(d_hi), U(d_lo), 0x07050301u);
  return (sg & 0x80808080u) | ((acc >> 1) & 0x7f7f7f7fu);
}

// Traceback of one pair (half h of its lane's packed words) over rows of
// bits staged in LDS, row r of a block at lds + r * 2 * planes * 64 words.
// The walk takes one op per step, chosen with selects: at a cell in state H
// either the diagonal, or (entering a gap) the gap run the D/I plane names,
// continued while the cell's extension plane says so.  Runs go to the pair's
// slot only; a pair with more runs than the slot holds is marked for the
// in-place re-run of the compaction (pool offset -2), which recomputes it.
template <bool AFF>
struct Walker16 {
  static constexpr int NP = AFF ? 4 : 2;
  int32_t i, j, b, st, nr, kmin;
  uint32_t cur_op, cur_len;
  uint32_t *slot;
  int32_t cap;

  __device__ void begin(const Outs &O, int64_t p, int32_t m, int32_t n, int32_t kmin_) {
    i = m;
    j = n;
    kmin = kmin_;
    b = n - m - kmin;
    st = 0;
    nr = 0;
    cur_op = 0xffu;
    cur_len = 0;
    slot = O.slot + p * (int64_t)O.slot_cap;
    cap = O.slot_cap;
  }
  __device__ void put(uint32_t op, uint32_t len) {
    if (op != cur_op) {
      if (cur_len && nr < cap) slot[nr] = (cur_len << 4) | cur_op;
      nr += cur_len ? 1 : 0;
      cur_op = op;
      cur_len = 0;
    }
    cur_len += len;
  }
  // 32 text bases from the one at ts + 32 tq0 on, ts = max(j - 1 - 32 tq0 -
  // 31, 0): with j - 1 >= 32 tq0 the window holds base j - 1 and the 31
  // below it, which the walk reaches before it needs another.
  __device__ void text_window(uint64_t tw0, uint64_t tw1, uint64_t tw2, int64_t tq0, uint64_t &win,
                              int32_t &base) {
    const int32_t ts = max((int32_t)((int64_t)(j - 1) - 32 * tq0) - 31, 0);  // 0 .. 38
    const uint64_t a = ts < 32 ? tw0 : tw1, c = ts < 32 ? tw1 : tw2;
    const uint32_t s2 = 2 * (ts & 31);
    win = s2 ? (a >> s2) | (c << (64 - s2)) : a;
    base = (int32_t)(32 * tq0) + ts;
  }
  // Steps while the path stays in rows lo+1 .. (the rows staged, at most 8).
  // Pattern bases lo .. lo+31 are in pw0/pw1 (words pq0, pq0+1); text bases
  // from lo+kmin on in tw0..tw2 (words tq0 ..).  Every step reads one cell's
  // bits (two words for four planes) and takes one op, with selects; the
  // bases it compares come from a 16-base pattern window of the block and a
  // 32-base text window below the walk's column.
  // Only the cell groups (8 band cells each) set in gmask are staged: a walk
  // that reaches another stops there and returns true.
  __device__ bool walk(const uint32_t *lds, int lane, int h, int32_t lo, uint64_t pw0, uint64_t pw1,
                       uint64_t tw0, uint64_t tw1, uint64_t tw2, int64_t pq0, int64_t tq0, uint32_t gmask) {
    if (i <= lo || j <= 0) return false;
    const uint32_t po = (uint32_t)(lo - 32 * pq0);  // 0 .. 31
    const uint32_t p0 = (uint32_t)pw0, p1 = (uint32_t)(pw0 >> 32), p2 = (uint32_t)pw1;
    // pattern base lo + r at bits 2r
    const uint32_t pwin = __builtin_amdgcn_alignbit(po < 16 ? p1 : p2, po < 16 ? p0 : p1, 2 * (po & 15));
    uint64_t twin;
    int32_t tbase;
    text_window(tw0, tw1, tw2, tq0, twin, tbase);
    do {
      if (!((gmask >> ((b >> 3) & 3)) & 1u)) return true;
      const int32_t r = i - lo - 1;
      const uint32_t *rw = lds + (r * NP * 2 + ((b >> 3) & 3) * (NP / 2)) * 64 + lane;
      uint32_t w01 = rw[0], w23 = AFF ? rw[64] : 0u;
      if (j - 1 < tbase) text_window(tw0, tw1, tw2, tq0, twin, tbase);
      uint32_t eq = (pwin >> (2 * r)) ^ (uint32_t)(twin >> (2 * (j - 1 - tbase)));
      // every lane computes every candidate: the empty asm statements keep the
      // compiler from turning the selects below into branches
      asm volatile("" : "+v"(w01), "+v"(w23), "+v"(eq));
      // plane q of pair h, band cell b: bit ((q & 1) * 2 + h) * 8 + (b & 7)
      // of the word of planes (q & ~1, q | 1)
      const uint32_t sh = (uint32_t)h * 8 + (b & 7);
      const uint32_t bd = (w01 >> sh) & 1u, b1 = (w01 >> (sh + 16)) & 1u;
      const int32_t g = st ? st : (int32_t)((bd ^ 1u) * (1u + b1));  // 0 diag, 1 I, 2 D
      // OP_EQ, OP_X on the diagonal; OP_I = 2 and OP_D = 3 are g + 1
      static_assert(OP_EQ == 0 && OP_X == 1 && OP_I == 2 && OP_D == 3, "op codes");
      const uint32_t op = g ? (uint32_t)g + 1u : (uint32_t)((eq & 3u) != 0);
      // runs: a new op closes the current run (kept if the slot has room)
      const bool close = op != cur_op && cur_len;
      if (close && nr < cap) slot[nr] = (cur_len << 4) | cur_op;
      nr += close ? 1 : 0;
      cur_len = op != cur_op ? 1u : cur_len + 1;
      cur_op = op;
      // a gap continues while its extension plane says so: plane 2 (bit sh)
      // for I, plane 3 (bit sh + 16) for D
      st = AFF ? g * (int32_t)((w23 >> (sh + 8 * (g & 2))) & 1u) : 0;
      i -= g != 2;
      j -= g != 1;
      b += g == 1 ? 1 : (g == 2 ? -1 : 0);
    } while (i > lo && j > 0);
    return false;
  }
  __device__ void finish(const Outs &O, int64_t p) {
    if (i > 0) put(OP_I, (uint32_t)i);
    if (j > 0) put(OP_D, (uint32_t)j);
    put(0xfu, 0);
    if (nr > cap) O.pool_off[p] = -2;
    O.nruns[p] = nr;
  }
};

// Rows walked per staged block by the fill kernel's own walk (8 KB of LDS
// for four affine planes).
constexpr int FUSED_ROWS = 4;

// SPLIT: the traceback bits of chunk c (128 pairs) go to a region of their
// own and the traceback runs in k_band16_tb; accepted pairs are marked with
// nruns = -1 until then.  Otherwise a wavefront reuses one slot and walks its
// pairs itself.
template <bool AFF, bool SPLIT>
__global__ __launch_bounds__(64, 3) void k_band16(Seqs Sq, Outs O, Scoring P, Work Wk, uint32_t *tb_all,
                                              int64_t tb_slot_words, int32_t rows_cap) {
  constexpr int NP = AFF ? 4 : 2;
  // rows staged for the traceback when the kernel walks its own pairs
  __shared__ u32x4 fused_stage[SPLIT ? 1 : FUSED_ROWS * NP * 2 * 64 / 4];
  const int lane = threadIdx.x;
  const int32_t x = P.x, o = P.o, e = P.e, oe = P.o + P.e;
  const int32_t hoff = AFF ? oe : e;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * 128 >= count) return;
  const s16x2 vx = spl(x), vxm1 = spl(x - 1), ve = spl(e), voe = spl(oe), vinf = spl(INF16);

  for (;;) {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(Wk.counter, 1);
    chunk = __shfl(chunk, 0);
    if ((int64_t)chunk * 128 >= count) break;
    uint32_t *tb = tb_all + (SPLIT ? (int64_t)chunk : (int64_t)blockIdx.x) * tb_slot_words;

    int64_t p[2];
    int32_t m[2], n[2], kmin[2], bstar[2];
    bool run[2], esc[2];
    const uint64_t *pat[2], *txt[2];
    int64_t pnw[2], tnw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t li = (int64_t)chunk * 128 + 64 * h + lane;
      bool has = li < count;
      p[h] = has ? (Wk.idx ? (int64_t)Wk.idx[li] : li) : 0;
      m[h] = n[h] = kmin[h] = 0;
      run[h] = esc[h] = false;
      if (has) {
        if (O.flags && O.flags[p[h]]) {
          O.score[p[h]] = -1;
          O.status[p[h]] = ST_INVALID;
          O.nruns[p[h]] = 0;
        } else {
          m[h] = Sq.pat_len[p[h]];
          n[h] = Sq.txt_len[p[h]];
          const int32_t d = n[h] - m[h], ad = d < 0 ? -d : d;
          const int32_t lb_any = ad ? o + ad * e : 0;
          // largest finite register value: H + 2 (o + e) + x (see the header)
          const int64_t vbound = (int64_t)x * max(m[h], n[h]) + 2 * (int64_t)o +
                                 (int64_t)e * (m[h] + n[h]) + 2 * (int64_t)hoff + 2 * (int64_t)x;
          if (P.max_score >= 0 && lb_any > P.max_score) {
            O.score[p[h]] = -1;
            O.status[p[h]] = ST_REJECTED;
            O.nruns[p[h]] = 0;
          } else if (ad > W - 1 || m[h] > rows_cap - 1 || vbound > VMAX) {
            esc[h] = true;
          } else {
            run[h] = true;
            kmin[h] = min(0, d) - (W - 1 - ad) / 2;
          }
        }
      }
      pat[h] = Sq.pat + (run[h] ? Sq.pat_off[p[h]] : 0);
      txt[h] = Sq.txt + (run[h] ? Sq.txt_off[p[h]] : 0);
      pnw[h] = run[h] ? (m[h] + 31) >> 5 : 0;
      tnw[h] = run[h] ? (n[h] + 31) >> 5 : 0;
      bstar[h] = n[h] - m[h] - kmin[h];
    }
    if (Wk.next_idx) {
      dev::wave_append(esc[0], (int32_t)p[0], Wk.next_idx, Wk.next_count);
      dev::wave_append(esc[1], (int32_t)p[1], Wk.next_idx, Wk.next_count);
    }
    const int Mmax = dev::wave_max(max(run[0] ? m[0] : 0, run[1] ? m[1] : 0));

    s16x2 Hs[W], E[W];
    auto border = [&](int32_t j) -> int32_t {
      return j < 0 ? INF16 : min((j == 0 ? 0 : (AFF ? o + j * e : j * e)) + hoff, (int32_t)INF16);
    };
#pragma unroll
    for (int b = 0; b < W; ++b) {
      Hs[b] = (s16x2){(short)border(kmin[0] + b), (short)border(kmin[1] + b)};
      E[b] = vinf;
    }
    int32_t score[2] = {DP_INF, DP_INF};
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (run[h] && m[h] == 0) {
#pragma unroll
        for (int b = 0; b < W; ++b)
          if (b == bstar[h]) score[h] = (h ? Hs[b].y : Hs[b].x) - hoff;
      }

    uint64_t pword[2] = {0, 0};
    for (int i = 1; i <= Mmax; ++i) {
      uint32_t mlo[2], mhi[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (((i - 1) & 31) == 0) pword[h] = run[h] ? dev::ld_word(pat[h], pnw[h], (i - 1) >> 5) : 0ull;
        const uint64_t prep = (uint64_t)((uint32_t)(pword[h] >> (2 * ((i - 1) & 31))) & 3u) * dev::K55;
        const uint64_t X = dev::window32(txt[h], tnw[h], (int64_t)i + kmin[h] - 1) ^ prep;
        const uint64_t mm = (X | (X >> 1)) & dev::K55;
        mlo[h] = (uint32_t)mm;
        mhi[h] = (uint32_t)(mm >> 32);
      }
      // packed mismatch bits, 8 cells per word: cell c of the group at bit 2c
      // of the low half (pair A) and of the high half (pair B)
      uint32_t X[4] = {(mlo[0] & 0xFFFFu) | (mlo[1] << 16), (mlo[0] >> 16) | (mlo[1] & 0xFFFF0000u),
                       (mhi[0] & 0xFFFFu) | (mhi[1] << 16), (mhi[0] >> 16) | (mhi[1] & 0xFFFF0000u)};
      uint32_t *row = tb + ((int64_t)i * NP * 2) * 64 + lane;
      s16x2 Hsl = vinf, Fl = vinf;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint32_t acc01 = 0u, acc23 = 0u;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int b = 8 * g + c;
          const s16x2 mmp = S((X[g] >> (2 * c)) & 0x00010001u);
          const s16x2 Hsd = Hs[b];
          const s16x2 Hsu = (b + 1 < W) ? Hs[b + 1] : vinf;
          const s16x2 diag = mad_sat(mmp, vx, Hsd);  // H(i-1,j-1) + cost + hoff
          const s16x2 dg = mmp * vxm1 + Hsd;         // ... with the match/mismatch tie offset
          if (AFF) {
            const s16x2 Eu = (b + 1 < W) ? E[b + 1] : vinf;
            const s16x2 bE = adds(Eu, ve), Ev = mn(Hsu, bE);
            const s16x2 bF = adds(Fl, ve), Fv = mn(Hsl, bF);
            const s16x2 G = mn(Ev, Fv);
            const s16x2 Gs = adds(G, voe);
            const s16x2 Hsv = mn(diag, Gs);
            acc01 = push_signs(acc01, dg - Gs, Fv - Ev);
            acc23 = push_signs(acc23, bE - Hsu, bF - Hsl);
            Hs[b] = Hsv;
            E[b] = Ev;
            Hsl = Hsv;
            Fl = Fv;
          } else {
            const s16x2 G = mn(Hsu, Hsl);
            const s16x2 Gs = adds(G, ve);
            const s16x2 Hsv = mn(diag, Gs);
            acc01 = push_signs(acc01, dg - Gs, Hsl - Hsu);
            Hs[b] = Hsv;
            Hsl = Hsv;
          }
          // keep each cell's bit packing next to its arithmetic (see the
          // 32-bit band kernel); the empty asm emits nothing
          asm volatile("" : "+v"(acc01));
          if (AFF) asm volatile("" : "+v"(acc23));
        }
        if (P.want_cigar) {
          row[(g * (NP / 2)) * 64] = acc01;
          if (AFF) row[(g * (NP / 2) + 1) * 64] = acc23;
        }
      }
      const bool cap0 = run[0] && i == m[0], cap1 = run[1] && i == m[1];
      if (__ballot(cap0 || cap1)) {
#pragma unroll
        for (int b = 0; b < W; ++b) {
          if (cap0 && b == bstar[0]) score[0] = Hs[b].x - hoff;
          if (cap1 && b == bstar[1]) score[1] = Hs[b].y - hoff;
        }
      }
    }

    bool accept[2] = {false, false};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!run[h]) continue;
      const int32_t d = n[h] - m[h], kmax = kmin[h] + W - 1;
      const int32_t lb_up = kmax + 1 > n[h] ? DP_INF : 2 * o + e * (2 * (kmax + 1) - d);
      const int32_t lb_lo = kmin[h] - 1 < -m[h] ? DP_INF : 2 * o + e * (2 * (1 - kmin[h]) + d);
      const int32_t LB = min(lb_up, lb_lo);
      esc[h] = false;
      if (score[h] < LB) {
        if (P.max_score >= 0 && score[h] > P.max_score) {
          O.score[p[h]] = -1;
          O.status[p[h]] = ST_REJECTED;
          O.nruns[p[h]] = 0;
        } else {
          accept[h] = true;
          O.score[p[h]] = score[h];
          O.status[p[h]] = ST_ALIGNED;
          O.nruns[p[h]] = (SPLIT && P.want_cigar) ? -1 : 0;
        }
      } else if (P.max_score >= 0 && LB > P.max_score) {
        O.score[p[h]] = -1;
        O.status[p[h]] = ST_REJECTED;
        O.nruns[p[h]] = 0;
      } else {
        esc[h] = true;
        // the split traceback must not take a stale -1 for its mark
        if (SPLIT) O.nruns[p[h]] = 0;
      }
    }
    if (Wk.next_idx) {
      dev::wave_append(run[0] && esc[0], (int32_t)p[0], Wk.next_idx, Wk.next_count);
      dev::wave_append(run[1] && esc[1], (int32_t)p[1], Wk.next_idx, Wk.next_count);
    }
    if (!P.want_cigar) continue;

    if (SPLIT) continue;
    // ---- traceback of both pairs of each lane over this wavefront's rows ----
    // The rows were stored by this wavefront during the fill; the fence makes
    // them visible to its loads (no stale L1 line from an earlier chunk).
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    {
      constexpr int ROW = NP * 2 * 64;
      constexpr int PRE = FUSED_ROWS * ROW / 4 / 64;
      Walker16<AFF> wk[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (accept[h]) wk[h].begin(O, p[h], m[h], n[h], kmin[h]);
      const int32_t top = dev::wave_max(max(accept[0] ? m[0] : 0, accept[1] ? m[1] : 0));
#pragma unroll 1
      for (int32_t hi = top; hi > 0; hi -= FUSED_ROWS) {
        const int32_t lo = max(hi - FUSED_ROWS, 0);  // rows lo+1 .. hi
        const int nq = (hi - lo) * (ROW / 4);
        const u32x4 *g = reinterpret_cast<const u32x4 *>(tb + (int64_t)(lo + 1) * ROW);
        u32x4 pre[PRE];
#pragma unroll
        for (int k = 0; k < PRE; ++k) pre[k] = g[min(lane + 64 * k, nq - 1)];
        uint64_t w[2][5];
        int64_t pq0[2], tq0[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          pq0[h] = lo >> 5;
          tq0[h] = ((int64_t)lo + kmin[h]) >> 5;
          const bool need = accept[h] && wk[h].i > lo && wk[h].j > 0;
          const int64_t pn = need ? pnw[h] : 0, tn = need ? tnw[h] : 0;
          w[h][0] = dev::ld_word(pat[h], pn, pq0[h]);
          w[h][1] = dev::ld_word(pat[h], pn, pq0[h] + 1);
          w[h][2] = dev::ld_word(txt[h], tn, tq0[h]);
          w[h][3] = dev::ld_word(txt[h], tn, tq0[h] + 1);
          w[h][4] = dev::ld_word(txt[h], tn, tq0[h] + 2);
        }
        __syncthreads();  // the previous block is no longer read
#pragma unroll
        for (int k = 0; k < PRE; ++k) fused_stage[lane + 64 * k] = pre[k];
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (accept[h])
            wk[h].walk(reinterpret_cast<const uint32_t *>(fused_stage), lane, h, lo, w[h][0], w[h][1],
                       w[h][2], w[h][3], w[h][4], pq0[h], tq0[h], 0xfu);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (accept[h]) wk[h].finish(O, p[h]);
    }
  }
}

// Traceback of the pairs the split fill accepted.  A workgroup of two
// wavefronts takes one chunk of 128 pairs; wavefront h walks the pairs held in
// half h of the packed words.  The chunk's rows are staged in LDS, TB_ROWS at
// a time from its last row down, with full-line loads, and every lane walks
// until its path leaves the staged rows; the sequence words the staged rows
// can touch are loaded into registers beside them.  A lane's row index only
// decreases, so each row is read from HBM once.
constexpr int TB_ROWS = 8;
// cells a lane's diagonal may move, over the block it is on and the next,
// with the next block's rows still staged (further moves re-stage the block)
constexpr int TB_TRACK = 3;

template <bool AFF>
__global__ __launch_bounds__(128) void k_band16_tb(Seqs Sq, Outs O, Work Wk, const uint32_t *tb_all,
                                                  int64_t tb_chunk_words) {
  constexpr int NP = AFF ? 4 : 2;
  constexpr int ROW = NP * 2 * 64;  // words per row
  __shared__ u32x4 stage[TB_ROWS * ROW / 4];
  __shared__ int32_t s_chunk, s_top;
  __shared__ uint32_t s_gm[2], s_miss[2];
  const uint32_t *lds = reinterpret_cast<const uint32_t *>(stage);
  const int tid = threadIdx.x, lane = tid & 63, h = tid >> 6;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * 128 >= count) return;
  for (;;) {
    if (tid == 0) {
      s_chunk = atomicAdd(Wk.counter, 1);
      s_top = 0;
    }
    __syncthreads();
    const int64_t chunk = s_chunk;
    if (chunk * 128 >= count) break;
    const int64_t li = chunk * 128 + 64 * h + lane;
    bool act = false;
    int64_t p = 0;
    if (li < count) {
      p = Wk.idx ? (int64_t)Wk.idx[li] : li;
      act = O.nruns[p] == -1;
    }
    int32_t m = 0, n = 0, kmin = 0;
    const uint64_t *pat = Sq.pat, *txt = Sq.txt;
    if (act) {
      m = Sq.pat_len[p];
      n = Sq.txt_len[p];
      const int32_t d = n - m, ad = d < 0 ? -d : d;
      kmin = min(0, d) - (W - 1 - ad) / 2;
      pat += Sq.pat_off[p];
      txt += Sq.txt_off[p];
    }
    const int32_t wm = dev::wave_max(m);
    if (lane == 0) atomicMax(&s_top, wm);
    __syncthreads();
    const int32_t top = s_top;
    const uint32_t *src = tb_all + chunk * tb_chunk_words;
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;

    Walker16<AFF> wk;
    if (act) wk.begin(O, p, m, n, kmin);
    // rows lo+1 .. hi of the block below `hi` go through registers: the
    // next block's loads are in flight while the lanes walk this one.  Of a
    // row only the cell groups near the lanes' diagonals are fetched: the
    // 16-byte piece at stage position tid + 128 k belongs to group qg (the
    // same for every k, 128 being a multiple of the pieces per row).
    constexpr int PRE = TB_ROWS * ROW / 4 / 128;
    constexpr int QR = ROW / 4;
    const int qg = ((tid % QR) * 4) / QR;
    u32x4 pre[PRE];
#define AIM_TB_FETCH(BHI, GM)                                                          \
  do {                                                                                 \
    const int32_t bhi_ = (BHI), blo_ = max(bhi_ - TB_ROWS, 0);                         \
    const int nq_ = (bhi_ - blo_) * QR;                                                \
    const u32x4 *g_ = reinterpret_cast<const u32x4 *>(src + (int64_t)(blo_ + 1) * ROW); \
    if (((GM) >> qg) & 1u)                                                             \
      _Pragma("unroll") for (int k = 0; k < PRE; ++k) pre[k] = g_[min(tid + 128 * k, nq_ - 1)]; \
  } while (0)
    uint32_t gcur = 0xfu;  // groups of the block being walked
    if (top > 0) AIM_TB_FETCH(top, gcur);
    // sequence words of the current block, reloaded only when the block's
    // first word moves (every fourth block or so)
    int64_t pq0 = INT64_MIN, tq0 = INT64_MIN;
    uint64_t pw0 = 0, pw1 = 0, tw0 = 0, tw1 = 0, tw2 = 0;
#pragma unroll 1
    for (int32_t hi = top; hi > 0; hi -= TB_ROWS) {
      const int32_t lo = max(hi - TB_ROWS, 0);  // rows lo+1 .. hi
      // pattern bases lo .. hi-1; text bases lo+kmin .. hi-1+kmin+W-1.  They
      // are loaded before the stage is written, whose wait for this block's
      // rows then covers them too: loaded after it, their wait would come
      // after the next block's loads are issued and wait for those as well
      // (the wait counter is in order), so the walk could not overlap them.
      const int64_t pq = lo >> 5, tq = ((int64_t)lo + kmin) >> 5;
      if (pq != pq0) {
        pq0 = pq;
        pw0 = dev::ld_word(pat, pnw, pq);
        pw1 = dev::ld_word(pat, pnw, pq + 1);
      }
      if (tq != tq0) {
        tq0 = tq;
        tw0 = dev::ld_word(txt, tnw, tq);
        tw1 = dev::ld_word(txt, tnw, tq + 1);
        tw2 = dev::ld_word(txt, tnw, tq + 2);
      }
      // the groups fetched are written; entries past nq (copies of the
      // block's last piece) belong to no staged row and are never read
      if ((gcur >> qg) & 1u) {
#pragma unroll
        for (int k = 0; k < PRE; ++k) stage[tid + 128 * k] = pre[k];
      }
      // groups for the next block: within TB_TRACK cells of the diagonals
      // of the lanes still walking, as they stand before this block
      const bool live = act && wk.i > 0 && wk.j > 0;
      const int32_t bmin = -dev::wave_max(live ? -max(wk.b - TB_TRACK, 0) : -W);
      const int32_t bmax = dev::wave_max(live ? min(wk.b + TB_TRACK, W - 1) : -1);
      if (lane == 0)
        s_gm[h] = bmax < 0 ? 0u : ((2u << (bmax >> 3)) - 1u) & ~((1u << (bmin >> 3)) - 1u);
      __syncthreads();
      const uint32_t gnext = s_gm[0] | s_gm[1];
      // the next block; after the last one, a one-row dummy
      AIM_TB_FETCH(lo > 0 ? lo : 1, gnext);
      const bool miss = act && wk.walk(lds, lane, h, lo, pw0, pw1, tw0, tw1, tw2, pq0, tq0, gcur);
      const bool wmiss = __ballot(miss) != 0;
      if (lane == 0) s_miss[h] = wmiss;
      __syncthreads();
      if (s_miss[0] | s_miss[1]) {
        // a path left the groups staged: stage the rest of the block, one
        // piece at a time (rare), and walk on
        const u32x4 *g = reinterpret_cast<const u32x4 *>(src + (int64_t)(lo + 1) * ROW);
        const int nq = (hi - lo) * QR;
        if (!((gcur >> qg) & 1u)) {
#pragma unroll 1
          for (int k = 0; k < PRE; ++k) stage[tid + 128 * k] = g[min(tid + 128 * k, nq - 1)];
        }
        __syncthreads();
        if (act) wk.walk(lds, lane, h, lo, pw0, pw1, tw0, tw1, tw2, pq0, tq0, 0xfu);
        __syncthreads();
      }
      gcur = gnext;
    }
    if (act) wk.finish(O, p);
    __syncthreads();
  }
}
#undef AIM_TB_FETCH

}  // namespace

bool band16_fits(int32_t max_len, const Scoring &P, bool affine) {
  const int64_t hoff = affine ? P.o + P.e : P.e;
  return (int64_t)P.x * max_len + 2 * (int64_t)P.o + (int64_t)P.e * 2 * max_len + 2 * hoff +
             2 * (int64_t)P.x <= VMAX;
}

hipError_t launch_band16(bool affine, bool split, const Seqs &S, const Outs &O, const Scoring &P,
                         const Work &Wk, uint32_t *tb, int64_t tb_slot_words, int32_t rows_cap,
                         int32_t nslots, hipStream_t s) {
  dim3 grid(nslots), block(64);
  if (affine && split)
    hipLaunchKernelGGL((k_band16<true, true>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else if (affine)
    hipLaunchKernelGGL((k_band16<true, false>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else if (split)
    hipLaunchKernelGGL((k_band16<false, true>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  else
    hipLaunchKernelGGL((k_band16<false, false>), grid, block, 0, s, S, O, P, Wk, tb, tb_slot_words, rows_cap);
  return hipGetLastError();
}

hipError_t launch_band16_tb(bool affine, const Seqs &S, const Outs &O, const Work &Wk, const uint32_t *tb,
                            int64_t tb_chunk_words, int32_t nslots, hipStream_t s) {
  dim3 grid(nslots), block(128);
  if (affine)
    hipLaunchKernelGGL((k_band16_tb<true>), grid, block, 0, s, S, O, Wk, tb, tb_chunk_words);
  else
    hipLaunchKernelGGL((k_band16_tb<false>), grid, block, 0, s, S, O, Wk, tb, tb_chunk_words);
  return hipGetLastError();
}

}  // namespace aim
