// Gap-affine wavefront alignment of pairs whose wavefronts outgrow the
// one-wavefront pass, with the recent wavefronts resident in LDS (k_wfa_lds).
//
// Paper: System and Methods, "Wavefront Algorithm (WFA)" (the recurrences of
// wfa.hip, restated there) and "Data Management" (the components a step
// needs are kept in fast on-chip memory, the rest off chip): here the last
// max(x, o+e) + 1 wavefronts of M and the last e + 1 of I and D live in the
// workgroup's LDS, the origin codes of every cell (what the backtrace
// chooses) go to an HBM slot, and the pair's CIGAR is walked from them.
//
// Layout.  A class has a window of W diagonals, [-W/2, W/2).  A ring row is
// indexed by absolute diagonal (entry k + W/2 + MG), two 16-bit offsets per
// 32-bit word (the even entry in the low half), with MG entries of margin at
// each end.  Entries outside a wavefront's range hold a negative (absent)
// value: each row is written over its range and over MG/2 words beyond each
// end, which covers every later read of it (a row is read for at most
// max(x, o+e) more scores, and the range grows by at most one diagonal per
// score at each end), so a cell needs no range tests, only the table bound
// j <= min(n, m + k).  Sources of a score that is absent (null, or negative)
// read a row of absent marks.
//
// Arithmetic.  A lane computes the two diagonals of one word with packed
// 16-bit max / add / subtract.  An absent mark starts at -32768 and can only
// grow by one per score, so a pair stays below s_cap (16,000) scores here;
// offsets are at most n <= 32,000.  The candidates are clipped as the oracle
// clips them: I = max(M_{s-o-e}[k+1], I_{s-e}[k+1]), dropped when its row
// passes m; D = max(M_{s-o-e}[k-1], D_{s-e}[k-1]) + 1, dropped past n;
// X = M_{s-x}[k] + 1, dropped past either end.
//
// A pair whose wavefront leaves the window goes to the next class (route),
// with a prediction of the window it needs.
#include "aim_internal.h"

namespace aim {
namespace {

#include "wfa_common.h"

constexpr int ENTRY_WORDS = 4;  // full-store table entry, as counted by the other passes
constexpr uint32_t ABSENT2 = 0x80008000u;

typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 as2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ uint32_t as1(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// c where c <= lim, else exactly the absent mark; an absent c stays negative.
// The sign mask is one packed arithmetic shift (written out: left to itself
// the compiler turns the shift-and-mask into a select, which it does half by
// half), the choice one bitfield insert.
__device__ __forceinline__ s16x2 clip2(s16x2 c, s16x2 lim) {
  const uint32_t d = as1(lim - c);  // sign set in a half where c > lim
  uint32_t bad;
  asm("v_pk_ashrrev_i16 %0, %1, %2" : "=v"(bad) : "v"(0x000f000fu), "v"(d));
  return as2((bad & ABSENT2) | (~bad & as1(c)));
}

// The origin codes of the two cells of a word as one byte (low nibble: the
// even diagonal): bits 0-1 the first of X, I, D that attains M, bit 2 I
// opened from M_{s-o-e} (also on a tie), bit 3 the same for D.  Computed
// from the signs of saturated packed differences.
__device__ __forceinline__ uint32_t codes2(s16x2 X, s16x2 I, s16x2 Mv, s16x2 Mo_up, s16x2 Ie_up,
                                           s16x2 Mo_dn, s16x2 De_dn) {
  const uint32_t sx = as1(__builtin_elementwise_sub_sat(X, Mv));         // sign: X < M
  const uint32_t si = as1(__builtin_elementwise_sub_sat(I, Mv));         // sign: I < M
  const uint32_t sio = as1(__builtin_elementwise_sub_sat(Mo_up, Ie_up));  // sign: I extended
  const uint32_t sdo = as1(__builtin_elementwise_sub_sat(Mo_dn, De_dn));  // sign: D extended
  const uint32_t a = (sx >> 15) & 0x10001u, b = (si >> 15) & 0x10001u;
  const uint32_t c = (~sio >> 15) & 0x10001u, d = (~sdo >> 15) & 0x10001u;
  const uint32_t nib = (a & ~b) | ((a & b) << 1) | (c << 2) | (d << 3);
  return (nib | (nib >> 12)) & 0xffu;
}

// Index of the lowest set bit, all ones for 0 (the instruction's own result;
// the C builtins leave 0 undefined or add a select for it).
__device__ __forceinline__ uint32_t ffbl_raw(uint32_t d) {
  uint32_t r;
  asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(d));
  return r;
}

// Equal bases (at most 16, at most le) from pattern base i and text base j.
__device__ __forceinline__ uint32_t run16(const uint32_t *P32, const uint32_t *T32, int32_t i, int32_t j,
                                          uint32_t le) {
  const uint32_t d = __builtin_amdgcn_alignbit(P32[(i >> 4) + 1], P32[i >> 4], (uint32_t)i << 1) ^
                     __builtin_amdgcn_alignbit(T32[(j >> 4) + 1], T32[j >> 4], (uint32_t)j << 1);
  return min(min(ffbl_raw(d) >> 1, 16u), le);
}

// Extension of both offsets of a word (diagonals k0 and k0 + 1; absent when
// negative; LIM = min(n, m + k) per half).  The first 16 bases of each by
// every lane without a branch -- an absent offset compares at base 0 under a
// zero limit (an absent mark is below -16,000 and |k| <= 16,001, so it
// clamps to 0) -- then one branch for the rare runs of 16 matches.
__device__ __forceinline__ void ext_pair(const uint32_t *P32, const uint32_t *T32, int32_t m, int32_t n,
                                         int32_t k0, s16x2 Mv, s16x2 LIM, int32_t &f0, int32_t &f1) {
  const int32_t a = Mv.x, b = Mv.y;
  const int32_t ja = max(a, 0), jb = max(b, 0);
  const int32_t ia = max(a - k0, 0), ib = max(b - k0 - 1, 0);
  const uint32_t lea = a >= 0 ? (uint32_t)(LIM.x - a) : 0u, leb = b >= 0 ? (uint32_t)(LIM.y - b) : 0u;
  const uint32_t ra = run16(P32, T32, ia, ja, lea), rb = run16(P32, T32, ib, jb, leb);
  int32_t ga = ja + (int32_t)ra, gb = jb + (int32_t)rb;
  if (ra == 16u || rb == 16u) {
    if (ra == 16u) ga = extend_lds(P32, m, T32, n, k0, ga);
    if (rb == 16u) gb = extend_lds(P32, m, T32, n, k0 + 1, gb);
  }
  f0 = a >= 0 ? ga : a;
  f1 = b >= 0 ? gb : b;
}

// Minimum (MAX false) or maximum over the 64 lanes of a wavefront, all
// active: shifts within rows of 16, then the row broadcasts of lanes 15 and
// 31 (lanes without a source keep the identity); lane 63 ends with the result.
template <bool MAX>
__device__ __forceinline__ int32_t wave_reduce(int32_t v) {
  constexpr int32_t id = MAX ? INT32_MIN : INT32_MAX;
  auto op = [](int32_t a, int32_t b) { return MAX ? max(a, b) : min(a, b); };
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Buffer resource word 3 for raw (untyped) buffer access on CDNA: 32-bit
// data format, so that loads return data and accesses past num_records read
// zero / are dropped.
constexpr int32_t BUF_FLAGS = 0x00027000;

// The ring rows of one workgroup: R rows of M, e + 1 of I, e + 1 of D, then
// a row of absent marks; row r, word q.  In LDS, or in a global slot reached
// through a buffer resource (a 32-bit lane offset, the row in the scalar
// offset), which spares the 64-bit address arithmetic per access.
template <bool G>
struct RingIO;
template <>
struct RingIO<false> {
  uint32_t *base;
  int32_t RW;
  __device__ __forceinline__ uint32_t ld(int32_t row, int32_t q, int32_t delta) const {
    return base[row * RW + q + delta];
  }
  __device__ __forceinline__ void st(int32_t row, int32_t q, uint32_t v) const { base[row * RW + q] = v; }
};
// The resource starts one word before row 0, so that the scalar offset of
// row 0 word q - 1 is (1 + 0 - 1) * 4 = 0 and never negative (the hardware
// adds it unsigned).
template <>
struct RingIO<true> {
  __amdgpu_buffer_rsrc_t rs;
  int32_t RW;
  __device__ __forceinline__ uint32_t ld(int32_t row, int32_t q, int32_t delta) const {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, q * 4, (1 + row * RW + delta) * 4, 0);
  }
  __device__ __forceinline__ void st(int32_t row, int32_t q, uint32_t v) const {
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, q * 4, (1 + row * RW) * 4, 0);
  }
};

// GRING: the ring rows live in this workgroup's slot of a global buffer
// (HBM, cached in L2 and the infinity cache) instead of LDS, so that many
// more workgroups fit a CU; the arithmetic is the same.
template <int T, bool GRING, bool ADAPT>
__global__ __launch_bounds__(T) void k_wfa_lds(Seqs S, Outs O, Scoring P, Work Wk, WfaLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int32_t x = P.x, oe = P.o + P.e, e = P.e, R = L.R, RE = P.e + 1;
  const int32_t W = L.W, kbase = -(W >> 1), MG = L.MG, MGW = L.MG >> 1;
  const int32_t RW = (W + 2 * MG) >> 1;  // 32-bit words per ring row
  const int32_t SW = L.seq_words + 1;     // staged words per sequence, one of padding
  uint64_t *sP = (uint64_t *)smem;
  uint64_t *sT = sP + SW;
  int32_t *tab = (int32_t *)(sT + SW);  // per M slot: lo, hi, flags (1 present, 2 has I and D), -
  int32_t *shv = tab + 4 * R;           // [0] work item, [1] end cell reached, [2] progress
  // a global slot: one guard word, then the rows (see RingIO<true>)
  uint32_t *ringM = GRING ? L.gring + (int64_t)blockIdx.x * L.gring_slot + 1 : (uint32_t *)(shv + 8);
  uint32_t *nullrow = ringM + (int64_t)(R + 2 * RE) * RW;
  const int32_t NULLR = R + 2 * RE;  // the row of absent marks
  RingIO<GRING> ring;
  if constexpr (GRING)
    ring.rs = __builtin_amdgcn_make_buffer_rsrc(ringM - 1, 0, (int32_t)(L.gring_slot * 4), BUF_FLAGS);
  else
    ring.base = ringM;
  ring.RW = RW;
  const uint32_t *P32 = reinterpret_cast<const uint32_t *>(sP);
  const uint32_t *T32 = reinterpret_cast<const uint32_t *>(sT);
  const int32_t count = Wk.count ? __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)Wk.count)
                                 : (int32_t)Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int32_t)blockIdx.x >= count) return;
  for (int32_t q = tid; q < RW; q += T) nullrow[q] = ABSENT2;
  uint8_t *cslot = L.codes + (int64_t)blockIdx.x * L.code_slot;
  int32_t *ctab = reinterpret_cast<int32_t *>(cslot);  // per score: lowest kept diagonal, hi, code offset
  uint8_t *cbytes = cslot + (int64_t)L.steps_cap * 12;
  auto widx = [&](int32_t k) { return (k - kbase + MG) >> 1; };
  // (adaptive) diagonals this workgroup dropped: one atomic at the end, not
  // one per score -- thousands of workgroups adding to one address every
  // score serialise on it
  uint64_t ad_drop = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) shv[0] = atomicAdd(Wk.counter, 1);
    __syncthreads();
    const int32_t li = __builtin_amdgcn_readfirstlane(shv[0]);
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)__builtin_amdgcn_readfirstlane(Wk.idx[li]) : li;
    if (O.flags && __builtin_amdgcn_readfirstlane((int32_t)O.flags[p])) {
      if (tid == 0) { O.score[p] = -1; O.status[p] = ST_INVALID; O.nruns[p] = 0; }
      continue;
    }
    const int32_t m = __builtin_amdgcn_readfirstlane(S.pat_len[p]);
    const int32_t n = __builtin_amdgcn_readfirstlane(S.txt_len[p]);
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    {
      // the host sends only batches whose sequences fit the staging area
      const uint64_t *gP = S.pat + S.pat_off[p], *gT = S.txt + S.txt_off[p];
      for (int64_t q = tid; q <= pnw; q += T) sP[q] = q < pnw ? gP[q] : 0ull;
      for (int64_t q = tid; q <= tnw; q += T) sT[q] = q < tnw ? gT[q] : 0ull;
    }
    if (tid < R) tab[4 * tid + 2] = 0;
    if (tid == 0) shv[1] = 0;
    const int32_t kend = n - m;
    const int64_t ad = m > n ? m - n : n - m;
    const int64_t up1 = (int64_t)x * min(m, n) + (ad ? (int64_t)P.o + ad * e : 0);
    const int64_t up2 = (m ? (int64_t)P.o + (int64_t)m * e : 0) + (n ? (int64_t)P.o + (int64_t)n * e : 0);
    const int32_t s_upper = (int32_t)min<int64_t>(min(up1, up2), INT32_MAX - 1);
    const int32_t s_lim = min(P.max_score >= 0 ? min(P.max_score, s_upper) : s_upper, L.s_cap);
    // 1 aligned, 2 rejected, 3 left the window, 4 past its bound, 5 past s_cap
    int result = (kend < kbase || kend >= kbase + W) ? 3 : 0;
    int32_t ext_out = result ? max(-kend, kend + 1) : 0;
    int32_t s = 0;
    int64_t need = 0, cb = 0;
    bool keep = P.want_cigar != 0;
    __syncthreads();  // staged words, cleared table and flag visible
    if (!result) {
      // s = 0: M_0[0] = extend(0); absent marks around it
      uint32_t *r0 = ringM;
      const int32_t qc = widx(0);
      for (int32_t q = qc - MGW - 1 + tid; q <= qc + MGW + 1; q += T)
        if (q != qc) r0[q] = ABSENT2;
      if (tid == 0) {
        const int32_t f = extend_lds(P32, m, T32, n, 0, 0);
        r0[qc] = (uint32_t)(f & 0xffff) | 0x80000000u;  // diagonal 1 (high half) absent
        tab[0] = 0;
        tab[1] = 0;
        tab[2] = 1;  // present, no I or D
        if (kend == 0 && f >= n) shv[1] = 1;
      }
      need = ENTRY_WORDS + 2;
      __syncthreads();  // the step loop reads the end-cell flag first
    }
    int32_t sl = 0, sE = 0;  // s mod R, s mod (e + 1)
    const s16x2 M2 = (s16x2)(short)m, N2 = (s16x2)(short)n;
    const int4 *tab4 = reinterpret_cast<const int4 *>(tab);
    // One word of score s (diagonals k0 = 2q - MG + kbase and k0 + 1) from
    // its eight source words: candidates, codes, extension, stores.
    // what a word leaves behind: whether it reached the end cell, its three
    // stored words, and (adaptive) the distance to the end of each offset
    struct WordRes {
      bool hit;
      uint32_t mw, iw, dw;
      int32_t d0, d1;
    };
    auto word = [&](int32_t q, uint32_t o_m, uint32_t o_0, uint32_t o_p, uint32_t i_0, uint32_t i_p,
                    uint32_t d_m, uint32_t d_0, uint32_t x_0, int32_t rM, int32_t rI, int32_t rD,
                    bool kc, uint8_t *crow, int32_t q_lo) -> WordRes {
      const int32_t k0 = 2 * q - MG + kbase;
      const s16x2 K2 = {(short)k0, (short)(k0 + 1)};
      const s16x2 LIM = __builtin_elementwise_min(__builtin_elementwise_add_sat(M2, K2), N2);
      const s16x2 Mo_up = as2(__builtin_amdgcn_alignbit(o_p, o_0, 16));  // M_{s-o-e}[k + 1]
      const s16x2 Mo_dn = as2(__builtin_amdgcn_alignbit(o_0, o_m, 16));  // M_{s-o-e}[k - 1]
      const s16x2 Ie_up = as2(__builtin_amdgcn_alignbit(i_p, i_0, 16));  // I_{s-e}[k + 1]
      const s16x2 De_dn = as2(__builtin_amdgcn_alignbit(d_0, d_m, 16));  // D_{s-e}[k - 1]
      const s16x2 I = clip2(__builtin_elementwise_max(Mo_up, Ie_up), LIM);
      const s16x2 D = clip2(__builtin_elementwise_max(Mo_dn, De_dn) + (short)1, LIM);
      const s16x2 X = clip2(as2(x_0) + (short)1, LIM);
      const s16x2 Mv = __builtin_elementwise_max(X, __builtin_elementwise_max(I, D));
      // a uniform row base and a 32-bit lane offset (a scalar-base store);
      // kc is uniform, so this is a scalar branch
      if (kc) crow[(uint32_t)(q - q_lo)] = (uint8_t)codes2(X, I, Mv, Mo_up, Ie_up, Mo_dn, De_dn);
      int32_t f0, f1;
      ext_pair(P32, T32, m, n, k0, Mv, LIM, f0, f1);
      const uint32_t mw = __builtin_amdgcn_perm((uint32_t)f1, (uint32_t)f0, 0x05040100u);
      ring.st(rM, q, mw);
      ring.st(rI, q, as1(I));
      ring.st(rD, q, as1(D));
      WordRes r;
      r.hit = (k0 == kend && f0 >= n) || (k0 + 1 == kend && f1 >= n);
      r.mw = mw;
      r.iw = as1(I);
      r.dw = as1(D);
      r.d0 = f0 >= 0 ? max(m - (f0 - k0), n - f0) : INT32_MAX;
      r.d1 = f1 >= 0 ? max(m - (f1 - k0 - 1), n - f1) : INT32_MAX;
      return r;
    };
    while (!result) {
      // after a barrier: the end-cell flag of the last score and the table
      // entries of this score's sources, in one round trip to LDS
      const int32_t nsl = sl + 1 == R ? 0 : sl + 1;
      const int32_t nsE = sE + 1 == RE ? 0 : sE + 1;
      const int32_t qx = nsl >= x ? nsl - x : nsl - x + R;
      const int32_t qo = nsl >= oe ? nsl - oe : nsl - oe + R;
      const int32_t qe = nsl >= e ? nsl - e : nsl - e + R;
      const int32_t qeE = nsE + 1 == RE ? 0 : nsE + 1;  // (s - e) mod (e + 1)
      const int32_t hitv = shv[1];
      const int4 ex = tab4[qx], eo = tab4[qo], ee = tab4[qe];
      if (__builtin_amdgcn_readfirstlane(hitv)) {
        result = 1;
        break;
      }
      ++s;
      if (s > s_lim) {
        result = (P.max_score >= 0 && s > P.max_score) ? 2 : (s > s_upper ? 4 : 5);
        break;
      }
      sl = nsl;
      sE = nsE;
      const int32_t fx = s >= x ? __builtin_amdgcn_readfirstlane(ex.z) : 0;
      const int32_t fo = s >= oe ? __builtin_amdgcn_readfirstlane(eo.z) : 0;
      const int32_t fe = s >= e ? __builtin_amdgcn_readfirstlane(ee.z) : 0;
      // the range: over the non-null sources (the one of s - e only when it
      // has I and D), widened by one diagonal and clipped to [-m, n]
      int32_t lo = INT32_MAX, hi = INT32_MIN;
      if (fx & 1) {
        lo = min(lo, __builtin_amdgcn_readfirstlane(ex.x));
        hi = max(hi, __builtin_amdgcn_readfirstlane(ex.y));
      }
      if (fo & 1) {
        lo = min(lo, __builtin_amdgcn_readfirstlane(eo.x));
        hi = max(hi, __builtin_amdgcn_readfirstlane(eo.y));
      }
      if (fe & 2) {
        lo = min(lo, __builtin_amdgcn_readfirstlane(ee.x));
        hi = max(hi, __builtin_amdgcn_readfirstlane(ee.y));
      }
      const bool present = ((fx | fo) & 1) || (fe & 2);
      if (present) {
        lo = max(lo - 1, -m);
        hi = min(hi + 1, n);
      }
      if (!present || lo > hi) {
        // a null wavefront: nothing to store, its readers take absent marks
        if (tid == 0) {
          tab[4 * sl + 2] = 0;
          if (keep && s < L.steps_cap) { ctab[3 * s] = 1; ctab[3 * s + 1] = 0; ctab[3 * s + 2] = 0; }
        }
        need += ENTRY_WORDS;
        __syncthreads();
        continue;
      }
      if (lo < kbase || hi >= kbase + W) {
        result = 3;
        ext_out = max(-lo, hi + 1);
        break;
      }
      // rows: sources (the absent row for a null source) and destinations
      const int32_t rX = (fx & 1) ? qx : NULLR, rO = (fo & 1) ? qo : NULLR;
      const int32_t rIe = (fe & 2) ? R + qeE : NULLR, rDe = (fe & 2) ? R + RE + qeE : NULLR;
      const int32_t rM = sl, rI = R + sE, rD = R + RE + sE;
      const int32_t q_lo = widx(lo), q_hi = widx(hi);
      const int32_t nbytes = q_hi - q_lo + 1;
      if (keep && (s >= L.steps_cap || cb + nbytes > L.code_cap)) keep = false;
      uint8_t *crow = keep ? cbytes + cb : nullptr;
      const bool kc = __builtin_amdgcn_readfirstlane((int32_t)keep) != 0;
      bool hit = false;  // this lane reached the end cell
      // (adaptive) this lane's words of the first trip, kept for the reduction
      int32_t fq[2] = {-1, -1};
      uint32_t fm[2] = {0u, 0u}, fi[2] = {0u, 0u}, fd[2] = {0u, 0u};
      int32_t fdist[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
      // two words per lane and trip, their sixteen source loads issued first
      for (int32_t qa = q_lo + tid; qa <= q_hi; qa += 2 * T) {
        const bool vb = qa + T <= q_hi;
        const int32_t qb = vb ? qa + T : qa;
        const uint32_t a_om = ring.ld(rO, qa, -1), a_o0 = ring.ld(rO, qa, 0), a_op = ring.ld(rO, qa, 1);
        const uint32_t a_i0 = ring.ld(rIe, qa, 0), a_ip = ring.ld(rIe, qa, 1);
        const uint32_t a_dm = ring.ld(rDe, qa, -1), a_d0 = ring.ld(rDe, qa, 0), a_x = ring.ld(rX, qa, 0);
        const uint32_t b_om = ring.ld(rO, qb, -1), b_o0 = ring.ld(rO, qb, 0), b_op = ring.ld(rO, qb, 1);
        const uint32_t b_i0 = ring.ld(rIe, qb, 0), b_ip = ring.ld(rIe, qb, 1);
        const uint32_t b_dm = ring.ld(rDe, qb, -1), b_d0 = ring.ld(rDe, qb, 0), b_x = ring.ld(rX, qb, 0);
        const WordRes ra = word(qa, a_om, a_o0, a_op, a_i0, a_ip, a_dm, a_d0, a_x, rM, rI, rD, kc, crow, q_lo);
        hit |= ra.hit;
        const bool first = qa == q_lo + tid;
        if (ADAPT && first) {
          fq[0] = qa; fm[0] = ra.mw; fi[0] = ra.iw; fd[0] = ra.dw; fdist[0] = ra.d0; fdist[1] = ra.d1;
        }
        if (vb) {
          const WordRes rb = word(qb, b_om, b_o0, b_op, b_i0, b_ip, b_dm, b_d0, b_x, rM, rI, rD, kc, crow, q_lo);
          hit |= rb.hit;
          if (ADAPT && first) {
            fq[1] = qb; fm[1] = rb.mw; fi[1] = rb.iw; fd[1] = rb.dw; fdist[2] = rb.d0; fdist[3] = rb.d1;
          }
        }
      }
      if (hit) shv[1] = 1;
      // absent marks for MG entries beyond each end of the three new rows
      for (int32_t t = tid; t < 2 * MGW; t += T) {
        const int32_t q = t < MGW ? q_lo - MGW + t : q_hi + 1 + (t - MGW);
        ring.st(rM, q, ABSENT2);
        ring.st(rI, q, ABSENT2);
        ring.st(rD, q, ABSENT2);
      }
      if constexpr (ADAPT) {
        // one wavefront whose lanes hold every word of this score (one trip):
        // the reduction in registers, no barrier; each lane rewrites the
        // dropped halves of its own words.  (A score that reached the end
        // cell is the last: no reduction.)
        const bool fast = T == 64 && q_hi - q_lo + 1 <= 2 * T;
        if (fast && hi - lo + 1 >= L.ad_min && !__ballot(hit)) {
          const int32_t dmin = wave_reduce<false>(min(min(fdist[0], fdist[1]), min(fdist[2], fdist[3])));
          if (dmin != INT32_MAX) {
            int32_t kl = INT32_MAX, kh = INT32_MIN;
            for (int32_t w = 0; w < 2; ++w) {
              const int32_t k0 = 2 * fq[w] - MG + kbase;
              for (int32_t h = 0; h < 2; ++h) {
                const int32_t d = fdist[2 * w + h];
                if (fq[w] >= 0 && d != INT32_MAX && d - dmin <= L.ad_max) {
                  kl = min(kl, k0 + h);
                  kh = max(kh, k0 + h);
                }
              }
            }
            const int32_t nlo = wave_reduce<false>(kl), nhi = wave_reduce<true>(kh);
            for (int32_t w = 0; w < 2; ++w) {
              if (fq[w] < 0) continue;
              const int32_t k0 = 2 * fq[w] - MG + kbase;
              const uint32_t mask = ((k0 < nlo || k0 > nhi) ? 0xffffu : 0u) |
                                    ((k0 + 1 < nlo || k0 + 1 > nhi) ? 0xffff0000u : 0u);
              if (mask) {
                ring.st(rM, fq[w], (fm[w] & ~mask) | (ABSENT2 & mask));
                ring.st(rI, fq[w], (fi[w] & ~mask) | (ABSENT2 & mask));
                ring.st(rD, fq[w], (fd[w] & ~mask) | (ABSENT2 & mask));
              }
            }
            ad_drop += (nlo - lo) + (hi - nhi);
            lo = nlo;
            hi = nhi;
          }
        }
        if (!fast && hi - lo + 1 >= L.ad_min) __syncthreads();  // the rows of this score, and shv, are settled
        if (!fast && hi - lo + 1 >= L.ad_min && !__builtin_amdgcn_readfirstlane(shv[1])) {
          // WFA-adaptive reduction of this score's range, from the extended
          // M row: d(k) = max(m - i, n - j) of its offset; the ends go while
          // absent or more than ad_max behind the best d
          __syncthreads();  // every lane has read the end flag
          if (tid == 0) {
            shv[3] = INT32_MAX;
            shv[4] = INT32_MAX;
            shv[5] = INT32_MIN;
          }
          __syncthreads();
          auto dist = [&](int32_t k, int32_t f) { return max(m - (f - k), n - f); };
          auto entry = [&](uint32_t wv, int32_t h) { return (int32_t)(int16_t)(h ? (wv >> 16) : (wv & 0xffffu)); };
          int32_t dl = INT32_MAX;
          for (int32_t q = q_lo + tid; q <= q_hi; q += T) {
            const uint32_t wv = ring.ld(rM, q, 0);
            const int32_t k0 = 2 * q - MG + kbase;
            for (int32_t h = 0; h < 2; ++h) {
              const int32_t k = k0 + h, f = entry(wv, h);
              if (k >= lo && k <= hi && f >= 0) dl = min(dl, dist(k, f));
            }
          }
          dl = -wave_max_i32(-dl);
          if ((tid & 63) == 0) atomicMin(&shv[3], dl);
          __syncthreads();
          const int32_t dmin = __builtin_amdgcn_readfirstlane(shv[3]);
          if (dmin != INT32_MAX) {
            int32_t kl = INT32_MAX, kh = INT32_MIN;
            for (int32_t q = q_lo + tid; q <= q_hi; q += T) {
              const uint32_t wv = ring.ld(rM, q, 0);
              const int32_t k0 = 2 * q - MG + kbase;
              for (int32_t h = 0; h < 2; ++h) {
                const int32_t k = k0 + h, f = entry(wv, h);
                if (k >= lo && k <= hi && f >= 0 && dist(k, f) - dmin <= L.ad_max) {
                  kl = min(kl, k);
                  kh = max(kh, k);
                }
              }
            }
            kl = -wave_max_i32(-kl);
            kh = wave_max_i32(kh);
            if ((tid & 63) == 0) {
              atomicMin(&shv[4], kl);
              atomicMax(&shv[5], kh);
            }
            __syncthreads();
            const int32_t nlo = __builtin_amdgcn_readfirstlane(shv[4]);
            const int32_t nhi = __builtin_amdgcn_readfirstlane(shv[5]);
            // absent marks over the dropped diagonals of the three rows; a
            // word is rewritten by one lane, its kept half unchanged
            auto trim = [&](int32_t ka, int32_t kb) {  // drop [ka, kb]
              if (ka > kb) return;
              for (int32_t q = widx(ka) + tid; q <= widx(kb); q += T) {
                const int32_t k0 = 2 * q - MG + kbase;
                const uint32_t mask = ((k0 >= ka && k0 <= kb) ? 0xffffu : 0u) |
                                      ((k0 + 1 >= ka && k0 + 1 <= kb) ? 0xffff0000u : 0u);
                ring.st(rM, q, (ring.ld(rM, q, 0) & ~mask) | (ABSENT2 & mask));
                ring.st(rI, q, (ring.ld(rI, q, 0) & ~mask) | (ABSENT2 & mask));
                ring.st(rD, q, (ring.ld(rD, q, 0) & ~mask) | (ABSENT2 & mask));
              }
            };
            trim(lo, nlo - 1);
            trim(nhi + 1, hi);
            ad_drop += (nlo - lo) + (hi - nhi);
            lo = nlo;
            hi = nhi;
          }
        }
      }
      if (tid == 0) {
        tab[4 * sl] = lo;
        tab[4 * sl + 1] = hi;
        tab[4 * sl + 2] = 3;
        if (keep) {
          ctab[3 * s] = 2 * q_lo - MG + kbase;
          ctab[3 * s + 1] = hi;
          ctab[3 * s + 2] = (int32_t)cb;
        }
      }
      if (keep) cb += nbytes;
      need += ENTRY_WORDS + (3 * (int64_t)(hi - lo + 1) + 1) / 2;
      __syncthreads();
    }
    if (ADAPT && (result == 3 || result == 5)) {
      // the window holds every diagonal of the batch, so only s_cap ends
      // here: a score this class cannot represent
      if (tid == 0) { O.score[p] = -1; O.status[p] = ST_INVALID; O.nruns[p] = 0; }
      continue;
    }
    if (result == 3 || result == 5) {
      // on to a wider class, with the window the pair is predicted to need:
      // from the furthest anti-diagonal i + j any kept M offset reaches
      int32_t pred = INT32_MAX;
      if (result == 3) {
        if (tid == 0) shv[2] = 0;
        __syncthreads();
        int32_t prog = 0;
        for (int32_t t = 0; t < R; ++t) {
          const int32_t fl = __builtin_amdgcn_readfirstlane(tab[4 * t + 2]);
          if (!(fl & 1)) continue;
          const int32_t tlo = __builtin_amdgcn_readfirstlane(tab[4 * t]);
          const int32_t thi = __builtin_amdgcn_readfirstlane(tab[4 * t + 1]);
          const uint32_t *row = ringM + (int64_t)t * RW;
          for (int32_t k = tlo + tid; k <= thi; k += T) {
            const int32_t ix = k - kbase + MG;
            const int32_t f = (int32_t)(int16_t)(row[ix >> 1] >> (16 * (ix & 1)));
            if (f >= 0) prog = max(prog, 2 * f - k);
          }
        }
        prog = wave_max_i32(prog);
        if ((tid & 63) == 0) atomicMax(&shv[2], prog);
        __syncthreads();
        pred = predict_extent(ext_out, __builtin_amdgcn_readfirstlane(shv[2]), m, n);
      }
      if (tid == 0) route_pair(L.route, L.my_class, p, pred);
      continue;
    }
    bool walked = false;
    if (result == 1 && keep) {
      // the codes and table are global stores of every wave of this
      // workgroup: the barrier orders them before the walk's loads, the
      // agent-scope acquire drops L1 lines of an earlier pair's walk
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int32_t tok_cap = (R + 2 * RE) * RW;  // the ring, free now, holds the walk's tokens
      if (tid < 64) {
        const int32_t sfin = s;
        auto code_at = [&](int32_t cs, int32_t k) -> int32_t {  // per lane
          if (cs < 1 || cs > sfin) return -1;
          const int32_t klo = ctab[3 * cs], khi = ctab[3 * cs + 1];
          if (k < klo || k > khi) return -1;
          const uint32_t b = cbytes[ctab[3 * cs + 2] + ((k - klo) >> 1)];
          return (int32_t)(((k - klo) & 1) ? (b >> 4) : (b & 15u));
        };
        auto ext = [&](int32_t k, int32_t f) { return extend_wave(P32, m, T32, n, k, f); };
        // a re-run of a pair whose runs outgrew its slot and the pool writes
        // them straight into its CIGAR range
        uint32_t *dst = (ADAPT && Wk.direct) ? O.cigar + O.cigar_off[p] : nullptr;
        walked = walk_codes<true>(O, p, code_at, ext, x, oe, e, m, n, s, ringM, tok_cap, dst,
                                  dst ? O.nruns[p] : 0);
        if (!walked && tid == 0 && L.walk_fail) atomicAdd(L.walk_fail, 1);
      }
      __syncthreads();
    } else if (result == 1 && P.want_cigar && tid == 0 && L.walk_skip) {
      atomicAdd(L.walk_skip, 1);  // codes not kept: the full-store pass walks it
    }
    if (ADAPT && Wk.direct) continue;  // a re-run: the other outputs are final
    if (tid == 0) {
      if (result == 2 || result == 4) {
        O.score[p] = -1;
        O.status[p] = result == 2 ? ST_REJECTED : ST_INVALID;
        O.nruns[p] = 0;
      } else {
        O.score[p] = s * P.unit;
        O.status[p] = ST_ALIGNED;
        if (!walked) O.nruns[p] = 0;
        if (ADAPT && P.want_cigar && !walked) {
          O.status[p] = ST_OVERFLOW;  // no exact fallback for a heuristic alignment
        } else if (P.want_cigar && !walked) {
          L.need[p] = need;
          int c = 0;
          while (c < 3 && need > L.need_cap[c]) ++c;
          if (need > L.need_cap[3]) {
            to_long_pass(O, p, L.long_list, L.long_count);  // full store larger than any arena class
          } else {
            const int32_t k = atomicAdd(L.need_count[c], 1);
            L.need_list[c][k] = (int32_t)p;
            atomicMax(L.need_max[c], (int32_t)need);
          }
        }
      }
    }
  }
  if (ADAPT && tid == 0 && L.ad_dropped && ad_drop) atomicAdd(L.ad_dropped, (unsigned long long)ad_drop);
}

}  // namespace

int64_t wfa_ring_words(int32_t W, int32_t MG, int32_t R, int32_t e) {
  return (int64_t)(R + 2 * (e + 1) + 1) * ((W + 2 * MG) / 2);
}

size_t wfa_lds_bytes(int32_t W, int32_t MG, int32_t R, int32_t e, int32_t seq_words, bool gring) {
  return 2 * (size_t)(seq_words + 1) * 8 + (size_t)R * 16 + 32 + (gring ? 0 : (size_t)wfa_ring_words(W, MG, R, e) * 4);
}

hipError_t launch_wfa_lds(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, const WfaLds &L,
                          int32_t threads, int32_t nslots, hipStream_t s) {
  const bool g = L.gring != nullptr;
  const size_t lds = wfa_lds_bytes(L.W, L.MG, L.R, P.e, L.seq_words, g);
  if (L.ad_min > 0) {
    // WFA-adaptive
#define AIM_LAUNCH_AD(TT)                                                                              \
  if (g)                                                                                               \
    hipLaunchKernelGGL((k_wfa_lds<TT, true, true>), dim3(nslots), dim3(TT), lds, s, S, O, P, Wk, L);   \
  else                                                                                                 \
    hipLaunchKernelGGL((k_wfa_lds<TT, false, true>), dim3(nslots), dim3(TT), lds, s, S, O, P, Wk, L);
    switch (threads) {
      case 64: AIM_LAUNCH_AD(64) break;
      case 128: AIM_LAUNCH_AD(128) break;
      case 256: AIM_LAUNCH_AD(256) break;
      default: return hipErrorInvalidValue;
    }
#undef AIM_LAUNCH_AD
    return hipGetLastError();
  }
#define AIM_LAUNCH_LDS(TT)                                                                             \
  if (g)                                                                                               \
    hipLaunchKernelGGL((k_wfa_lds<TT, true, false>), dim3(nslots), dim3(TT), lds, s, S, O, P, Wk, L);  \
  else                                                                                                 \
    hipLaunchKernelGGL((k_wfa_lds<TT, false, false>), dim3(nslots), dim3(TT), lds, s, S, O, P, Wk, L);
  switch (threads) {
    case 64: AIM_LAUNCH_LDS(64) break;
    case 128: AIM_LAUNCH_LDS(128) break;
    case 256: AIM_LAUNCH_LDS(256) break;
    case 512: AIM_LAUNCH_LDS(512) break;
    default: return hipErrorInvalidValue;
  }
#undef AIM_LAUNCH_LDS
  return hipGetLastError();
}

}  // namespace aim
