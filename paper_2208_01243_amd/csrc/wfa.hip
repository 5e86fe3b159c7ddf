// Gap-affine wavefront alignment (WFA): the diagonals of each wavefront spread
// over the lanes of one wavefront (k_wfa_score16) or of a workgroup (wide
// pairs, k_wfa_score).
//
// Paper: System and Methods, "Wavefront Algorithm (WFA)": successive
// furthest-reaching wavefronts, one per score s, each computed from the
// components of a few earlier wavefronts, until the end cell is reached; the
// components are allocated dynamically as they grow (Data Management: the
// per-thread bump allocator, here a per-pair arena with a bump pointer in the
// fallback pass).  The recurrences, restated on offsets j along diagonals
// k = j - i, are
//   I_s[k] = max(M_{s-o-e}[k+1], I_{s-e}[k+1])         (consumes P)
//   D_s[k] = max(M_{s-o-e}[k-1], D_{s-e}[k-1]) + 1     (consumes T)
//   M_s[k] = max(M_{s-x}[k] + 1, I_s[k], D_s[k])
// with every candidate that leaves the table (j > n or j - k > m) dropped,
// then each M_s[k] extended along matching bases.  M_0[0] = extend(0); the
// first s with M_s[n-m] >= n is the optimum; with a threshold the search stops
// (rejected) once s exceeds it.
//
// The score passes keep the last R = max(x, o+e) + 1 wavefronts in a ring (the
// oldest source is s - max(x, o+e)) and, when a CIGAR is wanted, 4 bits per
// cell recording how each component got its value (see walk_codes below).
// After the end cell is reached the pass walks those codes itself: from M emit
// the '=' run, then the first of X, I, D whose candidate attains the
// pre-extension offset; from I (D) prefer the opening source M_{s-o-e} over
// extension.  This reproduces the DP oracle's canonical CIGAR (same tie
// order).  Pairs whose codes do not fit their slot take the fallback pass
// (k_wfa_trace), which recomputes s = 0..score keeping every wavefront's
// offsets and walks those.
#include <algorithm>

#include "aim_internal.h"

namespace aim {
namespace {

#include "wfa_common.h"

// One wavefront step: compute components of score s into `dst` (three
// arrays of width hi-lo+1 at dst, dst+w, dst+2w).  Source tables/arrays are
// located through `tab`/`store` with slot(s') giving the table slot.
// Returns present bits of the new wavefront (0: null) and its lo/hi.
// Element type of a stored wavefront component: int32, or int16 when every
// offset fits (absent entries then read as -1; every reader treats negative
// values as absent).  Bases in tables are in 32-bit words.
template <class E>
__device__ __forceinline__ E wf_put(int32_t v) {
  return sizeof(E) == 4 ? (E)v : (E)(v < 0 ? -1 : v);
}
template <class E>
__device__ __forceinline__ int32_t wf_words(int32_t elems) {
  return sizeof(E) == 4 ? elems : (elems + 1) / 2;
}

// CLAMP: clamp every source index into its array.  Without it, an index may
// reach up to wlimit + 2 entries before a source array's start and up to
// 3 wlimit + blockDim.x + 2 past it; the caller guarantees that memory (an HBM
// ring padded by wfa_ring_pad(wcap) words at both ends), and a value read there is
// never used (each is taken only under its source's range test).
template <class E, bool CLAMP = true, class Q, class SlotOf>
__device__ __forceinline__ int wf_step(int32_t s, int32_t x, int32_t oe, int32_t e, int32_t m,
                                       int32_t n, const int32_t *tab, const int32_t *store,
                                       SlotOf slot_of, int32_t *dst_base_store, int32_t dst_base,
                                       int32_t wlimit, int32_t &lo_out, int32_t &hi_out,
                                       const Q &q, bool &overflow, uint8_t *crow = nullptr,
                                       int64_t cavail = 0, int32_t *cbytes = nullptr) {
  const int lane = threadIdx.x;
  int sx = -1, so = -1, se = -1;
  int fx = 0, fo = 0, fe = 0;
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  if (s - x >= 0) {
    sx = slot_of(s - x);
    fx = tab_get(tab, sx, 3) & 1;
    if (fx) { lo = min(lo, tab_get(tab, sx, 0)); hi = max(hi, tab_get(tab, sx, 1)); }
  }
  if (s - oe >= 0) {
    so = slot_of(s - oe);
    fo = tab_get(tab, so, 3) & 1;
    if (fo) { lo = min(lo, tab_get(tab, so, 0)); hi = max(hi, tab_get(tab, so, 1)); }
  }
  if (s - e >= 0) {
    se = slot_of(s - e);
    fe = tab_get(tab, se, 3) & 6;
    if (fe) { lo = min(lo, tab_get(tab, se, 0)); hi = max(hi, tab_get(tab, se, 1)); }
  }
  if (!fx && !fo && !fe) return 0;
  lo = max(lo - 1, -m);
  hi = min(hi + 1, n);
  if (lo > hi) return 0;
  const int32_t w = hi - lo + 1;
  if (w > wlimit) {
    overflow = true;
    return 0;
  }
  // origin codes of this score into crow (ceil(w / 2) bytes) when they fit
  if (crow) {
    if ((w + 1) / 2 > cavail) {
      crow = nullptr;
      *cbytes = -1;
    } else {
      *cbytes = (w + 1) / 2;
    }
  }
  const int32_t xlo = fx ? tab_get(tab, sx, 0) : 0, xhi = fx ? tab_get(tab, sx, 1) : -1;
  const int32_t xb = fx ? tab_get(tab, sx, 2) : 0;
  const int32_t olo = fo ? tab_get(tab, so, 0) : 0, ohi = fo ? tab_get(tab, so, 1) : -1;
  const int32_t ob = fo ? tab_get(tab, so, 2) : 0;
  const int32_t elo = fe ? tab_get(tab, se, 0) : 0, ehi = fe ? tab_get(tab, se, 1) : -1;
  const int32_t eb = fe ? tab_get(tab, se, 2) : 0, ew = ehi - elo + 1;
  const bool eI = fe & 2, eD = fe & 4;
  E *dM = reinterpret_cast<E *>(dst_base_store + dst_base);
  E *dI = dM + w;
  E *dD = dI + w;
  const E *so_ = reinterpret_cast<const E *>(store + ob);
  const E *se_ = reinterpret_cast<const E *>(store + eb);
  const E *sx_ = reinterpret_cast<const E *>(store + xb);
  // Source reads are issued for U diagonals per lane before any of them is
  // extended, so that up to 5 U loads are in flight.  Each index is clamped
  // into its source array (an absent source has base 0 and reads element 0 of
  // the store), and a value is used only under the bounds test of its source.
  constexpr int U = 4;
  const int32_t owm = max(ohi - olo, 0), ewm = max(ew - 1, 0), xwm = max(xhi - xlo, 0);
  const uint32_t ow = fo ? (uint32_t)(ohi - olo + 1) : 0u, xw = fx ? (uint32_t)(xhi - xlo + 1) : 0u;
  const uint32_t iw = eI ? (uint32_t)ew : 0u, dw = eD ? (uint32_t)ew : 0u;
  const int32_t nt = (int32_t)blockDim.x;
  for (int32_t kb = lo; kb <= hi; kb += U * nt) {  // kb: uniform batch start
    int32_t a_ou[U], a_ie[U], a_od[U], a_de[U], a_x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a_ou[u] = a_ie[u] = a_od[u] = a_de[u] = a_x[u] = NEG;
      if (kb + u * nt <= hi) {
        const int32_t k = kb + u * nt + lane;
        if (CLAMP) {
          a_ou[u] = so_[min(max(k + 1 - olo, 0), owm)];
          a_ie[u] = se_[ew + min(max(k + 1 - elo, 0), ewm)];
          a_od[u] = so_[min(max(k - 1 - olo, 0), owm)];
          a_de[u] = se_[2 * ew + min(max(k - 1 - elo, 0), ewm)];
          a_x[u] = sx_[min(max(k - xlo, 0), xwm)];
        } else {
          a_ou[u] = so_[k + 1 - olo];
          a_ie[u] = se_[ew + (k + 1 - elo)];
          a_od[u] = so_[k - 1 - olo];
          a_de[u] = se_[2 * ew + (k - 1 - elo)];
          a_x[u] = sx_[k - xlo];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t k = kb + u * nt + lane;
      if (kb + u * nt > hi) continue;  // (uniform) no diagonal of this row in range
      // Selects rather than branches: every range test is one unsigned
      // compare against a width that is 0 for an absent source, and a
      // candidate is dropped (NEG) unless it lies in the table.
      const int32_t vi0 = max((uint32_t)(k + 1 - olo) < ow ? a_ou[u] : NEG,
                              (uint32_t)(k + 1 - elo) < iw ? a_ie[u] : NEG);
      const int32_t vi = ((vi0 >= 0) & (vi0 - k <= m)) ? vi0 : NEG;
      const int32_t vd0 = max((uint32_t)(k - 1 - olo) < ow ? a_od[u] : NEG,
                              (uint32_t)(k - 1 - elo) < dw ? a_de[u] : NEG);
      const int32_t vd = ((vd0 >= 0) & (vd0 < n)) ? vd0 + 1 : NEG;
      const int32_t vx0 = (uint32_t)(k - xlo) < xw ? a_x[u] : NEG;
      const int32_t vx = ((vx0 >= 0) & (vx0 < n) & (vx0 + 1 - k <= m)) ? vx0 + 1 : NEG;
      int32_t vm = max(vx, max(vi, vd));
      if (crow) {
        // every lane of the row takes part (k - lo has the parity of the lane)
        const uint8_t b = code_pair(origin_code_of(
            vx, vi, vd, vm, (vi >= 0) & ((uint32_t)(k + 1 - olo) < ow) & (a_ou[u] == vi),
            (vd >= 0) & ((uint32_t)(k - 1 - olo) < ow) & (a_od[u] >= 0) & (a_od[u] + 1 == vd)));
        if (!(lane & 1) && k <= hi) crow[(k - lo) >> 1] = b;
      }
      vm = q.ext_all(m, n, k, vm);
      if (k <= hi) {
        dM[k - lo] = wf_put<E>(vm);
        dI[k - lo] = wf_put<E>(vi);
        dD[k - lo] = wf_put<E>(vd);
      }
    }
  }
  lo_out = lo;
  hi_out = hi;
  return 1 | ((fo || eI) ? 2 : 0) | ((fo || eD) ? 4 : 0);
}

// ------------------------------------------------ score pass, wide pairs
// RING_LDS: the ring lives in dynamic LDS, else in the HBM slot of this
// workgroup (a compile-time choice, so that each is reached with its own
// instructions rather than generic ones).
// E: element type of the ring (int16 when every offset of the batch fits).
template <bool RING_LDS, class E>
__global__ __launch_bounds__(WGMAX) __attribute__((amdgpu_waves_per_eu(7)))
void k_wfa_score(Seqs S, Outs O, Scoring P, Work Wk, WfaLaunch L, int32_t *hbm) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t sh_pair;
  const int lane = threadIdx.x;
  uint64_t *sP = (uint64_t *)smem;
  uint64_t *sT = sP + L.seq_words;
  int32_t *tab_ring = (int32_t *)(sT + L.seq_words);       // R entries
  int32_t *lds_ring = tab_ring + L.R * ENTRY;
  int32_t *ring = RING_LDS ? lds_ring : (hbm + (int64_t)blockIdx.x * L.slot_words);
  const int32_t slot_w = wf_words<E>(3 * L.wcap);  // words per ring slot
  const int32_t x = P.x, oe = P.o + P.e, e = P.e, R = L.R;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x * 1 >= count) return;
  for (;;) {
    __syncthreads();
    if (lane == 0) sh_pair = atomicAdd(Wk.counter, 1);
    __syncthreads();
    const int64_t li = sh_pair;
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)Wk.idx[li] : li;
    if (O.flags && O.flags[p]) {
      if (lane == 0) { O.score[p] = -1; O.status[p] = ST_INVALID; O.nruns[p] = 0; }
      continue;
    }
    const int32_t m = S.pat_len[p], n = S.txt_len[p];
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    const uint64_t *gP = S.pat + S.pat_off[p], *gT = S.txt + S.txt_off[p];
    const bool staged = pnw <= L.seq_words && tnw <= L.seq_words;
    if (staged) {
      stage_seq(sP, gP, pnw);
      stage_seq(sT, gT, tnw);
    }
    __syncthreads();
    auto slot_of = [&](int32_t s) { return s % R; };
    int32_t s = 0;
    int64_t need = 0;
    int result = 0;  // 1 aligned, 2 rejected, 3 ring overflow, 4 internal bound
    // origin codes for the fused walk: per score its range and code offset in
    // wtab, the codes in wcodes; `keep` drops to false once they do not fit
    bool keep = P.want_cigar && L.walk_steps > 0, walked = false;
    int32_t *wtab = reinterpret_cast<int32_t *>(L.walk + (int64_t)blockIdx.x * L.walk_slot);
    uint8_t *wcodes = reinterpret_cast<uint8_t *>(wtab + 4 * (int64_t)L.walk_steps);
    uint32_t *wtok = reinterpret_cast<uint32_t *>(wcodes + L.walk_codes);
    int64_t cbase = 0;
    const int32_t kend = n - m;
    // the cost of one concrete alignment bounds the optimum: all diagonal ops
    // plus one gap run for the length difference, or gap runs over both
    const int64_t ad = m > n ? m - n : n - m;
    const int64_t up1 = (int64_t)x * min(m, n) + (ad ? (int64_t)P.o + ad * e : 0);
    const int64_t up2 = (m ? (int64_t)P.o + (int64_t)m * e : 0) + (n ? (int64_t)P.o + (int64_t)n * e : 0);
    const int64_t s_upper = min(up1, up2);
    // the score loop, once per way of reading the sequences
    auto run = [&](const auto &q) {
    for (;; ++s) {
      if (P.max_score >= 0 && s > P.max_score) { result = 2; break; }
      if (s > s_upper) { result = 4; break; }
      const int sl = slot_of(s);
      int32_t lo = 0, hi = -1;
      int present;
      bool overflow = false;
      if (s == 0) {
        if (lane == 0) reinterpret_cast<E *>(ring + sl * slot_w)[0] = wf_put<E>(q.ext(m, n, 0, 0));
        present = 1;
        lo = hi = 0;
      } else {
        if (keep && s >= L.walk_steps) keep = false;
        int32_t cbytes = 0;
        present = wf_step<E, RING_LDS>(s, x, oe, e, m, n, tab_ring, ring, slot_of, ring, sl * slot_w, L.wcap,
                                   lo, hi, q, overflow, keep ? wcodes + cbase : nullptr,
                                   L.walk_codes - cbase, &cbytes);
        if (cbytes < 0) keep = false;
        cbase += cbytes > 0 ? cbytes : 0;
      }
      if (overflow) { result = 3; break; }
      __syncthreads();
      if (lane == 0) {
        tab_ring[sl * ENTRY + 0] = lo;
        tab_ring[sl * ENTRY + 1] = hi;
        tab_ring[sl * ENTRY + 2] = sl * slot_w;
        tab_ring[sl * ENTRY + 3] = present;
        if (keep) {
          wtab[4 * s + 0] = lo;
          wtab[4 * s + 1] = present ? hi : lo - 1;
          wtab[4 * s + 2] = (int32_t)(cbase - (present && s > 0 ? (hi - lo + 2) / 2 : 0));
        }
      }
      if (present) {
        const int64_t w3 = 3 * (int64_t)(hi - lo + 1);
        need += ENTRY + (L.store16 ? (w3 + 1) / 2 : w3);
      } else {
        need += ENTRY;
      }
      __syncthreads();
      if (present && kend >= lo && kend <= hi &&
          (int32_t)reinterpret_cast<const E *>(ring + sl * slot_w)[kend - lo] >= n) {
        result = 1;
        break;
      }
    }
    if (result == 1 && keep) {
      // the codes and table of every wave visible to the walk: the barrier
      // orders the stores, the agent-scope acquire drops L1 lines an earlier
      // pair's walk may have left at these addresses
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (threadIdx.x < 64) {
        const int32_t sfin = s;
        auto code_at = [&](int32_t cs, int32_t k) -> int32_t {  // per lane
          if (cs < 1 || cs > sfin) return -1;
          const int32_t lo = wtab[4 * cs + 0], hi = wtab[4 * cs + 1], cb = wtab[4 * cs + 2];
          if (k < lo || k > hi) return -1;
          const uint32_t b = wcodes[cb + ((k - lo) >> 1)];
          return (int32_t)(((k - lo) & 1) ? (b >> 4) : (b & 15u));
        };
        auto ext = [&](int32_t k, int32_t f) { return q.ext_wave(m, n, k, f); };
        walked = walk_codes<true>(O, p, code_at, ext, x, oe, e, m, n, s, wtok, L.walk_tok);
        if (!walked && threadIdx.x == 0 && L.walk_fail) atomicAdd(L.walk_fail, 1);
      }
      __syncthreads();
    } else if (result == 1 && P.want_cigar && lane == 0 && L.walk_skip) {
      atomicAdd(L.walk_skip, 1);  // codes not kept: the full-store pass walks it
    }
    };
    if (staged)
      run(SeqStaged{reinterpret_cast<const uint32_t *>(sP), reinterpret_cast<const uint32_t *>(sT)});
    else
      run(SeqInPlace{gP, gT, pnw, tnw});
    if (result == 3) {
      wave_append1(true, (int32_t)p, L.ring_list, L.ring_count);
      continue;
    }
    if (lane == 0) {
      if (result == 2 || result == 4) {
        O.score[p] = -1;
        O.status[p] = result == 2 ? ST_REJECTED : ST_INVALID;
        O.nruns[p] = 0;
      } else {
        O.score[p] = s * P.unit;
        O.status[p] = ST_ALIGNED;
        if (!walked) O.nruns[p] = 0;
        if (P.want_cigar && !walked) {
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
}

// -------------------------------------------- score pass, one wavefront per pair
// The wavefronts of k_wfa_score (same recurrences, bounds, presence bits and
// full-store size), computed by a single 64-lane wavefront with no barrier
// between waves: lane l owns diagonals kbase + l + 64 c for c < C, kbase =
// -32 C.  M of the last R scores and I, D of the last e + 1 live in LDS as
// 16-bit offsets (INT16_MIN: absent), the per-score bounds and presence bits
// in an R-entry LDS table; a source entry is read only inside that wavefront's
// bounds, so stale slots never leak.  A wavefront that leaves the window goes
// to the HBM-ring pass (ring_list), as does a pair whose end diagonal lies
// outside it.  The host sends only batches with max_len <= WFA16_MAX_LEN (so
// offsets fit 16 bits) whose sequences fit the LDS staging area.
__global__ __launch_bounds__(64) void k_wfa_score16(Seqs S, Outs O, Scoring P, Work Wk, WfaLaunch L,
                                                   int32_t C) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int32_t x = P.x, oe = P.o + P.e, e = P.e, R = L.R, RE = P.e + 1;
  const int32_t W = 64 * C, kbase = -32 * C;
  // ring rows and code rows carry 64 entries / 32 bytes of padding past the
  // window, where the lanes of a chunk that runs past it write unmasked
  const int32_t WS = W + 64, BR = C * 32 + 32;
  uint64_t *sP = (uint64_t *)smem;
  uint64_t *sT = sP + L.seq_words;
  // per ring slot, the diagonal range of each component (empty when the
  // component is absent): I lo, hi, D lo, hi, M lo, hi, -, -
  int32_t *tab = (int32_t *)(sT + L.seq_words);
  int16_t *rM = (int16_t *)(tab + R * TAB16);     // R x WS
  int16_t *rI = rM + R * WS;                       // (e+1) x WS
  int16_t *rD = rI + RE * WS;                      // (e+1) x WS
  const int32_t count = Wk.count ? __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)Wk.count)
                                 : (int32_t)Wk.n;
  if ((int32_t)blockIdx.x >= count) return;
  // Control flow is kept provably uniform (scalar values, no lane-dependent
  // branch around the work counter, one loop latch, no continue).  With a
  // lane-0-only atomic and a loop exit the compiler took for divergent, it
  // split the loop so that lanes 1..63 looped back to the broadcast without a
  // new index.  Every lane adds here (lane 0 one, the others zero), and lane
  // 0's return value is the item.
  for (;;) {
    const int32_t t = atomicAdd(Wk.counter, lane == 0 ? 1 : 0);
    const int32_t li = __builtin_amdgcn_readfirstlane(t);
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)__builtin_amdgcn_readfirstlane(Wk.idx[li]) : li;
    const bool invalid = O.flags && __builtin_amdgcn_readfirstlane((int32_t)O.flags[p]);
    if (invalid) {
      if (lane == 0) { O.score[p] = -1; O.status[p] = ST_INVALID; O.nruns[p] = 0; }
    } else {
    const int32_t m = __builtin_amdgcn_readfirstlane(S.pat_len[p]);
    const int32_t n = __builtin_amdgcn_readfirstlane(S.txt_len[p]);
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    __syncthreads();  // the previous pair's LDS is no longer read
    // the host sends only batches whose sequences fit the staging area
    stage_seq(sP, S.pat + S.pat_off[p], pnw);
    stage_seq(sT, S.txt + S.txt_off[p], tnw);
    const uint32_t *P32 = reinterpret_cast<const uint32_t *>(sP);
    const uint32_t *T32 = reinterpret_cast<const uint32_t *>(sT);
    __syncthreads();  // staged words visible to every lane
    const int32_t kend = n - m;
    const int32_t bits_steps = P.want_cigar ? L.bits_steps : 0;
    uint8_t *bslot = L.bits + (int64_t)blockIdx.x * bits_steps * BR;
    const int64_t ad = m > n ? m - n : n - m;
    const int64_t up1 = (int64_t)x * min(m, n) + (ad ? (int64_t)P.o + ad * e : 0);
    const int64_t up2 = (m ? (int64_t)P.o + (int64_t)m * e : 0) + (n ? (int64_t)P.o + (int64_t)n * e : 0);
    const int32_t s_upper = (int32_t)min<int64_t>(min(up1, up2), INT32_MAX - 1);
    // one test per score: past s_lim the pair is rejected (threshold) or
    // out of its bound
    const int32_t s_lim = P.max_score >= 0 ? min(P.max_score, s_upper) : s_upper;
    int result = (kend < kbase || kend >= kbase + W) ? 3 : 0;  // 1 aligned, 2 rejected, 3 overflow, 4 bound
    int32_t s = 0;
    int64_t need = 0;
    if (!result) {
      // every slot starts empty, so a source of negative score (a slot not
      // yet written for this pair, as R > max(x, o + e)) contributes nothing
      if (lane < R) {
        int32_t *t = tab + lane * TAB16;
        t[0] = EMPTY_LO; t[1] = EMPTY_HI; t[2] = EMPTY_LO; t[3] = EMPTY_HI; t[4] = EMPTY_LO; t[5] = EMPTY_HI;
      }
      if (lane == 0) {
        const int32_t f = extend_lds(P32, m, T32, n, 0, 0);
        rM[0 - kbase] = (int16_t)f;
        tab[4] = 0;
        tab[5] = 0;
      }
      need = ENTRY + 2;  // s = 0: three 16-bit entries
      __syncthreads();
      if (kend == 0 && __builtin_amdgcn_readfirstlane((int32_t)rM[0 - kbase]) >= n) result = 1;
    }
    // ring slots kept incrementally: sl = s mod R, sE = s mod (e + 1)
    int32_t sl = 0, sE = 0;
    while (!result) {
      ++s;
      if (s > s_lim) { result = (P.max_score >= 0 && s > P.max_score) ? 2 : 4; break; }
      sl = sl + 1 == R ? 0 : sl + 1;
      sE = sE + 1 == RE ? 0 : sE + 1;
      const int32_t qx = sl >= x ? sl - x : sl - x + R;
      const int32_t qo = sl >= oe ? sl - oe : sl - oe + R;
      const int32_t qe = sl >= e ? sl - e : sl - e + R;
      const int32_t qeE = sE + 1 == RE ? 0 : sE + 1;  // (s - e) mod (e + 1)
      // the source ranges: M of s - x and s - o - e, I and D of s - e
      const int32_t xlo = __builtin_amdgcn_readfirstlane(tab[qx * TAB16 + 4]);
      const int32_t xhi = __builtin_amdgcn_readfirstlane(tab[qx * TAB16 + 5]);
      const int32_t olo = __builtin_amdgcn_readfirstlane(tab[qo * TAB16 + 4]);
      const int32_t ohi = __builtin_amdgcn_readfirstlane(tab[qo * TAB16 + 5]);
      const int32_t ilo = __builtin_amdgcn_readfirstlane(tab[qe * TAB16 + 0]);
      const int32_t ihi = __builtin_amdgcn_readfirstlane(tab[qe * TAB16 + 1]);
      const int32_t dlo = __builtin_amdgcn_readfirstlane(tab[qe * TAB16 + 2]);
      const int32_t dhi = __builtin_amdgcn_readfirstlane(tab[qe * TAB16 + 3]);
      const int32_t bx = qx * WS, bo = qo * WS, beI = qeE * WS;
      const int32_t lo = max(min(min(xlo, olo), min(ilo, dlo)) - 1, -m);
      const int32_t hi = min(max(max(xhi, ohi), max(ihi, dhi)) + 1, n);
      const bool present = lo <= hi;
      if (present && (lo < kbase || hi >= kbase + W)) { result = 3; break; }
      // range widths (0 when empty): a range test is one unsigned compare
      const int32_t xw = max(xhi - xlo + 1, 0), ow = max(ohi - olo + 1, 0);
      const int32_t iw = max(ihi - ilo + 1, 0), dw = max(dhi - dlo + 1, 0);
      const bool hasI = present && (ow | iw), hasD = present && (ow | dw);
      bool hit = false;  // this lane reached the end cell
      const bool keep = s < bits_steps;  // origin codes of this score kept
      if (present) {
        const int32_t bM = sl * WS, bID = sE * WS;
        // Chunks of 64 diagonals slide with the wavefront: the first starts
        // at lo (rounded down to even, so that lanes 2q, 2q+1 share a code
        // byte), which makes a wavefront of w diagonals cost ceil(w / 64)
        // chunks wherever it lies in the window.  Every lane of a chunk runs
        // the same code: a diagonal outside [lo, hi] finds no source in range
        // (or only candidates the table bounds drop), so its offset comes out
        // absent and it writes the absent mark into a part of the slot no
        // reader takes; lanes past the window's end write into the padding.
        const int32_t start = (lo - kbase) & ~1, nch = ((hi - kbase - start) >> 6) + 1;
        for (int32_t c = 0; c < nch; ++c) {
          const int32_t idx = start + 64 * c + lane, k = kbase + idx;
          // five source reads issued together, indices clamped into the window
          const int32_t up = min(idx + 1, W - 1), dn = min(max(idx - 1, 0), W - 1), ix = min(idx, W - 1);
          const int32_t a_ou = rM[bo + up], a_od = rM[bo + dn], a_x = rM[bx + ix];
          const int32_t a_iu = rI[beI + up], a_dd = rD[beI + dn];
          // absent entries are stored as exactly INT16_MIN, so one added
          // base keeps them negative
          int32_t vi = max((uint32_t)(k + 1 - olo) < (uint32_t)ow ? a_ou : NEG,
                           (uint32_t)(k + 1 - ilo) < (uint32_t)iw ? a_iu : NEG);
          if (vi - k > m) vi = NEG;
          int32_t vd = max((uint32_t)(k - 1 - olo) < (uint32_t)ow ? a_od : NEG,
                           (uint32_t)(k - 1 - dlo) < (uint32_t)dw ? a_dd : NEG) + 1;
          if (vd > n) vd = NEG;
          int32_t vx = ((uint32_t)(k - xlo) < (uint32_t)xw ? a_x : NEG) + 1;
          if (vx > n || vx - k > m) vx = NEG;
          int32_t vm = max(vx, max(vi, vd));
          if (keep) {
            // origin code of this cell; lanes 2q and 2q+1 share byte q
            const int32_t code = origin_code_of(
                vx, vi, vd, vm, vi >= 0 && (uint32_t)(k + 1 - olo) < (uint32_t)ow && a_ou == vi,
                vd >= 0 && (uint32_t)(k - 1 - olo) < (uint32_t)ow && a_od >= 0 && a_od + 1 == vd);
            const uint8_t b = code_pair(code);
            // odd lanes (and lanes past the window) write into the row's padding
            bslot[(int64_t)s * BR + ((lane & 1) ? BR - 1 : (idx >> 1))] = b;
          }
          // extend: the first 16 bases by every lane without a branch (a lane
          // with no offset compares at base 0 under a zero limit), the rest
          // only where all 16 matched
          const bool live = vm >= 0;
          const int32_t i0 = live ? vm - k : 0, j0 = live ? vm : 0;
          const int32_t lim = live ? min(m - i0, n - j0) : 0;
          const uint32_t d = __builtin_amdgcn_alignbit(P32[(i0 >> 4) + 1], P32[i0 >> 4], (uint32_t)(i0 & 15) * 2) ^
                             __builtin_amdgcn_alignbit(T32[(j0 >> 4) + 1], T32[j0 >> 4], (uint32_t)(j0 & 15) * 2);
          const int32_t run = min(d ? (int32_t)(__builtin_ctz(d) >> 1) : 16, lim);
          int32_t f = j0 + run;
          if (run == 16) f = extend_lds(P32, m, T32, n, k, f);
          if (live) vm = f;
          rM[bM + idx] = (int16_t)(vm < 0 ? -32768 : vm);
          rI[bID + idx] = (int16_t)(vi < 0 ? -32768 : vi);
          rD[bID + idx] = (int16_t)(vd < 0 ? -32768 : vd);
          hit = hit || (k == kend && vm >= n);
        }
      }
      if (lane == 0) {
        int32_t *t = tab + sl * TAB16;
        t[0] = hasI ? lo : EMPTY_LO;
        t[1] = hasI ? hi : EMPTY_HI;
        t[2] = hasD ? lo : EMPTY_LO;
        t[3] = hasD ? hi : EMPTY_HI;
        t[4] = present ? lo : EMPTY_LO;
        t[5] = present ? hi : EMPTY_HI;
      }
      need += ENTRY + (present ? (3 * (int64_t)(hi - lo + 1) + 1) / 2 : 0);  // 16-bit store
      __syncthreads();
      if (__ballot(hit)) result = 1;
    }
    bool walked = false;
    if (result == 1 && s < bits_steps) {
      // The codes were stored by this wavefront's lanes; the walk reads them
      // back, among addresses whose earlier contents (an earlier pair's
      // codes) this workgroup's loads may have left in the CU's vector L1.
      // The barrier orders the stores before the loads; the agent-scope
      // acquire invalidates the L1 so that no load hits such a line.
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int32_t sfin = s;
      auto code_at = [&](int32_t cs, int32_t k) -> int32_t {  // per lane
        const int32_t idx = k - kbase;
        if (cs < 1 || cs > sfin || (uint32_t)idx >= (uint32_t)W) return -1;
        const uint32_t b = bslot[(int64_t)cs * BR + (idx >> 1)];
        return (int32_t)((idx & 1) ? (b >> 4) : (b & 15u));
      };
      auto ext = [&](int32_t k, int32_t f) { return extend_wave(P32, m, T32, n, k, f); };
      walked = walk_codes<false>(O, p, code_at, ext, x, oe, e, m, n, s, reinterpret_cast<uint32_t *>(rM),
                          (R + 2 * RE) * WS / 2);
      if (!walked && lane == 0 && L.walk_fail) atomicAdd(L.walk_fail, 1);
    } else if (result == 1 && P.want_cigar && lane == 0 && L.walk_skip) {
      atomicAdd(L.walk_skip, 1);  // codes not kept: the full-store pass walks it
    }
    if (result == 3) {
      if (L.route.nclass > 0) {
        // the furthest anti-diagonal any kept M offset reaches, for the
        // prediction of the window this pair needs
        const bool kend_out = kend < kbase || kend >= kbase + W;  // left before any score
        int32_t prog = 0;
        for (int32_t t = 0; t < (kend_out ? 0 : R); ++t) {
          const int32_t tlo = __builtin_amdgcn_readfirstlane(tab[t * TAB16 + 4]);
          const int32_t thi = __builtin_amdgcn_readfirstlane(tab[t * TAB16 + 5]);
          for (int32_t k = tlo + lane; k <= thi; k += 64) {
            const int32_t f = rM[t * WS + (k - kbase)];
            if (f >= 0) prog = max(prog, 2 * f - k);
          }
        }
        prog = wave_max_i32(prog);
        const int32_t ext = kend_out ? max(-kend, kend + 1) : W / 2 + 1;
        if (lane == 0) route_pair(L.route, 0, p, predict_extent(ext, prog, m, n));
      } else {
        wave_append1(true, (int32_t)p, L.ring_list, L.ring_count);
      }
    } else if (lane == 0) {
      if (result == 2 || result == 4) {
        O.score[p] = -1;
        O.status[p] = result == 2 ? ST_REJECTED : ST_INVALID;
        O.nruns[p] = 0;
      } else {
        O.score[p] = s * P.unit;
        O.status[p] = ST_ALIGNED;
        if (!walked) O.nruns[p] = 0;
        if (P.want_cigar && !walked) {
          L.need[p] = need;
          int cl = 0;
          while (cl < 3 && need > L.need_cap[cl]) ++cl;
          if (need > L.need_cap[3]) {
            to_long_pass(O, p, L.long_list, L.long_count);
          } else {
            const int32_t k = atomicAdd(L.need_count[cl], 1);
            L.need_list[cl][k] = (int32_t)p;
            atomicMax(L.need_max[cl], (int32_t)need);
          }
        }
      }
    }
    }  // valid pair
  }
}

// ----------------------------------------------- fallback: full-store walk
// LDSA: the full store lives in this workgroup's LDS (else in its HBM slot);
// a compile-time choice, so that LDS traffic is issued as LDS instructions.
template <class E, bool LDSA>
__global__ __launch_bounds__(WGMAX) void k_wfa_trace(Seqs S, Outs O, Scoring P, Work Wk, WfaLaunch L,
                                                  int32_t *hbm) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t sh_pair, sh_top;
  const int lane = threadIdx.x;
  uint64_t *sP = (uint64_t *)smem;
  uint64_t *sT = sP + L.seq_words;
  const int32_t x = P.x, o = P.o, oe = P.o + P.e, e = P.e;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // HBM slots sized by the largest full store of this launch's pairs: as many
  // workgroups take pairs as such slots fit the pool (at least one, since the
  // pool holds the class capacity)
  int64_t slot_words = L.slot_words, nslots = gridDim.x;
  if (!LDSA && L.slot_need_max) {
    const int64_t mx = *(volatile const int32_t *)L.slot_need_max;
    slot_words = (max<int64_t>(mx, 1) + 63) / 64 * 64;
    nslots = min<int64_t>(nslots, L.pool_words / slot_words);
  }
  // a workgroup the work can never reach, or without a slot, leaves before
  // touching the counter
  if ((int64_t)blockIdx.x >= min<int64_t>(count, nslots)) return;
  int32_t *arena = LDSA ? (int32_t *)(sT + L.seq_words) : (hbm + (int64_t)blockIdx.x * slot_words);
  // With the store in HBM, the entries of the last R scores are also kept in
  // an LDS ring, from which the steps read their sources; the full table in
  // HBM serves the backtrace.
  constexpr bool ring = !LDSA;
  const int32_t R = L.R;
  int32_t *tab_ring = (int32_t *)(sT + L.seq_words);
  for (;;) {
    __syncthreads();
    if (lane == 0) sh_pair = atomicAdd(Wk.counter, 1);
    __syncthreads();
    const int64_t li = sh_pair;
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)Wk.idx[li] : li;
    const int32_t m = S.pat_len[p], n = S.txt_len[p];
    const int32_t sfin = O.score[p] / P.unit;
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    const uint64_t *gP = S.pat + S.pat_off[p], *gT = S.txt + S.txt_off[p];
    const bool staged = pnw <= L.seq_words && tnw <= L.seq_words;
    if (staged) {
      stage_seq(sP, gP, pnw);
      stage_seq(sT, gT, tnw);
    }
    // table of sfin + 1 entries at the start of the arena, data after it
    int32_t *tab = arena;
    const int32_t data0 = (sfin + 1) * ENTRY;
    if (lane == 0) sh_top = data0;
    __syncthreads();
    const int32_t *stab = ring ? tab_ring : tab;
    auto slot_of = [&](int32_t s2) { return ring ? s2 % R : s2; };
    // the forward steps, once per way of reading the sequences
    auto forward = [&](const auto &q) {
    for (int32_t s = 0; s <= sfin; ++s) {
      const int32_t base = sh_top;
      int32_t lo = 0, hi = -1;
      int present;
      bool overflow = false;
      if (s == 0) {
        if (lane == 0) reinterpret_cast<E *>(arena + base)[0] = wf_put<E>(q.ext(m, n, 0, 0));
        present = 1;
        lo = hi = 0;
      } else {
        present = wf_step<E>(s, x, oe, e, m, n, stab, arena, slot_of, arena, base, INT32_MAX, lo, hi,
                             q, overflow);
      }
      __syncthreads();
      if (lane == 0) {
        tab[s * ENTRY + 0] = lo;
        tab[s * ENTRY + 1] = hi;
        tab[s * ENTRY + 2] = base;
        tab[s * ENTRY + 3] = present;
        if (ring) {
          const int32_t q = s % R;
          tab_ring[q * ENTRY + 0] = lo;
          tab_ring[q * ENTRY + 1] = hi;
          tab_ring[q * ENTRY + 2] = base;
          tab_ring[q * ENTRY + 3] = present;
        }
        if (present) sh_top = base + wf_words<E>(3 * (hi - lo + 1));
      }
      __syncthreads();
    }
    };
    if (staged)
      forward(SeqStaged{reinterpret_cast<const uint32_t *>(sP), reinterpret_cast<const uint32_t *>(sT)});
    else
      forward(SeqInPlace{gP, gT, pnw, tnw});
    // ---- backtrace (one lane) ----
    if (lane == 0) {
      const int32_t total = Wk.direct ? O.nruns[p] : 0;
      uint32_t *dst = Wk.direct ? (O.cigar + O.cigar_off[p]) : nullptr;
      RunSink sink;
      sink.begin(O, p);
      uint32_t cur_op = 0xffu, cur_len = 0;
      int32_t nr = 0;
      // runs still to come are at most 2 * (score left) / min(x, o + e) + 2
      const int32_t cmin = max(1, min(x, oe));
      int32_t cs = sfin;
      auto put = [&](uint32_t op, uint32_t len) {
        if (len == 0) return;
        if (op == cur_op) {
          cur_len += len;
        } else {
          if (cur_len) {
            const uint32_t run = (cur_len << 4) | cur_op;
            if (Wk.direct) { if (nr < total) dst[total - 1 - nr] = run; }
            else sink.put(nr, run, 2 * (int64_t)(cs / cmin) + 3);
            ++nr;
          }
          cur_op = op;
          cur_len = len;
        }
      };
      auto val = [&](int32_t s2, int comp, int32_t k) -> int32_t {
        // comp 0 M, 1 I, 2 D; NEG when absent
        if (s2 < 0) return NEG;
        const int32_t lo = tab[s2 * ENTRY], hi = tab[s2 * ENTRY + 1], pr = tab[s2 * ENTRY + 3];
        if (!(pr & (1 << comp)) || k < lo || k > hi) return NEG;
        return (int32_t)reinterpret_cast<const E *>(arena + tab[s2 * ENTRY + 2])[comp * (hi - lo + 1) + (k - lo)];
      };
      int32_t k = n - m, f = n, comp = 0;
      // each step emits one op or closes a run; the walk has at most m + n ops
      int64_t guard = 2 * ((int64_t)m + n) + 8;
      while (guard-- > 0) {
        if (comp == 0) {
          if (cs == 0) {
            put(OP_EQ, (uint32_t)f);
            break;
          }
          int32_t vx = val(cs - x, 0, k);
          if (vx >= 0) { vx += 1; if (vx > n || vx - k > m) vx = NEG; } else vx = NEG;
          const int32_t vi = val(cs, 1, k), vd = val(cs, 2, k);
          const int32_t f0 = max(vx, max(vi, vd));
          if (f0 < 0) break;  // cannot happen for a reached end cell
          put(OP_EQ, (uint32_t)(f - f0));
          if (vx == f0) { put(OP_X, 1); cs -= x; f = f0 - 1; }
          else if (vi == f0) { comp = 1; f = f0; }
          else { comp = 2; f = f0; }
        } else if (comp == 1) {
          put(OP_I, 1);
          const int32_t vo = val(cs - oe, 0, k + 1);
          if (vo == f) { comp = 0; cs -= oe; } else { cs -= e; }
          k += 1;
        } else {
          put(OP_D, 1);
          const int32_t vo = val(cs - oe, 0, k - 1);
          if (vo >= 0 && vo + 1 == f) { comp = 0; cs -= oe; } else { cs -= e; }
          k -= 1;
          f -= 1;
        }
        if (cs < 0) break;
      }
      put(0xfu, 1);
      if (!Wk.direct) {
        sink.finish();
        O.nruns[p] = nr;
      }
    }
    (void)o;
  }
}


// ------------------------------------- long pairs: checkpoints and recompute
// See WfaLong.  Slot layout (int32 words): the ring (R slots of slot_w), the
// checkpoints (ck_cap of R slots of slot_w plus R table entries), the width
// of every score, the code table of one recompute (4 words per score), its
// codes (code_cap bytes), the walk tokens.
template <class E>
__global__ __launch_bounds__(WGMAX) void k_wfa_long(Seqs S, Outs O, Scoring P, Work Wk, WfaLong L) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t sh_pair, sh_res, sh_cs, sh_k, sh_comp, sh_nt, sh_wlo, sh_whi;
  const int lane = threadIdx.x;
  const int nthr = blockDim.x;
  uint64_t *sP = (uint64_t *)smem;
  uint64_t *sT = sP + L.seq_words;
  int32_t *tab_ring = (int32_t *)(sT + L.seq_words);  // R entries
  const int32_t x = P.x, oe = P.o + P.e, e = P.e, R = L.R;
  const int32_t slot_w = wf_words<E>(3 * L.wcap);
  const int64_t ckw = (int64_t)R * slot_w + (int64_t)R * ENTRY;  // words per checkpoint
  int32_t *ring = L.slots + (int64_t)blockIdx.x * L.slot_words;
  int32_t *ck = ring + (int64_t)R * slot_w;
  int32_t *wid = ck + (int64_t)L.ck_cap * ckw;
  int32_t *wtab = wid + L.sw_cap;
  uint8_t *codes = reinterpret_cast<uint8_t *>(wtab + 4 * (int64_t)L.wt_cap);
  uint32_t *tok = reinterpret_cast<uint32_t *>(codes + L.code_cap);
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a workgroup the work can never reach leaves before touching the counter
  if ((int64_t)blockIdx.x >= count) return;
  auto slot_of = [&](int32_t s2) { return s2 % R; };
  // live words of ring slot q (per its table entry)
  auto live = [&](const int32_t *tb, int32_t q) -> int32_t {
    return (tb[q * ENTRY + 3] & 7) ? wf_words<E>(3 * (tb[q * ENTRY + 1] - tb[q * ENTRY + 0] + 1)) : 0;
  };
  for (;;) {
    __syncthreads();
    if (lane == 0) sh_pair = atomicAdd(Wk.counter, 1);
    __syncthreads();
    const int64_t li = sh_pair;
    if (li >= count) break;
    const int64_t p = Wk.idx ? (int64_t)Wk.idx[li] : li;
    const int32_t m = S.pat_len[p], n = S.txt_len[p];
    const int32_t sfin = O.score[p] / P.unit;
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    const uint64_t *gP = S.pat + S.pat_off[p], *gT = S.txt + S.txt_off[p];
    const bool staged = pnw <= L.seq_words && tnw <= L.seq_words;
    if (staged) {
      stage_seq(sP, gP, pnw);
      stage_seq(sT, gT, tnw);
    }
    // no score of a slot exists before the pass fills it
    for (int32_t q = lane; q < R; q += nthr) {
      tab_ring[q * ENTRY + 0] = 0;
      tab_ring[q * ENTRY + 1] = -1;
      tab_ring[q * ENTRY + 2] = q * slot_w;
      tab_ring[q * ENTRY + 3] = 0;
    }
    const int32_t K = max(1, (sfin + L.ck_cap) / L.ck_cap);  // checkpoints at 0, K, 2K, ... (<= ck_cap)
    bool ok = sfin >= 0 && sfin < L.sw_cap;
    __syncthreads();
    // one score of the pass: into its ring slot, its table entry, and (when
    // codes_from <= s) its origin codes at *cbase with its code-table entry
    auto step = [&](const auto &q, int32_t s, int32_t codes_from, int64_t &cbase) -> bool {
      const int sl = slot_of(s);
      int32_t lo = 0, hi = -1;
      int present;
      bool overflow = false, fits = true;
      const int64_t c0 = cbase;
      if (s == 0) {
        if (lane == 0) reinterpret_cast<E *>(ring + sl * slot_w)[0] = wf_put<E>(q.ext(m, n, 0, 0));
        present = 1;
        lo = hi = 0;
      } else {
        const bool keep = s >= codes_from;
        int32_t cbytes = 0;
        present = wf_step<E>(s, x, oe, e, m, n, tab_ring, ring, slot_of, ring, sl * slot_w, L.wcap, lo, hi, q,
                             overflow, keep ? codes + cbase : nullptr, L.code_cap - cbase, &cbytes);
        if (keep) {
          if (cbytes < 0) fits = false;
          else cbase += cbytes;
        }
      }
      __syncthreads();
      if (lane == 0) {
        tab_ring[sl * ENTRY + 0] = lo;
        tab_ring[sl * ENTRY + 1] = hi;
        tab_ring[sl * ENTRY + 2] = sl * slot_w;
        tab_ring[sl * ENTRY + 3] = present;
        if (s >= codes_from && s > 0) {
          int32_t *t = wtab + 4 * (s - codes_from);
          t[0] = lo;
          t[1] = present ? hi : lo - 1;
          t[2] = (int32_t)c0;
        }
      }
      __syncthreads();
      return !overflow && fits;
    };
    // checkpoint c <-> the ring and its table (live words only)
    auto save = [&](int32_t c) {
      int32_t *dst = ck + (int64_t)c * ckw;
      for (int32_t q = 0; q < R; ++q) {
        const int32_t w = live(tab_ring, q);
        for (int32_t t = lane; t < w; t += nthr) dst[(int64_t)q * slot_w + t] = ring[(int64_t)q * slot_w + t];
      }
      for (int32_t t = lane; t < R * ENTRY; t += nthr) dst[(int64_t)R * slot_w + t] = tab_ring[t];
      __syncthreads();
    };
    auto restore = [&](int32_t c) {
      const int32_t *src = ck + (int64_t)c * ckw;
      // the agent-scope acquire drops L1 lines of these addresses that an
      // earlier recompute or pair may have left
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      for (int32_t t = lane; t < R * ENTRY; t += nthr) tab_ring[t] = src[(int64_t)R * slot_w + t];
      __syncthreads();
      for (int32_t q = 0; q < R; ++q) {
        const int32_t w = live(tab_ring, q);
        for (int32_t t = lane; t < w; t += nthr) ring[(int64_t)q * slot_w + t] = src[(int64_t)q * slot_w + t];
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    };
    auto run = [&](const auto &q) {
      // ---- the score pass: widths and checkpoints ----
      int64_t none = 0;
      for (int32_t s = 0; ok && s <= sfin; ++s) {
        if (!step(q, s, INT32_MAX, none)) ok = false;
        if (lane == 0) {
          const int32_t sl = slot_of(s);
          wid[s] = (tab_ring[sl * ENTRY + 3] & 7) ? tab_ring[sl * ENTRY + 1] - tab_ring[sl * ENTRY + 0] + 1 : 0;
        }
        if (s % K == 0) save(s / K);
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // ---- the walk, a window of recomputed codes at a time ----
      if (lane == 0) {
        sh_cs = sfin;
        sh_k = n - m;
        sh_comp = 0;
        sh_nt = 0;
        sh_wlo = 1;
        sh_whi = 0;  // no codes yet
        sh_res = ok ? 0 : -1;
      }
      __syncthreads();
      while (sh_res == 0) {
        if (lane < 64) {
          // the token walk of walk_codes, paused when it needs a score
          // outside the window (run by the first wavefront, lane 0 writes)
          int32_t cs = sh_cs, k = sh_k, comp = sh_comp, nt = sh_nt, code = -1, res = 0;
          const int32_t wlo = sh_wlo, whi = sh_whi;
          auto code_at = [&](int32_t c2, int32_t k2) -> int32_t {
            const int32_t *t = wtab + 4 * (c2 - wlo);
            const int32_t lo = t[0], hi = t[1], cb = t[2];
            if (k2 < lo || k2 > hi) return -1;
            const uint32_t b = codes[cb + ((k2 - lo) >> 1)];
            return (int32_t)(((k2 - lo) & 1) ? (b >> 4) : (b & 15u));
          };
          for (;;) {
            if (nt + 2 > L.tok_cap || cs < 0) { res = -1; break; }
            if (comp == 0) {
              if (cs == 0) {
                if (lane == 0) tok[nt] = TOK_M;
                ++nt;
                res = k == 0 ? 1 : -1;
                break;
              }
              if (cs < wlo || cs > whi) break;  // pause: codes of cs needed
              if (lane == 0) tok[nt] = TOK_M;
              ++nt;
              code = __builtin_amdgcn_readfirstlane(code_at(cs, k));
              if (code < 0) { res = -1; break; }
              const int32_t src = code & 3;
              if (src == 0) {
                if (lane == 0) tok[nt] = OP_X;
                ++nt;
                cs -= x;
                code = -1;
              } else {
                comp = src;  // I or D of the same cell
              }
            } else {
              if (code < 0) {
                if (cs < wlo || cs > whi) break;
                code = __builtin_amdgcn_readfirstlane(code_at(cs, k));
                if (code < 0) { res = -1; break; }
              }
              const bool open = (code >> (comp + 1)) & 1;
              if (lane == 0) tok[nt] = comp == 1 ? OP_I : OP_D;
              ++nt;
              k += comp == 1 ? 1 : -1;
              if (open) { cs -= oe; comp = 0; } else { cs -= e; }
              code = -1;
            }
          }
          if (lane == 0) {
            sh_cs = cs;
            sh_k = k;
            sh_comp = comp;
            sh_nt = nt;
            sh_res = res;
            if (res == 0) {
              // the next window: the checkpoint below cs, then as many of the
              // scores up to cs as the code area and table hold
              const int32_t cK = (cs - 1) / K * K;
              int32_t lo2 = cs;
              int64_t bytes = (wid[cs] + 1) / 2;
              if (bytes > L.code_cap) {
                sh_res = -1;
              } else {
                while (lo2 - 1 > cK && cs - lo2 + 2 <= L.wt_cap && bytes + (wid[lo2 - 1] + 1) / 2 <= L.code_cap) {
                  --lo2;
                  bytes += (wid[lo2] + 1) / 2;
                }
                sh_wlo = lo2;
                sh_whi = cs;
              }
            }
          }
        }
        __syncthreads();
        if (sh_res != 0) break;
        // recompute from the checkpoint below the window, keeping its codes
        const int32_t wlo = sh_wlo, whi = sh_whi, c = (wlo - 1) / K;
        restore(c);
        int64_t cbase = 0;
        bool fine = true;
        for (int32_t s = c * K + 1; s <= whi; ++s) fine = step(q, s, wlo, cbase) && fine;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!fine && lane == 0) sh_res = -1;
        __syncthreads();
      }
      // ---- forward replay and the runs ----
      if (lane < 64 && sh_res == 1) {
        auto ext = [&](int32_t k2, int32_t f) { return q.ext_wave(m, n, k2, f); };
        const int32_t total = Wk.direct ? O.nruns[p] : 0;
        uint32_t *dst = Wk.direct ? (O.cigar + O.cigar_off[p]) : nullptr;
        const bool good = replay_tokens(O, p, ext, m, n, tok, sh_nt, dst, total);
        if (!good && lane == 0) sh_res = -1;
      }
      __syncthreads();
    };
    if (staged)
      run(SeqStaged{reinterpret_cast<const uint32_t *>(sP), reinterpret_cast<const uint32_t *>(sT)});
    else
      run(SeqInPlace{gP, gT, pnw, tnw});
    if (lane == 0 && sh_res != 1) {
      O.status[p] = ST_OVERFLOW;
      if (!Wk.direct) O.nruns[p] = 0;
      if (L.failed) atomicAdd(L.failed, 1);
    }
  }
}

}  // namespace

int64_t wfa_long_slot_words(const WfaLong &L, bool i16) {
  const int64_t slot_w = i16 ? (3 * (int64_t)L.wcap + 1) / 2 : 3 * (int64_t)L.wcap;
  const int64_t ckw = (int64_t)L.R * slot_w + (int64_t)L.R * ENTRY;
  return ((int64_t)L.R * slot_w + L.ck_cap * ckw + L.sw_cap + 4 * (int64_t)L.wt_cap + L.code_cap / 4 +
          L.tok_cap + 63) / 64 * 64;
}

hipError_t launch_wfa_long(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, const WfaLong &L,
                           int32_t nslots, int32_t threads, bool i16, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const size_t lds = 2 * (size_t)L.seq_words * 8 + (size_t)L.R * ENTRY * 4;
  if (i16)
    hipLaunchKernelGGL((k_wfa_long<int16_t>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L);
  else
    hipLaunchKernelGGL((k_wfa_long<int32_t>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L);
  return hipGetLastError();
}

WfaPlan wfa_plan(int32_t max_len, const Scoring &P, int64_t budget_bytes, int32_t cus, bool plain,
                 int32_t ring_kb, int32_t trace_kb, int32_t long_threads, bool strict) {
  // budget split: HBM rings 1/8, origin codes 1/4 (HBM-ring pass) and 1/16
  // (one-wavefront pass), arena classes 1/32, 1/8 and 1/4
  WfaPlan pl{};
  const int32_t oe = P.o + P.e;
  pl.R = std::max(P.x, oe) + 1;
  const int32_t c = std::min(P.x, P.e);
  int64_t w = 2 * (int64_t)max_len + 1;
  if (P.max_score >= 0) w = std::min<int64_t>(w, 2 * (int64_t)(P.max_score / c) + 3);
  pl.wcap = (int32_t)std::max<int64_t>(w, 1);
  const int64_t seqw = ((int64_t)max_len + 31) / 32;
  pl.seq_words = seqw <= 320 ? (int32_t)seqw : 0;
  const int64_t lds_score = (int64_t)ring_kb * 1024, lds_trace = (int64_t)trace_kb * 1024;
  const int64_t fixed = 2 * (int64_t)pl.seq_words * 8 + (int64_t)pl.R * ENTRY * 4;
  const int64_t wl = (lds_score - fixed) / ((int64_t)pl.R * 12);
  pl.wcap_lds = plain ? 0 : (int32_t)std::max<int64_t>(0, std::min<int64_t>(wl, pl.wcap));
  pl.lds_score_bytes = (int32_t)(fixed + (int64_t)pl.R * 3 * pl.wcap_lds * 4);
  pl.ring_slot_words = (int64_t)pl.R * 3 * pl.wcap;
  pl.ring_slots = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>((int64_t)cus * 7, budget_bytes / 8 / (pl.ring_slot_words * 4)));
  pl.ring_threads = max_len > 1024 ? long_threads : 64;
  // full-store arena classes (words): LDS, then HBM stores of up to 1 MB,
  // 16 MB and 192 MB, with wider workgroups for the larger classes
  pl.lds_arena_words = plain ? 0 : (int32_t)((lds_trace - 2 * (int64_t)pl.seq_words * 8) / 4);
  pl.need_cap[0] = pl.lds_arena_words;
  pl.need_cap[1] = (int64_t)1 << 18;
  pl.need_cap[2] = (int64_t)1 << 22;
  pl.need_cap[3] = std::max<int64_t>(pl.need_cap[2], std::min<int64_t>((int64_t)48 << 20, budget_bytes / 2 / 4));
  pl.arena_slots[0] = cus * 8;
  pl.threads[0] = 64;
  // pools: 1/32, 1/8 and 1/4 of the budget (the origin codes of the HBM-ring
  // pass take another 1/4), each at least one slot of its class capacity; the
  // workgroups that take pairs are those whose slot (the class's largest
  // store) fits the pool
  const int64_t share[4] = {0, budget_bytes / 32, budget_bytes / 8, budget_bytes / 4};
  const int64_t cap_slots[4] = {0, (int64_t)cus * 8, (int64_t)cus * 4, (int64_t)cus * 4};
  if (strict) {
    // a pair whose store passes the last class then has no CIGAR (overflow)
    for (int k = 1; k < 4; ++k)
      pl.need_cap[k] = std::max<int64_t>(64, std::min<int64_t>(pl.need_cap[k], share[k] / 4 / 64 * 64));
    for (int k = 2; k < 4; ++k) pl.need_cap[k] = std::max(pl.need_cap[k], pl.need_cap[k - 1]);
  }
  for (int k = 1; k < 4; ++k) {
    const int64_t cap = (pl.need_cap[k] + 63) / 64 * 64;
    pl.pool_words[k] = std::max<int64_t>(cap, std::min<int64_t>(share[k] / 4, cap_slots[k] * cap));
    pl.arena_slots[k] = (int32_t)cap_slots[k];
  }
  pl.threads[1] = 64;
  pl.threads[2] = long_threads;
  pl.threads[3] = long_threads;
  return pl;
}

hipError_t launch_wfa_score(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                            const WfaLaunch &L, int32_t *hbm, bool ring_in_lds, int32_t nslots,
                            int32_t threads, bool ring16, hipStream_t s) {
  const size_t lds = 2 * (size_t)L.seq_words * 8 + (size_t)L.R * ENTRY * 4 +
                     (ring_in_lds ? (size_t)L.R * 3 * L.wcap * 4 : 0);
  if (ring_in_lds)
    hipLaunchKernelGGL((k_wfa_score<true, int32_t>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
  else if (ring16)
    hipLaunchKernelGGL((k_wfa_score<false, int16_t>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
  else
    hipLaunchKernelGGL((k_wfa_score<false, int32_t>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
  return hipGetLastError();
}

size_t wfa_score16_lds(const WfaLaunch &L, int32_t e, int32_t C) {
  return 2 * (size_t)L.seq_words * 8 + (size_t)L.R * TAB16 * 4 + (size_t)(L.R + 2 * (e + 1)) * (64 * C + 64) * 2;
}

hipError_t launch_wfa_score16(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                              const WfaLaunch &L, int32_t C, int32_t nslots, hipStream_t s) {
  hipLaunchKernelGGL(k_wfa_score16, dim3(nslots), dim3(64), wfa_score16_lds(L, P.e, C), s, S, O, P, Wk, L, C);
  return hipGetLastError();
}

hipError_t launch_wfa_trace(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk,
                            const WfaLaunch &L, int32_t *hbm, int32_t nslots, int32_t threads,
                            bool i16, hipStream_t s) {
  const size_t lds = 2 * (size_t)L.seq_words * 8 +
                     (L.full_in_lds ? (size_t)L.slot_words * 4 : (size_t)L.R * ENTRY * 4);
  if (L.full_in_lds) {
    if (i16)
      hipLaunchKernelGGL((k_wfa_trace<int16_t, true>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
    else
      hipLaunchKernelGGL((k_wfa_trace<int32_t, true>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
  } else {
    if (i16)
      hipLaunchKernelGGL((k_wfa_trace<int16_t, false>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
    else
      hipLaunchKernelGGL((k_wfa_trace<int32_t, false>), dim3(nslots), dim3(threads), lds, s, S, O, P, Wk, L, hbm);
  }
  return hipGetLastError();
}

}  // namespace aim
