// GenASM: windowed bitap distance calculation with a traceback, one pair
// per lane.
//
// Paper, System and Methods, "GenASM": bitap extended with a traceback, a
// bound k on the edits, and per thread a bit-mask of the pattern per
// character, two status bit-vectors and four intermediate bit-vectors (match,
// substitution, deletion, insertion).  The library's reading (unit edits,
// windows of 64 bases with an overlap of 24, the traceback's order, the
// threshold) is the following:
//
// The pair is aligned from its end towards its start in windows of at most
// 64 pattern and 64 text bases, taken from the end of the bases still to
// align (me pattern, ne text bases).  The final window (me, ne <= 64) starts
// at the start of both sequences; any other may start anywhere on its first
// row or column.  With D(i, j) the fewest edits aligning the window's first
// i pattern and j text bases, the status vector of text position j at level
// d holds bit i - 1 = [D(i, j) <= d] for i = 1..a; the start row D(0, j) is
// implicit.  Level d at position j follows from level d at j - 1 and level
// d - 1 at j - 1 and j:
//   match        = ((R_d[j-1] << 1) | [D(0, j-1) <= d]) & PM[t_j]
//   substitution =  (R_{d-1}[j-1] << 1) | [D(0, j-1) <= d-1]
//   insertion    =  (R_{d-1}[j] << 1)   | [D(0, j) <= d-1]
//   deletion     =   R_{d-1}[j-1]
// The window's distance is the least d whose vector at j = b has bit a - 1
// set, searched up to max(a, b) (and the edits k still allows).  The
// traceback walks from (a, b) back with that budget and takes the first of:
// the previous op again if it was a gap ('I' / 'D') and still within budget;
// '='; 'X'; 'I'; 'D'.  A window other than the final commits ops until 40
// bases of either sequence are consumed or its first row or column is
// reached.  When either sequence runs out, the rest of the other is one gap.
// The score is the number of edits; more than k rejects the pair.
//
// MI355X mapping.  A lane owns a pair: the pattern masks (4 x 64 bits) live
// in registers.  The window's distance comes first, from a register-only
// pass over its text (Myers' recurrence on the vertical deltas of the same
// table).  Then only the levels the traceback can read (0 .. distance - 1)
// are built: a sweep over the window's text builds LB consecutive levels at
// once, each level's vector at j - 1 in a register, reading only the level
// below the block (the previous sweep's carry row) once per text position.
// Those levels are stored for the traceback in the wavefront's slot (see
// Slot below), as 32-bit slices around the window's end diagonal unless a
// window of the wavefront has a distance above 14, and only at positions the
// traceback can reach; a wavefront's accesses at one text position are one
// contiguous group.  The traceback compares bases on '=' steps (a run of
// matches at once) and reads stored vectors only around edits, in rounds in
// which every lane of the wavefront that needs them reads them together.
// Work comes 64 pairs at a time from an atomic counter.
#include "aim_internal.h"
#include "dev_util.h"

namespace aim {
namespace {

constexpr int32_t GW = 64;       // window bases
constexpr int32_t GC = GW - 24;  // bases a window other than the final one commits
constexpr int32_t LB = 6;        // edit levels built per sweep over a window's text
constexpr int32_t JB = 8;        // text positions whose lower-level vectors are read ahead
constexpr uint32_t OP_NONE = 4;

__device__ __forceinline__ uint64_t low_bits(int32_t q) {
  return q >= 64 ? ~0ull : (q <= 0 ? 0ull : ((1ull << q) - 1ull));
}

// Masks of the a pattern bases from s0: bit q of pm[c] = [base s0 + q == c];
// lo / hi receive the bases themselves (2-bit codes of window positions
// 1..32 and 33..64).
__device__ __forceinline__ void pattern_masks(const uint64_t *s, int64_t nw, int64_t s0, int32_t a,
                                              uint64_t pm[4], uint64_t &lo, uint64_t &hi) {
  lo = dev::window32(s, nw, s0);
  hi = dev::window32(s, nw, s0 + 32);
  const uint64_t am = low_bits(a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t cc = (uint64_t)c * dev::K55;
    const uint64_t xl = lo ^ cc, xh = hi ^ cc;
    const uint64_t zl = ~(xl | (xl >> 1)) & dev::K55, zh = ~(xh | (xh >> 1)) & dev::K55;
    pm[c] = (((uint64_t)dev::even_bits(zh) << 32) | dev::even_bits(zl)) & am;
  }
}

// The 32 bases of a window ending at position q (1-based; bases lo = 1..32,
// hi = 33..64), position q in the top two bits; positions before 1 read 0.
__device__ __forceinline__ uint64_t tail32(uint64_t lo, uint64_t hi, int32_t q) {
  const int32_t sh = 2 * (q - 32);
  if (sh <= 0) return sh == 0 ? lo : (lo << (-sh));
  if (sh >= 64) return hi;
  return (lo >> sh) | (hi << (64 - sh));
}

// text base j (1-based) of a window whose bases are lo (1..32), hi (33..64)
__device__ __forceinline__ uint32_t base_at(uint64_t lo, uint64_t hi, int32_t j) {
  return (uint32_t)(((j <= 32) ? (lo >> (2 * (j - 1))) : (hi >> (2 * (j - 33)))) & 3u);
}

__device__ __forceinline__ uint64_t pick(const uint64_t pm[4], uint32_t c) {
  const uint64_t a = (c & 1u) ? pm[1] : pm[0];
  const uint64_t b = (c & 1u) ? pm[3] : pm[2];
  return (c & 2u) ? b : a;
}

// A wavefront's slot, reached through a buffer resource.  Raw buffer
// accesses at or past the resource's size are dropped (stores) or read zero
// (loads), so a lane that must not store passes OFF_NONE instead of
// branching around the store.  Byte layout (L levels):
//   narrow: entry (d, j) of lane l, 32 bits at ((d * 64 + j - 1) * 64 + l) * 4:
//           bits j + delta - 16 .. j + delta + 15 of R_d[j] (delta = a - b),
//           all the traceback reads when the window's distance is <= 14;
//   wide:   the same entries as whole 64-bit vectors, at L * 16 KiB + 8 x
//           that index, for wavefronts with a window of distance > 14;
//   carry:  two rows of 64 64-bit vectors per lane, at L * 48 KiB: a sweep's
//           top level, the level below of the next sweep (alternating).
constexpr uint32_t OFF_NONE = 0x80000000u;
constexpr int32_t BUF_FLAGS = 0x00027000;  // word 3 of a raw CDNA buffer resource (32-bit format)
constexpr int32_t NARROW_MAX = 14;         // largest distance the 32-bit slices serve

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

struct Slot {
  __amdgpu_buffer_rsrc_t rs;
  uint32_t wide_base, carry_base;
  __device__ __forceinline__ uint64_t ld64(uint32_t off) const {
    const u32x2 r = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    return ((uint64_t)r.y << 32) | r.x;
  }
  __device__ __forceinline__ void st64(uint64_t v, uint32_t off) const {
    u32x2 w;
    w.x = (uint32_t)v;
    w.y = (uint32_t)(v >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(w, rs, off, 0, 0);
  }
  __device__ __forceinline__ uint32_t ld32(uint32_t off) const {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
  }
  __device__ __forceinline__ void st32(uint32_t v, uint32_t off) const {
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, off, 0, 0);
  }
  __device__ __forceinline__ static uint32_t entry(int32_t d, int32_t j, int lane) {
    return (uint32_t)((d * 64 + j - 1) * 64 + lane);
  }
  __device__ __forceinline__ uint32_t narrow_off(int32_t d, int32_t j, int lane) const { return entry(d, j, lane) * 4u; }
  __device__ __forceinline__ uint32_t wide_off(int32_t d, int32_t j, int lane) const {
    return wide_base + entry(d, j, lane) * 8u;
  }
  __device__ __forceinline__ uint32_t carry_off(int32_t par, int32_t j, int lane) const {
    return carry_base + entry(par, j, lane) * 8u;
  }
};

// bits lo .. lo + 31 of v (bits outside 0..63 read 0)
__device__ __forceinline__ uint32_t slice32(uint64_t v, int32_t lo) {
  if (lo >= 64 || lo <= -32) return 0u;
  return (uint32_t)(lo >= 0 ? (v >> lo) : (v << (-lo)));
}

// D(a, b) of a window: fewest edits aligning its a pattern bases (masks pm)
// with its b text bases, its start anchored (D(i, 0) = i, D(0, j) = j) or
// free (both 0).  Myers' bit-vector recurrence on the vertical deltas of one
// text position after another (bit i - 1: D(i, j) - D(i - 1, j) = +1 in pv,
// -1 in mv); the horizontal delta entering at the start row is +1 when
// anchored, 0 when free; bits at and above a only carry upwards and are
// masked off at the end.
__device__ __forceinline__ int32_t window_distance(const uint64_t pm[4], uint64_t tlo, uint64_t thi, int32_t a,
                                                   int32_t b, bool anchored) {
  uint64_t pv = anchored ? ~0ull : 0ull, mv = 0ull;
  const uint64_t hin = anchored ? 1ull : 0ull;
  for (int32_t j = 1; j <= b; ++j) {
    const uint64_t eq = pick(pm, base_at(tlo, thi, j));
    const uint64_t xv = eq | mv;
    const uint64_t xh = (((eq & pv) + pv) ^ pv) | eq;
    uint64_t ph = mv | ~(xh | pv);
    uint64_t mh = pv & xh;
    ph = (ph << 1) | hin;
    mh = mh << 1;
    pv = mh | ~(xv | ph);
    mv = ph & xv;
  }
  const uint64_t am = low_bits(a);
  return (anchored ? b : 0) + __popcll(pv & am) - __popcll(mv & am);
}

// words of a 256-thread block's slots: per wavefront, narrow entries (4
// bytes), wide entries (8 bytes) and two carry rows (8 bytes)
__host__ __device__ __forceinline__ int64_t block_words(int32_t levels) {
  return (int64_t)4 * ((int64_t)levels * 64 * 64 * 12 + 2 * 64 * 64 * 8) / 8;
}

__global__ __launch_bounds__(256) void k_genasm(Seqs S, Outs O, int32_t k, int32_t want_cigar, Work Wk,
                                                uint64_t *store, int32_t levels) {
  const int lane = threadIdx.x & 63;
  // wavefront-uniform (kept in scalar registers, as the slot's resource must be)
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Slot slot;
  slot.rs = __builtin_amdgcn_make_buffer_rsrc(store + wave * (block_words(levels) / 4), 0,
                                              (int32_t)(block_words(levels) / 4 * 8), BUF_FLAGS);
  slot.wide_base = (uint32_t)levels * 64 * 64 * 4;
  slot.carry_base = (uint32_t)levels * 64 * 64 * 12;
  const int64_t count = Wk.count ? (int64_t)(*(volatile const int32_t *)Wk.count) : Wk.n;
  // a wavefront the work can never reach leaves before touching the counter
  if (wave * 64 >= count) return;

  for (;;) {
    int32_t chunk = 0;
    if (lane == 0) chunk = atomicAdd(Wk.counter, 1);
    chunk = __shfl(chunk, 0);
    if ((int64_t)chunk * 64 >= count) break;
    const int64_t li = (int64_t)chunk * 64 + lane;
    const bool has = li < count;
    const int64_t p = has ? (Wk.idx ? (int64_t)Wk.idx[li] : li) : 0;
    bool live = has;
    if (has && !Wk.direct && O.flags && O.flags[p]) {
      O.score[p] = -1;
      O.status[p] = ST_INVALID;
      O.nruns[p] = 0;
      live = false;
    }
    const int32_t m = live ? S.pat_len[p] : 0, n = live ? S.txt_len[p] : 0;
    const uint64_t *pat = S.pat + (live ? S.pat_off[p] : 0);
    const uint64_t *txt = S.txt + (live ? S.txt_off[p] : 0);
    const int64_t pnw = (m + 31) >> 5, tnw = (n + 31) >> 5;
    const bool cig = live && want_cigar;
    const bool direct = Wk.direct != 0;
    const int32_t total = (cig && direct) ? O.nruns[p] : 0;
    uint32_t *dst = (cig && direct) ? O.cigar + O.cigar_off[p] : nullptr;
    RunSink sink;
    if (cig && !direct) sink.begin(O, p);
    uint32_t cur_op = 0xffu, cur_len = 0;
    int32_t nr = 0;
    int32_t me = m, ne = n, used = 0;
    uint32_t prev = OP_NONE;
    bool rej = false;
    // runs still to come, this one included, at most: one per base left, and
    // with a threshold two per edit left plus the current and a last '=' run
    auto put = [&](uint32_t op, uint32_t len, int64_t left) {
      if (!cig) return;
      if (op == cur_op) {
        cur_len += len;
        return;
      }
      if (cur_len) {
        const uint32_t run = (cur_len << 4) | cur_op;
        if (direct) {
          if (nr < total) dst[total - 1 - nr] = run;
        } else {
          int64_t more = left;
          if (k >= 0) more = min<int64_t>(more, 2 * (int64_t)(k - used) + 3);
          sink.put(nr, run, more);
        }
        ++nr;
      }
      cur_op = op;
      cur_len = len;
    };

    while (live && me > 0 && ne > 0) {
      const bool anchored = me <= GW && ne <= GW;
      const int32_t a = min(GW, me), b = min(GW, ne);
      uint64_t pm[4], plo, phi;
      pattern_masks(pat, pnw, me - a, a, pm, plo, phi);
      const uint64_t tlo = dev::window32(txt, tnw, ne - b), thi = dev::window32(txt, tnw, ne - b + 32);
      int32_t lw = max(a, b);
      if (k >= 0) lw = min(lw, k - used);
      // ---- the window's distance, from vertical deltas alone ----
      int32_t dist = window_distance(pm, tlo, thi, a, b, anchored);
      if (dist > lw) dist = -1;
      if (dist < 0) {
        rej = true;
        break;
      }
      if (!cig && anchored) {
        // score only: the final window adds its distance, no walk needed
        used += dist;
        me = ne = 0;
        break;
      }
      // ---- status vectors of the levels the traceback reads, 0..dist-1,
      // LB levels per sweep over the text ----
      // the traceback of a window other than the final one reads positions
      // j >= b - GC only; a wavefront with a window of distance > 14 keeps
      // whole vectors
      const int32_t jmin = anchored ? 1 : max(1, b - GC);
      const int32_t delta = a - b;
      const bool wide = __any(dist > NARROW_MAX);
      // wavefront-uniform: the first position any lane stores (1, or GC
      // positions before the end of a full window when every lane's window
      // is one), so that earlier positions issue no store at all
      const int32_t jlo = __any(jmin < GW - GC) ? 1 : GW - GC;
      for (int32_t d0 = 0; d0 < dist; d0 += LB) {
        uint64_t v[LB];  // R_{d0+q}[j-1]; bits at and above a are never read
#pragma unroll
        for (int q = 0; q < LB; ++q) v[q] = anchored ? low_bits(d0 + q) : ~0ull;
        uint64_t pp = d0 > 0 ? (anchored ? low_bits(d0 - 1) : ~0ull) : 0ull;  // R_{d0-1}[j-1]
        // R_{d0-1}[j] from the previous sweep's carry row, read (only when
        // d0 > 0) JB positions ahead of use
        const int32_t par = (d0 / LB) & 1;
        // wavefront-uniform: which of this sweep's levels some lane keeps,
        // and whether some lane needs a further sweep
        bool need[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) need[q] = __any(d0 + q < dist);
        const bool carry = __any(d0 + LB < dist);
        uint64_t nxt[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u)
          nxt[u] = slot.ld64((d0 > 0 && u < b) ? slot.carry_off(par ^ 1, u + 1, lane) : OFF_NONE);
        for (int32_t j0 = 1; j0 <= b; j0 += JB) {
          uint64_t cur[JB];
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            cur[u] = nxt[u];
            const int32_t jn = j0 + JB + u;  // next chunk's position
            nxt[u] = slot.ld64((d0 > 0 && jn <= b) ? slot.carry_off(par ^ 1, jn, lane) : OFF_NONE);
          }
          // positions past b (the last chunk of a short window) compute
          // values nobody reads and store nothing
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            const int32_t j = j0 + u;
            const uint64_t pmc = pick(pm, base_at(tlo, thi, j));
            uint64_t old_lo = pp, new_lo = cur[u];  // the level below at j - 1 and at j
            const bool keep = j <= b && j >= jmin;
#pragma unroll
            for (int q = 0; q < LB; ++q) {
              const int32_t d = d0 + q;
              // [D(0, j - 1) <= d]
              uint64_t nv = ((v[q] << 1) | ((!anchored || j - 1 <= d) ? 1ull : 0ull)) & pmc;
              if (d > 0) {
                // substitution | insertion | deletion; [D(0, j) <= d - 1]
                // implies [D(0, j - 1) <= d - 1], so one start bit serves both
                nv |= ((old_lo | new_lo) << 1) | ((!anchored || j - 1 <= d - 1) ? 1ull : 0ull) | old_lo;
              }
              old_lo = v[q];
              new_lo = nv;
              v[q] = nv;
              if (need[q] && j >= jlo) {
                const bool st = keep && d < dist;
                if (wide)
                  slot.st64(nv, st ? slot.wide_off(d, j, lane) : OFF_NONE);
                else
                  slot.st32(slice32(nv, j + delta - 16), st ? slot.narrow_off(d, j, lane) : OFF_NONE);
              }
            }
            // the top level, for the next sweep of a lane that needs one
            if (carry) slot.st64(v[LB - 1], (j <= b && d0 + LB < dist) ? slot.carry_off(par, j, lane) : OFF_NONE);
            pp = cur[u];
          }
        }
      }
      // ---- traceback over the stored levels ----
      int32_t i = a, j = b, d = dist;
      // R_dd[jj] as stored, shifted so that bit p of R_dd[jj] is bit p of the
      // result for every bit the traceback reads
      auto R = [&](int32_t dd, int32_t jj) -> uint64_t {
        if (jj == 0) return anchored ? low_bits(dd) : ~0ull;
        if (wide) return slot.ld64(slot.wide_off(dd, jj, lane));
        const int32_t lo = jj + delta - 16;
        const uint64_t w = slot.ld32(slot.narrow_off(dd, jj, lane));
        if (lo >= 64 || lo <= -32) return 0ull;  // no bit the walk reads
        return lo >= 0 ? (w << lo) : (w >> (-lo));
      };
      // [D(ii - 1, jj) <= dd] from v = R_dd[jj] (ii >= 1)
      auto up = [&](uint64_t v, int32_t dd, int32_t jj, int32_t ii) -> bool {
        if (ii == 1) return !anchored || jj <= dd;
        return (v >> (ii - 2)) & 1ull;
      };
      // a window other than the final one stops after GC bases of either
      // sequence or at its first row or column
      auto stop = [&]() -> bool {
        return anchored ? (i == 0 && j == 0) : (a - i >= GC || b - j >= GC || i == 0 || j == 0);
      };
      auto apply = [&](uint32_t op) {
        if (op != OP_EQ) {
          d -= 1;
          used += 1;
        }
        if (op != OP_D) --i;
        if (op != OP_I) --j;
        put(op, 1, (int64_t)(me - a + i) + (ne - b + j) + 2);
        prev = op;
      };
      // In rounds: every lane first takes the steps that need no stored
      // vector, then the lanes at a decision read theirs together (one memory
      // wait per round for the wavefront rather than one per step).
      for (;;) {
        bool done = false;
        for (;;) {
          if (stop()) {
            done = true;
            break;
          }
          if (i == 0) {
            apply(OP_D);
            continue;
          }
          if (j == 0) {
            apply(OP_I);
            continue;
          }
          if (prev == OP_I || prev == OP_D) break;
          // The walk only visits cells whose distance equals its budget d
          // (it starts at the window's distance and every op keeps to an
          // optimal continuation).  Adjacent cells of an edit-distance table
          // differ by at most one and D(i-1, j-1) <= D(i, j), so where the
          // bases match D(i-1, j-1) = d and '=' is available: a run of
          // matching bases along the diagonal is taken at once, up to where
          // the window stops (or its first row or column).
          const uint64_t x = tail32(plo, phi, i) ^ tail32(tlo, thi, j);
          int32_t r = x ? (__clzll(x) >> 1) : 32;
          int32_t lim = min(i, j);
          if (!anchored) lim = min(lim, min(GC - (a - i), GC - (b - j)));
          r = min(r, lim);
          if (r == 0) break;
          i -= r;
          j -= r;
          put(OP_EQ, (uint32_t)r, (int64_t)(me - a + i) + (ne - b + j) + 2);
          prev = OP_EQ;
        }
        if (done) break;
        const uint64_t ri = d > 0 ? R(d - 1, j) : 0ull;      // [D(., j) <= d - 1]
        const uint64_t rd = d > 0 ? R(d - 1, j - 1) : 0ull;  // [D(., j - 1) <= d - 1]
        const bool eq = (pick(pm, base_at(tlo, thi, j)) >> (i - 1)) & 1ull;
        const bool ins = d > 0 && up(ri, d - 1, j, i);
        const bool del = d > 0 && ((rd >> (i - 1)) & 1ull);
        uint32_t op;
        if (prev == OP_I && ins) op = OP_I;
        else if (prev == OP_D && del) op = OP_D;
        else if (eq) op = OP_EQ;
        else if (d > 0 && up(rd, d - 1, j - 1, i)) op = OP_X;
        else if (ins) op = OP_I;
        else op = OP_D;
        apply(op);
      }
      me -= a - i;
      ne -= b - j;
    }
    if (live && !rej) {
      if (me > 0) put(OP_I, (uint32_t)me, 2);
      if (ne > 0) put(OP_D, (uint32_t)ne, 2);
      used += me + ne;
      if (k >= 0 && used > k) rej = true;
      if (!rej) put(0xfu, 0, 1);  // flush the last run
    }
    if (!live || direct) continue;
    if (cig) sink.finish();
    O.score[p] = rej ? -1 : used;
    O.status[p] = rej ? ST_REJECTED : ST_ALIGNED;
    O.nruns[p] = rej ? 0 : nr;
  }
}

}  // namespace

// levels 0..min(k, 64), rounded up to whole sweeps (the last sweep may build
// levels past the cap; they are stored but never used)
int32_t genasm_levels(int32_t max_score) {
  const int32_t top = max_score < 0 ? 64 : min(max_score, 64);
  return (top + 1 + LB - 1) / LB * LB;
}

int64_t genasm_block_words(int32_t levels) { return block_words(levels); }

hipError_t launch_genasm(const Seqs &S, const Outs &O, const Scoring &P, const Work &Wk, uint64_t *store,
                         int32_t levels, int32_t nblocks, hipStream_t s) {
  if (nblocks <= 0 || levels < genasm_levels(P.max_score)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_genasm, dim3(nblocks), dim3(256), 0, s, S, O, P.max_score, P.want_cigar, Wk, store,
                     levels);
  return hipGetLastError();
}

}  // namespace aim
