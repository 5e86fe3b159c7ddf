// Device helpers shared by the wavefront kernels (wfa.hip, wfa_lds.hip):
// sequence windows and the extend step, the origin codes of a cell and the
// walk that turns kept codes into a CIGAR, staging and list appends.
// Included inside an anonymous namespace of each translation unit.
#pragma once

constexpr int32_t NEG = INT32_MIN / 4;  // absent / invalid offset
constexpr int WGMAX = 256;             // largest workgroup (wide pairs)
constexpr int ENTRY = 4;                // table entry: lo, hi, base, present-bits
constexpr int TAB16 = 8;                // one-wavefront score pass: ranges of I, D, M
constexpr int32_t EMPTY_LO = 0x3fffffff, EMPTY_HI = -0x3fffffff;  // an empty range



__device__ __forceinline__ uint64_t seq_window(const uint64_t *w, int64_t nw, int64_t t) {
  // 32 bases starting at base t (t >= 0); words past the end read as zero
  const int64_t q = t >> 5;
  const uint32_t r = (uint32_t)(t & 31);
  const uint64_t w0 = q < nw ? w[q] : 0ull;
  const uint64_t w1 = q + 1 < nw ? w[q + 1] : 0ull;
  return r ? ((w0 >> (2 * r)) | (w1 << (64 - 2 * r))) : w0;
}

// Extend offset f on diagonal k while P[i] == T[j] (i = f - k, j = f).
__device__ __forceinline__ int32_t extend(const uint64_t *P, int64_t pnw, int32_t m,
                                          const uint64_t *T, int64_t tnw, int32_t n, int32_t k,
                                          int32_t f) {
  int32_t i = f - k, j = f;
  for (;;) {
    const int32_t lim = min(m - i, n - j);
    if (lim <= 0) break;
    const uint64_t x = seq_window(P, pnw, i) ^ seq_window(T, tnw, j);
    int32_t run = x ? (int32_t)(__builtin_ctzll(x) >> 1) : 32;
    if (run > lim) run = lim;
    i += run;
    j += run;
    if (run < 32) break;
  }
  return j;
}

// Sequence access for the extend step: words read in place (HBM or LDS), or
// staged in LDS and compared 16 bases at a time.
// ext_all(m, n, k, f) is called by every lane: it extends f when f >= 0 and
// returns it unchanged otherwise.
struct SeqInPlace {
  const uint64_t *P, *T;
  int64_t pnw, tnw;
  __device__ __forceinline__ int32_t ext(int32_t m, int32_t n, int32_t k, int32_t f) const;
  __device__ __forceinline__ int32_t ext_all(int32_t m, int32_t n, int32_t k, int32_t f) const;
  // by the whole wavefront, for the replay of a walk (same arguments in every lane)
  __device__ __forceinline__ int32_t ext_wave(int32_t m, int32_t n, int32_t k, int32_t f) const;
};
struct SeqStaged {
  const uint32_t *P32, *T32;
  __device__ __forceinline__ int32_t ext(int32_t m, int32_t n, int32_t k, int32_t f) const;
  __device__ __forceinline__ int32_t ext_all(int32_t m, int32_t n, int32_t k, int32_t f) const;
  // by the whole wavefront, for the replay of a walk (same arguments in every lane)
  __device__ __forceinline__ int32_t ext_wave(int32_t m, int32_t n, int32_t k, int32_t f) const;
};

// Table entries are the same for every lane: read them as scalars, so that the
// source arrays they locate are addressed from scalar bases.
__device__ __forceinline__ int32_t tab_get(const int32_t *tab, int32_t slot, int f) {
  return __builtin_amdgcn_readfirstlane(tab[slot * ENTRY + f]);
}

// extend() on sequences staged in LDS, 16 bases per step: the 32-bit window
// at any base is one funnel shift of two adjacent 32-bit words.  It reads up
// to one word past a sequence's last; the staged layout keeps that read inside
// the workgroup's LDS, and bases past either end are cut by the limit.
__device__ __forceinline__ int32_t extend_lds(const uint32_t *P32, int32_t m, const uint32_t *T32,
                                              int32_t n, int32_t k, int32_t f) {
  int32_t i = f - k, j = f;
  for (;;) {
    const int32_t lim = min(m - i, n - j);
    if (lim <= 0) break;
    const uint32_t pw = __builtin_amdgcn_alignbit(P32[(i >> 4) + 1], P32[i >> 4], (uint32_t)(i & 15) * 2);
    const uint32_t tw = __builtin_amdgcn_alignbit(T32[(j >> 4) + 1], T32[j >> 4], (uint32_t)(j & 15) * 2);
    const uint32_t d = pw ^ tw;
    int32_t run = d ? (int32_t)(__builtin_ctz(d) >> 1) : 16;
    if (run > lim) run = lim;
    i += run;
    j += run;
    if (run < 16) break;
  }
  return j;
}

// extend_lds by a whole wavefront, for the serial walk's replay: lane l
// compares the 16 bases that start 16 l bases along the diagonal, so one
// round of LDS reads covers 1,024 bases; the first lane whose bases stop
// matching, or that reaches an end, gives the run.  Every lane of the
// wavefront calls it with the same arguments and gets the same result.  A
// lane reads only where its first base lies before both ends: the words
// extend_lds itself would read.
__device__ __forceinline__ int32_t extend_wave(const uint32_t *P32, int32_t m, const uint32_t *T32, int32_t n,
                                               int32_t k, int32_t f) {
  const int32_t off = 16 * (int32_t)(threadIdx.x & 63);
  int32_t i = f - k, j = f;
  for (;;) {
    const int32_t lim = min(m - i, n - j);
    if (lim <= 0) return j;
    const int32_t left = lim - off;  // bases this lane may compare
    int32_t run = 0;
    if (left > 0) {
      const int32_t a = i + off, b = j + off;
      const uint32_t d = __builtin_amdgcn_alignbit(P32[(a >> 4) + 1], P32[a >> 4], (uint32_t)(a & 15) * 2) ^
                         __builtin_amdgcn_alignbit(T32[(b >> 4) + 1], T32[b >> 4], (uint32_t)(b & 15) * 2);
      run = min(d ? (int32_t)(__builtin_ctz(d) >> 1) : 16, left);
    }
    const uint64_t stop = __ballot(run < 16);
    if (stop) {
      const int32_t first = (int32_t)__builtin_ctzll(stop);
      return j + 16 * first + __builtin_amdgcn_readlane(run, first);
    }
    i += 1024;
    j += 1024;
  }
}

__device__ __forceinline__ int32_t SeqInPlace::ext(int32_t m, int32_t n, int32_t k, int32_t f) const {
  return extend(P, pnw, m, T, tnw, n, k, f);
}
__device__ __forceinline__ int32_t SeqStaged::ext(int32_t m, int32_t n, int32_t k, int32_t f) const {
  return extend_lds(P32, m, T32, n, k, f);
}
// in place (HBM): the serial extend, as ext
__device__ __forceinline__ int32_t SeqInPlace::ext_wave(int32_t m, int32_t n, int32_t k, int32_t f) const {
  return extend(P, pnw, m, T, tnw, n, k, f);
}
__device__ __forceinline__ int32_t SeqStaged::ext_wave(int32_t m, int32_t n, int32_t k, int32_t f) const {
  return extend_wave(P32, m, T32, n, k, f);
}
__device__ __forceinline__ int32_t SeqInPlace::ext_all(int32_t m, int32_t n, int32_t k, int32_t f) const {
  return f >= 0 ? extend(P, pnw, m, T, tnw, n, k, f) : f;
}
// The first 16 bases by every lane without a branch (a lane with no offset
// compares at base 0 under a zero limit), the rest only where all 16 matched.
__device__ __forceinline__ int32_t SeqStaged::ext_all(int32_t m, int32_t n, int32_t k, int32_t f) const {
  const bool live = f >= 0;
  const int32_t i0 = live ? f - k : 0, j0 = live ? f : 0;
  const int32_t lim = live ? min(m - i0, n - j0) : 0;
  const uint32_t d = __builtin_amdgcn_alignbit(P32[(i0 >> 4) + 1], P32[i0 >> 4], (uint32_t)(i0 & 15) * 2) ^
                     __builtin_amdgcn_alignbit(T32[(j0 >> 4) + 1], T32[j0 >> 4], (uint32_t)(j0 & 15) * 2);
  const int32_t run = min(d ? (int32_t)(__builtin_ctz(d) >> 1) : 16, lim);
  int32_t g = j0 + run;
  if (run == 16) g = extend_lds(P32, m, T32, n, k, g);
  return live ? g : f;
}

// ------------------------------------------- origin codes and the fused walk
// A score pass can keep, per cell, how each component got its value (4 bits:
// bits 0-1 the source of M in the canonical order, 0 X, 1 I, 2 D; bit 2 I
// opened from M_{s-o-e} rather than extended; bit 3 the same for D), which is
// all the backtrace chooses.  The walk then needs no offsets: it follows the
// codes back from the end cell, recording one token per state (an M visit, or
// an X, I or D op), and a forward replay of the tokens from (0, 0), extending
// every M visit as far as the bases match, recovers the '=' runs -- the M
// offsets are exactly those maximal extensions.  Two neighbouring lanes hold
// neighbouring diagonals; the even lane stores the byte of both codes.
constexpr uint32_t TOK_M = 4;  // token of an M visit (its run length above bit 4)

__device__ __forceinline__ int32_t origin_code_of(int32_t vx, int32_t vi, int32_t vd, int32_t vm,
                                                  bool i_open, bool d_open) {
  return (vx == vm ? 0 : (vi == vm ? 1 : 2)) | (i_open ? 4 : 0) | (d_open ? 8 : 0);
}

// The pair's neighbour code (lane l + 1) joined with this lane's, for the
// even lane to store.
__device__ __forceinline__ uint8_t code_pair(int32_t code) {
  const int32_t up = __builtin_amdgcn_update_dpp(0, code, 0x130, 0xF, 0xF, false);  // lane l + 1
  return (uint8_t)(code | (up << 4));
}

// The second half of a walk: from the nt tokens (last first) in `tok`,
// written by lane 0 of the calling wavefront, replay the alignment forward
// from (0, 0), extending every M visit as far as the bases match, and write
// the runs (to the pair's slot and pool, or to dst as walk_codes does).
// Returns false if the tokens do not end at (m, n).
//
// The tokens are taken 64 at a time, one per lane, into a register, and each
// is read from there with a lane read: the walk over them is serial, and a
// load per token would put one memory round trip on its path per token.  The
// replay keeps the run lengths it finds in the same register and stores the
// 64 tokens back together; the run-length pass reads them the same way.
template <class Ext>
__device__ bool replay_tokens(const Outs &O, int64_t p, Ext ext, int32_t m, int32_t n, uint32_t *tok, int32_t nt,
                              uint32_t *dst, int32_t total) {
  const int lane = threadIdx.x & 63;
  __threadfence_block();  // lane 0's tokens visible to the wavefront
  // forward replay: the '=' run of each M visit; lane l holds token t0 - l
  int32_t i = 0, j = 0;
  for (int32_t t0 = nt - 1; t0 >= 0; t0 -= 64) {
    const int32_t cnt = min(t0 + 1, 64);
    uint32_t v = lane < cnt ? tok[t0 - lane] : 0u;
    for (int32_t c = 0; c < cnt; ++c) {
      const uint32_t tk = __builtin_amdgcn_readlane(v, c);
      if (tk == TOK_M) {
        const int32_t len = __builtin_amdgcn_readfirstlane(ext(j - i, j)) - j;
        if (lane == c) v = TOK_M | ((uint32_t)len << 4);
        i += len;
        j += len;
      } else if (tk == OP_X) {
        ++i; ++j;
      } else if (tk == OP_I) {
        ++i;
      } else {
        ++j;
      }
    }
    if (lane < cnt) tok[t0 - lane] = v;
  }
  if (i != m || j != n) return false;  // cannot happen for a reached end cell
  __threadfence_block();
  RunSink sink;
  if (lane == 0 && !dst) sink.begin(O, p);
  auto put = [&](int32_t nr, uint32_t run, int64_t more) {
    if (!dst) sink.put(nr, run, more);
    else if (nr < total) dst[total - 1 - nr] = run;
  };
  // lane 0 merges the tokens into runs; lane l holds token t0 + l
  uint32_t cur_op = 0xffu, cur_len = 0;
  int32_t nr = 0;
  for (int32_t t0 = 0; t0 < nt; t0 += 64) {
    const int32_t cnt = min(nt - t0, 64);
    const uint32_t v = lane < cnt ? tok[t0 + lane] : 0u;
    if (lane == 0) {
      for (int32_t c = 0; c < cnt; ++c) {
        const uint32_t tk = __builtin_amdgcn_readlane(v, c);
        const uint32_t op = (tk & 15u) == TOK_M ? (uint32_t)OP_EQ : (tk & 15u);
        const uint32_t len = (tk & 15u) == TOK_M ? (tk >> 4) : 1u;
        if (len == 0) continue;
        if (op == cur_op) {
          cur_len += len;
        } else {
          if (cur_len) put(nr++, (cur_len << 4) | cur_op, nt - (t0 + c) + 1);
          cur_op = op;
          cur_len = len;
        }
      }
    }
  }
  if (lane == 0) {
    if (cur_len) put(nr++, (cur_len << 4) | cur_op, 1);
    if (!dst) {
      sink.finish();
      O.nruns[p] = nr;
    }
  }
  return true;
}


// Run by one whole wavefront on uniform values; its lane 0 writes.
// code_at(s, k) is evaluated per lane and gives the code of a kept cell, or
// -1; ext(k, f) extends offset f on diagonal k.  Returns false (nothing
// written to the CIGAR outputs) when a code is missing or the tokens outgrow
// `tok`.
//
// A move leaves a cell (s, k) for one of five cells: X (s-x, k), I opened
// (s-o-e, k+1) or extended (s-e, k+1), D opened (s-o-e, k-1) or extended
// (s-e, k-1).  With AHEAD, each round of loads fetches, one cell per lane, the
// codes of the five successors of the current cell and of their 25 successors,
// so that two moves follow every round trip to memory (worth it where the walk
// is on the critical path: the few long pairs of a wide-pair pass); without,
// each move loads the one code it needs.
// dst non-null: the runs go straight to dst (the pair's CIGAR range, `total`
// runs, filled last run first as the slots are) and nruns is left as is.
template <bool AHEAD, class CodeAt, class Ext>
__device__ bool walk_codes(const Outs &O, int64_t p, CodeAt code_at, Ext ext, int32_t x, int32_t oe,
                           int32_t e, int32_t m, int32_t n, int32_t sfin, uint32_t *tok, int32_t tok_cap,
                           uint32_t *dst = nullptr, int32_t total = 0) {
  const int lane = threadIdx.x & 63;
  int32_t cs = sfin, k = n - m, comp = 0, nt = 0;
  bool ok = true;
  if constexpr (!AHEAD) {
    int32_t code = -1;
    for (;;) {
      if (nt + 2 > tok_cap || cs < 0) { ok = false; break; }
      if (comp == 0) {
        if (lane == 0) tok[nt] = TOK_M;
        ++nt;
        if (cs == 0) { ok = k == 0; break; }
        if (code < 0) code = __builtin_amdgcn_readfirstlane(code_at(cs, k));
        if (code < 0) { ok = false; break; }
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
        if (code < 0) code = __builtin_amdgcn_readfirstlane(code_at(cs, k));
        if (code < 0) { ok = false; break; }
        const bool open = (code >> (comp + 1)) & 1;
        if (lane == 0) tok[nt] = comp == 1 ? OP_I : OP_D;
        ++nt;
        k += comp == 1 ? 1 : -1;
        if (open) { cs -= oe; comp = 0; } else { cs -= e; }
        code = -1;
      }
    }
  } else {
    auto dstep = [&](int j) { return j == 0 ? x : ((j & 1) ? oe : e); };  // score drop of move j
    auto dkst = [&](int j) { return j == 0 ? 0 : (j <= 2 ? 1 : -1); };    // diagonal change of move j
    // this lane's cell of a round: lanes 0..4 the successors, 5..29 theirs
    const int j1 = lane < 5 ? lane : (lane - 5) / 5, j2 = lane < 5 ? -1 : (lane - 5) % 5;
    const int32_t lds_ = lane < 30 ? dstep(j1) + (j2 >= 0 ? dstep(j2) : 0) : 0;
    const int32_t ldk = lane < 30 ? dkst(j1) + (j2 >= 0 ? dkst(j2) : 0) : 0;
    int32_t code = __builtin_amdgcn_readfirstlane(code_at(cs, k));
    bool done = false;
    while (ok && !done) {
      // one round: the codes two moves ahead of (cs, k)
      const int32_t v = lane < 30 ? code_at(cs - lds_, k + ldk) : -1;
      int moves = 0, j0 = 0;
      while (moves < 2) {
        if (nt + 2 > tok_cap || cs < 0) { ok = false; break; }
        int j = -1;  // move taken from this cell, if any
        if (comp == 0) {
          if (lane == 0) tok[nt] = TOK_M;
          ++nt;
          if (cs == 0) { ok = k == 0; done = true; break; }
          if (code < 0) { ok = false; break; }
          const int32_t src = code & 3;
          if (src == 0) {
            if (lane == 0) tok[nt] = OP_X;
            ++nt;
            j = 0;
          } else {
            comp = src;  // I or D of the same cell
          }
        } else {
          if (code < 0) { ok = false; break; }
          const bool open = (code >> (comp + 1)) & 1;
          if (lane == 0) tok[nt] = comp == 1 ? OP_I : OP_D;
          ++nt;
          j = comp == 1 ? (open ? 1 : 2) : (open ? 3 : 4);
          if (open) comp = 0;
        }
        if (j >= 0) {
          cs -= dstep(j);
          k += dkst(j);
          code = __builtin_amdgcn_readlane(v, moves == 0 ? j : 5 + 5 * j0 + j);
          j0 = j;
          ++moves;
        }
      }
    }
  }
  if (!ok) return false;
  return replay_tokens(O, p, ext, m, n, tok, nt, dst, total);
}

// An accepted pair whose full store passes the largest class: to the
// memory-bounded long pass when one runs, else no CIGAR.  One thread.
__device__ __forceinline__ void to_long_pass(const Outs &O, int64_t p, int32_t *list, int32_t *count) {
  if (list) {
    const int32_t k = atomicAdd(count, 1);
    list[k] = (int32_t)p;
  } else {
    O.status[p] = ST_OVERFLOW;
  }
}

__device__ __forceinline__ void stage_seq(uint64_t *lds, const uint64_t *g, int64_t nw) {
  for (int64_t q = threadIdx.x; q < nw; q += blockDim.x) lds[q] = g[q];
}

__device__ __forceinline__ void wave_append1(bool pred, int32_t v, int32_t *list, int32_t *cnt) {
  if (pred && threadIdx.x == 0) {
    const int32_t k = atomicAdd(cnt, 1);
    list[k] = v;
  }
}


// ------------------------------------------------------------ window classes
// Predicted extent of a pair that reached diagonal extent `ext` when its
// furthest M offset had come `prog` bases along both sequences (i + j): the
// score, and with it the span of diagonals, grows about in proportion to the
// progress along the pair; 5/4 of that, and never more than [-m, n] allows.
// With too little progress to extrapolate from, the widest span.
__device__ __forceinline__ int32_t predict_extent(int32_t ext, int32_t prog, int32_t m, int32_t n) {
  const int64_t total = (int64_t)m + n;
  const int32_t cap = max(m, n + 1);
  if ((int64_t)prog * 64 < total) return cap;
  const int64_t pr = (int64_t)ext * total * 5 / (4 * (int64_t)prog) + 1;
  return (int32_t)min<int64_t>(max<int64_t>(pr, ext + 1), cap);
}

// Sends pair p, which left the window of class `from`, to the first later
// class whose half-window holds `pred` (the last class takes any pair).
// Called by one thread.
__device__ __forceinline__ void route_pair(const WfaRoute &rt, int32_t from, int64_t p, int32_t pred) {
  int c = from + 1;
  while (c < rt.nclass && rt.half[c] < pred) ++c;
  rt.pred[p] = pred;
  const int32_t at = atomicAdd(rt.count[c], 1);
  rt.list[c][at] = (int32_t)p;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
