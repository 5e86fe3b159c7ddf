// Sequence packing, per-pair validation, prefix scan and CIGAR compaction.
#include "aim_internal.h"

namespace aim {
namespace {

constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_pair_flags(int64_t n, int32_t max_len, const int32_t *pl, const int32_t *tl,
                             const int8_t *pf, const int8_t *tf, int8_t *flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = pl[i], b = tl[i];
    int8_t f = (a < 0 || b < 0 || a > max_len || b > max_len) ? 1 : 0;
    if (pf && pf[i]) f = 1;
    if (tf && tf[i]) f = 1;
    flags[i] = f;
  }
}

// words per sequence for packing
__global__ void k_word_counts(int64_t n, const int32_t *len, int32_t max_len, int32_t *cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t L = len[i];
    // sequences beyond max_len are invalid pairs: give them no words so they
    // do not shift the layout of the others
    cnt[i] = (L > 0 && L <= max_len) ? (L + 31) >> 5 : 0;
  }
}

// One wavefront per sequence; lane l packs bytes [32 l, 32 l + 32) of each
// 64-word group, so a wave reads 2 KB of contiguous input per iteration.
// stride > 0: sequence s starts at word s * stride, written to woff_set
// (entries 0..n); else at woff[s].
__global__ __launch_bounds__(256) void k_pack(int64_t n, int32_t enc, const uint8_t *seq,
                                              const int64_t *off, const int32_t *len,
                                              int32_t max_len, uint64_t *words,
                                              int64_t words_cap, const int64_t *woff,
                                              int8_t *flags, int64_t stride, int64_t *woff_set) {
  const int lane = threadIdx.x & 63;
  const int64_t s = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
  if (s >= n) return;
  if (stride > 0 && lane == 0) {
    woff_set[s] = s * stride;
    if (s == n - 1) woff_set[n] = n * stride;
  }
  if (len[s] > max_len) {
    if (flags && lane == 0) flags[s] = 1;
    return;
  }
  const int32_t L = len[s] > 0 ? len[s] : 0;
  const uint8_t *src = seq + off[s];
  const int64_t w0 = stride > 0 ? s * stride : woff[s];
  const int32_t nw = (L + 31) >> 5;
  bool bad = false;
  for (int32_t w = lane; w < nw; w += 64) {
    uint64_t v = 0;
    const int32_t b0 = w * 32;
    const int32_t cnt = min(32, L - b0);
    for (int32_t t = 0; t < cnt; ++t) {
      const uint8_t c = src[b0 + t];
      uint32_t code;
      if (enc == 0) {
        code = c == 'A' ? 0u : c == 'C' ? 1u : c == 'G' ? 2u : c == 'T' ? 3u : 4u;
      } else {
        code = c;
      }
      if (code > 3u) { bad = true; code = 0; }
      v |= (uint64_t)code << (2 * t);
    }
    if (w0 + w < words_cap) words[w0 + w] = v;
    else bad = true;
  }
  const bool any_bad = __ballot(bad) != 0;
  if (flags && lane == 0) flags[s] = any_bad ? 1 : 0;
}

// ---- three-phase exclusive scan of int32 -> int64 ----
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t *in, int64_t n,
                                                           int64_t *tmp) {
  __shared__ int64_t red[SCAN_BLOCK];
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * SCAN_BLOCK + threadIdx.x;
    if (i < n) s += in[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = SCAN_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) tmp[blockIdx.x] = red[0];
}

// exclusive scan in place of tmp[0..nb), tmp[nb] = total; one block
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t *tmp, int64_t nb) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? tmp[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
      const int64_t add = threadIdx.x >= w ? buf[threadIdx.x - w] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    const int64_t incl = buf[threadIdx.x];
    if (i < nb) tmp[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) tmp[nb] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int32_t *in, int64_t n,
                                                          const int64_t *tmp, int64_t *out,
                                                          int64_t nb) {
  __shared__ int64_t buf[SCAN_TILE];
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * SCAN_BLOCK + threadIdx.x;
    buf[k * SCAN_BLOCK + threadIdx.x] = i < n ? in[i] : 0;
  }
  __syncthreads();
  // each thread scans a contiguous run of SCAN_ITEMS, then a block scan of sums
  __shared__ int64_t sums[SCAN_BLOCK];
  int64_t local[SCAN_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    local[k] = s;
    s += buf[threadIdx.x * SCAN_ITEMS + k];
  }
  sums[threadIdx.x] = s;
  __syncthreads();
  for (int w = 1; w < SCAN_BLOCK; w <<= 1) {
    const int64_t add = threadIdx.x >= w ? sums[threadIdx.x - w] : 0;
    __syncthreads();
    sums[threadIdx.x] += add;
    __syncthreads();
  }
  const int64_t pre = tmp[blockIdx.x] + sums[threadIdx.x] - s;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + threadIdx.x * SCAN_ITEMS + k;
    if (i < n) out[i] = pre + local[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tmp[nb];
}

// ---- CIGAR compaction ----
// total_written = the largest inclusive prefix that fits in cigar_cap
__global__ void k_cut(int64_t n, const int64_t *excl, int64_t cap, unsigned long long *tw) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t incl = excl[i + 1];
    if (incl <= cap && (i + 1 == n || excl[i + 2] > cap))
      atomicMax(tw, (unsigned long long)incl);
  }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One pair per thread.  Slots hold a pair's runs last-op-first; slot_cap is a
// multiple of 4 and slots are 16-byte aligned, so each 16-byte load stays in
// the pair's slot.
__global__ __launch_bounds__(256) void k_scatter(
    int64_t n, const int64_t *__restrict__ excl, const unsigned long long *__restrict__ tw_p,
    const int32_t *__restrict__ nruns, const uint32_t *__restrict__ slot, int32_t slot_cap,
    const uint32_t *__restrict__ pool, const int64_t *__restrict__ pool_off,
    int64_t *__restrict__ cigar_off, uint32_t *__restrict__ cigar, int32_t *spill_idx,
    int32_t *spill_count, int8_t *__restrict__ status) {
  const int64_t tw = (int64_t)*tw_p;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = excl[i], b = excl[i + 1];
    cigar_off[i] = a < tw ? a : tw;
    if (i + 1 == n) cigar_off[n] = tw;
    const int32_t r = nruns[i];
    if (r == 0) continue;
    if (b > tw) {
      status[i] = ST_OVERFLOW;
      continue;
    }
    const int64_t pb = r > slot_cap ? pool_off[i] : -1;
    if (r > slot_cap && pb < 0) {
      const int32_t k = atomicAdd(spill_count, 1);
      spill_idx[k] = (int32_t)i;
      continue;
    }
    const uint32_t *src = slot + i * (int64_t)slot_cap;
    uint32_t *dst = cigar + a + r - 1;  // run k goes to dst[-k]
    const int32_t r0 = r < slot_cap ? r : slot_cap;
    for (int32_t k = 0; k < r0; k += 4) {
      const u32x4 v = *reinterpret_cast<const u32x4 *>(src + k);
      dst[-k] = v.x;
      if (k + 1 < r0) dst[-k - 1] = v.y;
      if (k + 2 < r0) dst[-k - 2] = v.z;
      if (k + 3 < r0) dst[-k - 3] = v.w;
    }
    for (int32_t k = r0; k < r; ++k) dst[-k] = pool[pb + (k - slot_cap)];
  }
}

__global__ void k_zero_offsets(int64_t n, int64_t *off) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x)
    off[i] = 0;
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// ---- length buckets: counting sort of pairs, longest first ----
constexpr int NBUCKET = 128;

__device__ __forceinline__ int len_bucket(int32_t m, int32_t n) {
  // 8 buckets per octave of max(m, n); reversed so that long pairs come first
  const uint32_t L = (uint32_t)max(max(m, n), 0) + 1u;
  const int lg = 31 - __clz(L);
  const int frac = lg >= 3 ? (int)((L >> (lg - 3)) & 7u) : (int)((L << (3 - lg)) & 7u);
  const int b = min(lg * 8 + frac, NBUCKET - 1);
  return NBUCKET - 1 - b;
}

__global__ void k_bucket_hist(int64_t n, const int32_t *pl, const int32_t *tl, int32_t *hist) {
  __shared__ int32_t h[NBUCKET];
  for (int k = threadIdx.x; k < NBUCKET; k += blockDim.x) h[k] = 0;
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[len_bucket(pl[i], tl[i])], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < NBUCKET; k += blockDim.x)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

// hist -> exclusive offsets in place (one block)
__global__ void k_bucket_scan(int32_t *hist) {
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int k = 0; k < NBUCKET; ++k) {
      const int32_t v = hist[k];
      hist[k] = acc;
      acc += v;
    }
  }
}

// Per tile of blockDim pairs: ranks within the tile's buckets from LDS
// atomics, then one global atomic per non-empty bucket reserves the tile's
// range (fixed-length batches put nearly every pair in one bucket, where one
// global atomic per pair would serialise).
__global__ __launch_bounds__(256) void k_bucket_scatter(int64_t n, const int32_t *pl, const int32_t *tl,
                                                       int32_t *cursor, int32_t *order) {
  __shared__ int32_t cnt[NBUCKET], base[NBUCKET];
  for (int64_t t0 = blockIdx.x * (int64_t)blockDim.x; t0 < n; t0 += (int64_t)gridDim.x * blockDim.x) {
    for (int k = threadIdx.x; k < NBUCKET; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    const int64_t i = t0 + threadIdx.x;
    int b = 0, r = 0;
    if (i < n) {
      b = len_bucket(pl[i], tl[i]);
      r = atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NBUCKET; k += blockDim.x)
      if (cnt[k]) base[k] = atomicAdd(&cursor[k], cnt[k]);
    __syncthreads();
    if (i < n) order[base[b] + r] = (int32_t)i;
    __syncthreads();
  }
}

inline dim3 grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return dim3((unsigned)g);
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 2); }

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, grid_for(n, 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_pair_flags(int64_t n, int32_t max_len, const int32_t *pl, const int32_t *tl,
                             const int8_t *pf, const int8_t *tf, int8_t *flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_flags, grid_for(n, 256), dim3(256), 0, s, n, max_len, pl, tl, pf, tf,
                     flags);
  return hipGetLastError();
}

hipError_t launch_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *tmp,
                           hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) {
    hipLaunchKernelGGL(k_zero_offsets, dim3(1), dim3(64), 0, s, (int64_t)0, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp, out, nb);
  return hipGetLastError();
}

hipError_t launch_pack(int64_t n, int32_t enc, const uint8_t *seq, const int64_t *off,
                       const int32_t *len, int32_t max_len, uint64_t *words, int64_t words_cap,
                       int64_t *out_off, int8_t *flags, int64_t *scan_tmp, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_offsets, dim3(1), dim3(64), 0, s, (int64_t)0, out_off);
    return hipGetLastError();
  }
  // word counts go into the tail of scan_tmp's companion area: reuse flags-free int32 buffer
  int32_t *cnt = (int32_t *)(scan_tmp + scan_tmp_elems(n));
  hipLaunchKernelGGL(k_word_counts, grid_for(n, 256), dim3(256), 0, s, n, len, max_len, cnt);
  hipError_t err = launch_scan_i32(cnt, n, out_off, scan_tmp, s);
  if (err != hipSuccess) return err;
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, n, enc, seq, off, len, max_len,
                     words, words_cap, out_off, flags, (int64_t)0, (int64_t *)nullptr);
  return hipGetLastError();
}

hipError_t launch_pack_strided(int64_t n, int32_t enc, const uint8_t *seq, const int64_t *off,
                               const int32_t *len, int32_t max_len, uint64_t *words,
                               int64_t words_cap, int64_t *out_off, int8_t *flags, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_offsets, dim3(1), dim3(64), 0, s, (int64_t)0, out_off);
    return hipGetLastError();
  }
  const int64_t stride = ((int64_t)max_len + 31) / 32 > 0 ? ((int64_t)max_len + 31) / 32 : 1;
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, n, enc, seq, off, len, max_len,
                     words, words_cap, (const int64_t *)nullptr, flags, stride, out_off);
  return hipGetLastError();
}

hipError_t launch_compact(int64_t n, const Outs &O, int64_t *cigar_off, uint32_t *cigar,
                          int64_t cigar_cap, int64_t *scan_tmp, int64_t *total_written,
                          int32_t *spill_idx, int32_t *spill_count, int8_t *status,
                          hipStream_t s) {
  // scan_tmp layout: [scan blocks | excl (n+1)]
  int64_t *excl = scan_tmp + scan_tmp_elems(n);
  hipError_t err = launch_scan_i32(O.nruns, n, excl, scan_tmp, s);
  if (err != hipSuccess) return err;
  unsigned long long *tw = (unsigned long long *)total_written;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, tw);
  if (n > 0) {
    hipLaunchKernelGGL(k_cut, grid_for(n, 256), dim3(256), 0, s, n, excl, cigar_cap, tw);
    hipLaunchKernelGGL(k_scatter, grid_for(n, 256), dim3(256), 0, s, n, excl,
                       (const unsigned long long *)tw, O.nruns, O.slot, O.slot_cap, O.pool,
                       O.pool_off, cigar_off, cigar, spill_idx, spill_count, status);
  } else {
    hipLaunchKernelGGL(k_zero_offsets, dim3(1), dim3(64), 0, s, (int64_t)0, cigar_off);
  }
  return hipGetLastError();
}

hipError_t launch_length_sort(int64_t n, const int32_t *pl, const int32_t *tl, int32_t *hist,
                              int32_t *order, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(NBUCKET), 0, s, hist, 0, (int64_t)NBUCKET);
  hipLaunchKernelGGL(k_bucket_hist, grid_for(n, 256), dim3(256), 0, s, n, pl, tl, hist);
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, s, hist);
  hipLaunchKernelGGL(k_bucket_scatter, grid_for(n, 256), dim3(256), 0, s, n, pl, tl, hist, order);
  return hipGetLastError();
}

hipError_t launch_zero_offsets(int64_t n, int64_t *cigar_off, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_offsets, grid_for(n + 1, 256), dim3(256), 0, s, n, cigar_off);
  return hipGetLastError();
}

}  // namespace aim
