// Small device helpers shared by the DP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aim {
namespace dev {

constexpr uint64_t K55 = 0x5555555555555555ull;

__device__ __forceinline__ uint64_t ld_word(const uint64_t *s, int64_t nw, int64_t q) {
  return (q >= 0 && q < nw) ? s[q] : 0ull;
}

// 32 bases starting at base index s0 (which may lie outside the sequence;
// missing words read as zero -- those cells are never used).
__device__ __forceinline__ uint64_t window32(const uint64_t *s, int64_t nw, int64_t s0) {
  const int64_t q = s0 >> 5;
  const uint32_t r = (uint32_t)(s0 & 31);
  const uint64_t w0 = ld_word(s, nw, q), w1 = ld_word(s, nw, q + 1);
  return r ? ((w0 >> (2 * r)) | (w1 << (64 - 2 * r))) : w0;
}

// even bits of w gathered into 32 bits (bit 2i -> bit i)
__device__ __forceinline__ uint32_t even_bits(uint64_t w) {
  w &= K55;
  w = (w | (w >> 1)) & 0x3333333333333333ull;
  w = (w | (w >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  w = (w | (w >> 4)) & 0x00FF00FF00FF00FFull;
  w = (w | (w >> 8)) & 0x0000FFFF0000FFFFull;
  w = (w | (w >> 16)) & 0x00000000FFFFFFFFull;
  return (uint32_t)w;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s));
  return v;
}

// Append the calling lanes with `pred` to a device list, one atomic per wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t value, int32_t *list, int32_t *count) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, (int)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = value;
}

}  // namespace dev
}  // namespace aim
