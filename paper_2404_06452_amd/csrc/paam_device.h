// Device helpers shared by the kernels of libpaam: the candidate-order walk
// of the priority search and bfloat16 rounding.  Every function here runs in
// a one-wave workgroup (64 lanes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace paam {

// SplitMix64 [Steele, Lea & Flood 2014]: the output function, and output m of
// the stream of a set, whose state starts at mix(seed + G*(set+1)) and
// advances by G per output.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t swap_stream(uint64_t seed, int64_t set, uint64_t m) {
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  return splitmix_mix(splitmix_mix(seed + G * (uint64_t)(set + 1)) + G * (m + 1));
}

// Positions exchanged by swap q >= 1 of the walk over C >= 2 chains:
// i = u1 mod C, j = (i + 1 + u2 mod (C-1)) mod C with u1, u2 the stream
// outputs 2q-2 and 2q-1.  Packed as i | j << 16.
__device__ __forceinline__ int32_t swap_positions(uint64_t seed, int64_t set, int64_t q, int C) {
  const uint64_t u1 = swap_stream(seed, set, 2 * (uint64_t)(q - 1));
  const uint64_t u2 = swap_stream(seed, set, 2 * (uint64_t)(q - 1) + 1);
  const int i = (int)(u1 % (uint64_t)C);
  const int j = (int)((i + 1 + (int64_t)(u2 % (uint64_t)(C - 1))) % C);
  return i | (j << 16);
}

// Advances a candidate order from candidate k_from to k_to >= k_from:
// order[r] = chain at rank r, rank[c] = rank of chain c.  The lanes compute
// the swap positions of 64 steps at a time; every lane then follows the
// positions of its own chains (lane, lane + 64, ...: up to 256 per pass)
// through those swaps, reading each swap from a register of the lane that
// computed it, and finally writes their ranks and the order.  Called by all
// lanes; ends synchronised.  buf is unused (kept for the callers' layout).
__device__ inline void walk_order(int32_t *order, int16_t *rank, int C, uint64_t seed, int64_t set,
                                  int64_t k_from, int64_t k_to, int32_t *buf) {
  (void)buf;
  if (C < 2 || k_to <= k_from) return;
  const int lane = threadIdx.x;
  for (int cb = 0; cb < C; cb += 4 * 64) {
    int pos[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = cb + lane + 64 * j;
      pos[j] = c < C ? rank[c] : -1;
    }
    for (int64_t q0 = k_from + 1; q0 <= k_to; q0 += 64) {
      const int64_t q = q0 + lane;
      const int32_t sw = q <= k_to ? swap_positions(seed, set, q, C) : 0;
      const int n = (int)((k_to - q0 + 1) < 64 ? (k_to - q0 + 1) : 64);
      for (int t = 0; t < n; ++t) {
        const int32_t st = __builtin_amdgcn_readlane(sw, t);
        const int pa = st & 0xffff, pb = st >> 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) pos[j] = pos[j] == pa ? pb : (pos[j] == pb ? pa : pos[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = cb + lane + 64 * j;
      if (c < C) {
        rank[c] = (int16_t)pos[j];
        order[pos[j]] = c;
      }
    }
  }
  __syncthreads();
}

// float -> bfloat16 bit pattern, round to nearest, ties to even (finite input).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

}  // namespace paam
