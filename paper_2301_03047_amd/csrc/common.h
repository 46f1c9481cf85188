// Device helpers shared by the libglr kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GLR_WAVE 64

// ------------------------------------------------------------------ wave ops
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int wave_sum_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one int per thread.  `scratch` holds at least
// (blockDim.x / 64 + 1) ints of LDS.  Returns the exclusive prefix; *total
// receives the block sum.  Every thread of the block must call it.
__device__ __forceinline__ int block_excl_scan(int v, int* scratch, int* total) {
  const int l = lane_id();
  const int w = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  int incl = wave_incl_scan(v);
  if (l == 63) scratch[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < nw; ++i) {
      int t = scratch[i];
      scratch[i] = run;
      run += t;
    }
    scratch[nw] = run;
  }
  __syncthreads();
  int res = scratch[w] + incl - v;
  *total = scratch[nw];
  __syncthreads();
  return res;
}

// ------------------------------------------------------------------ orderings
// Monotone map float -> uint32 (total order, -0 < +0, NaN above +inf).
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  uint32_t b = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(b);
}

// ------------------------------------------------------------------ rescored distances
// A rescored distance s (FP64) is carried as the FP32 pair (hi, lo) =
// (fl32(s), fl32(s - hi)); pairs order lexicographically as s does.
struct df32 {
  float hi, lo;
};

// lexicographic (hi, lo, j) order of rescored candidates
__device__ __forceinline__ bool df_less(float ah, float al, int aj, float bh, float bl, int bj) {
  if (ah != bh) return ah < bh;
  if (al != bl) return al < bl;
  return aj < bj;
}
