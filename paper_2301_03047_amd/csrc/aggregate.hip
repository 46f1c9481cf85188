// Aggregation of the group estimates back into the image (the grouping
// operator's adjoint for the low-rank objective of the Method section).
// Reading: every member estimate weighs 1; a pixel is the mean of all
// estimates covering it; uncovered pixels keep the pre-prior value.
//
// Atomic-free and deterministic: entries e = g*K + q are sorted by
// (position, e) with a bitonic network on unique 64-bit keys, CSR offsets per
// position come from binary searches, and each pixel gathers its covering
// estimates in a fixed order (dy, dx, e ascending).
#include "common.h"
#include "internal.h"

namespace {

constexpr int LT = 1024;          // threads of the local sort kernels
constexpr int LN = 2 * LT;        // elements sorted in LDS per block

__global__ void k_pairs(const int32_t* __restrict__ idx, int M, int M2,
                        unsigned long long* __restrict__ keys) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M2) return;
  keys[e] = e < M ? (((unsigned long long)(uint32_t)idx[e]) << 32) | (uint32_t)e : ~0ull;
}

__device__ __forceinline__ void cmpx(unsigned long long* s, int i, int p, bool up) {
  unsigned long long a = s[i], b = s[p];
  if ((a > b) == up) {
    s[i] = b;
    s[p] = a;
  }
}

// all stages k <= LN within each 2048-element block
__global__ void __launch_bounds__(LT) k_bitonic_local_sort(unsigned long long* __restrict__ keys) {
  __shared__ unsigned long long s[LN];
  const size_t base = (size_t)blockIdx.x * LN;
  s[threadIdx.x] = keys[base + threadIdx.x];
  s[threadIdx.x + LT] = keys[base + threadIdx.x + LT];
  __syncthreads();
  for (int k = 2; k <= LN; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < LN; t += LT) {
        int p = t ^ j;
        if (p > t) cmpx(s, t, p, (((size_t)base + t) & k) == 0);
      }
      __syncthreads();
    }
  keys[base + threadIdx.x] = s[threadIdx.x];
  keys[base + threadIdx.x + LT] = s[threadIdx.x + LT];
}

// stage (k, j) with j >= LN: pairs span blocks
__global__ void k_bitonic_global(unsigned long long* __restrict__ keys, size_t n, size_t k, size_t j) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  size_t p = i ^ j;
  if (p > i) {
    bool up = (i & k) == 0;
    unsigned long long a = keys[i], b = keys[p];
    if ((a > b) == up) {
      keys[i] = b;
      keys[p] = a;
    }
  }
}

// stages j < LN of merge step k (k > LN) inside each block
__global__ void __launch_bounds__(LT) k_bitonic_local_merge(unsigned long long* __restrict__ keys,
                                                            size_t k) {
  __shared__ unsigned long long s[LN];
  const size_t base = (size_t)blockIdx.x * LN;
  s[threadIdx.x] = keys[base + threadIdx.x];
  s[threadIdx.x + LT] = keys[base + threadIdx.x + LT];
  __syncthreads();
  const bool up = (base & k) == 0;      // constant within the block since k > LN
  for (int j = LN >> 1; j > 0; j >>= 1) {
    for (int t = threadIdx.x; t < LN; t += LT) {
      int p = t ^ j;
      if (p > t) cmpx(s, t, p, up);
    }
    __syncthreads();
  }
  keys[base + threadIdx.x] = s[threadIdx.x];
  keys[base + threadIdx.x + LT] = s[threadIdx.x + LT];
}

// offs[t] = first sorted entry whose position is >= t, t in [0, Ncand]
__global__ void k_offsets(const unsigned long long* __restrict__ keys, int M, int Ncand,
                          int32_t* __restrict__ offs) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > Ncand) return;
  int lo = 0, hi = M;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if ((int)(keys[mid] >> 32) < t) lo = mid + 1; else hi = mid;
  }
  offs[t] = lo;
}

constexpr int CB = 8;             // channels per gather block
constexpr int GX = 64;            // pixels per gather block (one image row segment)

// One thread per (pixel, dy): sums the estimates of the patches whose top
// row covers the pixel at offset dy, over dx and the CSR bucket; the P
// partial sums of a pixel are then added in dy order (fixed order).
__global__ void k_gather(const float* __restrict__ xbar, const float* __restrict__ xhat,
                         const unsigned long long* __restrict__ keys,
                         const int32_t* __restrict__ offs, int Cp, int H, int W, int P, int D,
                         int K, float* __restrict__ out, int32_t* __restrict__ cover) {
  extern __shared__ float part[];          // [P][GX][CB + 1]
  const int tx = threadIdx.x, dy = threadIdx.y;
  const int r = blockIdx.y;
  const int c = blockIdx.x * GX + tx;
  const int cb = blockIdx.z;
  const int Hc = H - P + 1, Wc = W - P + 1;
  const int PP = P * P;
  const int nch = min(CB, Cp - cb * CB);
  float acc[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u) acc[u] = 0.f;
  int cnt = 0;
  const int gr = r - dy;
  if (c < W && gr >= 0 && gr < Hc) {
    for (int dx = 0; dx < P; ++dx) {
      const int gc = c - dx;
      if (gc < 0 || gc >= Wc) continue;
      const int t = gr * Wc + gc;
      const int a = offs[t], b = offs[t + 1];
      cnt += b - a;
      for (int i = a; i < b; ++i) {
        // entry e = g*K + j; estimates are entry-major: xhat[e*D + d]
        const uint32_t e = (uint32_t)(keys[i] & 0xffffffffull);
        const float* src = xhat + (size_t)e * D + (size_t)(cb * CB) * PP + dy * P + dx;
#pragma unroll
        for (int u = 0; u < CB; ++u)
          if (u < nch) acc[u] += src[(size_t)u * PP];
      }
    }
  }
  float* mine = part + ((size_t)dy * GX + tx) * (CB + 1);
#pragma unroll
  for (int u = 0; u < CB; ++u) mine[u] = acc[u];
  mine[CB] = __int_as_float(cnt);
  __syncthreads();
  if (dy == 0 && c < W) {
    float sum[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) sum[u] = 0.f;
    int n = 0;
    for (int y = 0; y < P; ++y) {
      const float* pp = part + ((size_t)y * GX + tx) * (CB + 1);
#pragma unroll
      for (int u = 0; u < CB; ++u) sum[u] += pp[u];
      n += __float_as_int(pp[CB]);
    }
    const size_t HW = (size_t)H * W;
    if (cover && cb == 0) cover[(size_t)r * W + c] = n;
    for (int u = 0; u < nch; ++u) {
      const size_t o = (size_t)(cb * CB + u) * HW + (size_t)r * W + c;
      out[o] = n ? sum[u] / (float)n : xbar[o];
    }
  }
}

}  // namespace

void launch_aggregate(const glr_plan* pl, const float* xbar, const int32_t* idx,
                      const float* xhat, unsigned long long* pairs, int32_t* offs, float* out,
                      int32_t* cover, hipStream_t s) {
  const int M = pl->M, M2 = pl->M2;
  hipLaunchKernelGGL(k_pairs, dim3((M2 + 255) / 256), dim3(256), 0, s, idx, M, M2, pairs);
  hipLaunchKernelGGL(k_bitonic_local_sort, dim3(M2 / LN), dim3(LT), 0, s, pairs);
  for (size_t k = 2 * LN; k <= (size_t)M2; k <<= 1) {
    for (size_t j = k >> 1; j >= (size_t)LN; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_global, dim3((M2 + 255) / 256), dim3(256), 0, s, pairs,
                         (size_t)M2, k, j);
    hipLaunchKernelGGL(k_bitonic_local_merge, dim3(M2 / LN), dim3(LT), 0, s, pairs, k);
  }
  hipLaunchKernelGGL(k_offsets, dim3((pl->Ncand + 1 + 255) / 256), dim3(256), 0, s, pairs, M,
                     pl->Ncand, offs);
  dim3 grid((pl->W + GX - 1) / GX, pl->H, (pl->Cp + CB - 1) / CB);
  const size_t lds = (size_t)pl->P * GX * (CB + 1) * sizeof(float);
  hipLaunchKernelGGL(k_gather, grid, dim3(GX, pl->P), lds, s, xbar, xhat, pairs, offs, pl->Cp,
                     pl->H, pl->W, pl->P, pl->D, pl->K, out, cover);
}
