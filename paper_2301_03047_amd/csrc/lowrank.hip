// Low-rank step: WNNM shrinkage of every patch group (the rank-minimisation
// objective of the Method section, solved by weighted nuclear-norm
// minimisation [Gu et al. 2014]).
//
// One workgroup per group Y (D x K, column q = member patch q):
//  1. row means mu and Yc = Y - mu 1^T, streamed in chunks of 64 rows;
//  2. R = triangular factor of Yc by a streaming (TSQR-style) Householder QR:
//     each chunk B is folded into the running R by eliminating [R; B];
//  3. one-sided Jacobi SVD of R (columns orthogonalised in a round-robin
//     order, rotation angles computed in FP64), accumulating V;  R and Yc
//     share singular values and right singular vectors;
//  4. WNNM: sigma_hat = sqrt(max(s^2 - K sigma^2, 0)),
//     tau = c sqrt(K) sigma^2 / (sigma_hat + eps), s' = max(s - tau, 0);
//  5. X = Y - Yc W with W = V diag((s - s')/s) V^T, i.e. the residual
//     sum_i (s_i - s'_i) u_i v_i^T, accumulated in FP64 (sigma = 0 gives
//     W = 0 and X = Y exactly).
// Data and the SVD are FP32; only the angles and the residual use FP64.
#include "common.h"
#include "internal.h"

namespace {

constexpr int WT = 256;
constexpr int KMAX = 64;
constexpr int BR = 64;           // rows per streamed chunk
constexpr int RS = KMAX + 1;     // LDS row stride

struct GroupGeom {
  int H, W, P, Cp, D, K;
  size_t HW;
};

// image offset of row d of member patch with top-left pixel offset `base`
__device__ __forceinline__ size_t elem_off(const GroupGeom& G, int base, int d) {
  const int PP = G.P * G.P;
  int ch = d / PP;
  int rem = d - ch * PP;
  int dy = rem / G.P, dx = rem - dy * G.P;
  return (size_t)ch * G.HW + base + dy * G.W + dx;
}

// Load rows [d0, d0+nb) of Y into B (raw values) and their means into smu.
__device__ void load_chunk(const GroupGeom& G, const float* __restrict__ xp, const int* spos, int d0,
                           int nb, float* B, float* smu) {
  const int K = G.K;
  for (int e = threadIdx.x; e < nb * K; e += WT) {
    int i = e % nb, j = e / nb;
    B[i * RS + j] = xp[elem_off(G, spos[j], d0 + i)];
  }
  __syncthreads();
  if (threadIdx.x < nb) {
    const int i = threadIdx.x;
    float s = 0.f;
    for (int j = 0; j < K; ++j) s += B[i * RS + j];
    smu[i] = s / (float)K;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(WT)
k_wnnm(const float* __restrict__ xp, int H, int W, int P, int Cp, int D,
       const int32_t* __restrict__ idx, int K, float sigma, float wc, float weps, int max_sweeps,
       float* __restrict__ xhat, float* __restrict__ sv, DevStats* st) {
  __shared__ float Rm[KMAX * RS];
  __shared__ float Vm[KMAX * RS];
  __shared__ float Bm[BR * RS];
  __shared__ float red[4][KMAX];
  __shared__ float smu[BR];
  __shared__ float swt[KMAX];
  __shared__ float ssig[KMAX];
  __shared__ int spos[KMAX];
  __shared__ int sflag[3];

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int Wc = W - P + 1;
  GroupGeom G{H, W, P, Cp, D, K, (size_t)H * W};

  if (tid < K) {
    int t = idx[(size_t)g * K + tid];
    int r = t / Wc, c = t - r * Wc;
    spos[tid] = r * W + c;
  }
  for (int e = tid; e < KMAX * RS; e += WT) {
    Rm[e] = 0.f;
    Vm[e] = 0.f;
  }
  if (tid < 3) sflag[tid] = 0;
  __syncthreads();

  // ---- 1-2: streamed Householder QR of Yc
  const int jc = tid & 63, part = tid >> 6;
  for (int d0 = 0; d0 < D; d0 += BR) {
    const int nb = min(BR, D - d0);
    load_chunk(G, xp, spos, d0, nb, Bm, smu);
    for (int e = tid; e < nb * K; e += WT) {
      int i = e % nb, j = e / nb;
      Bm[i * RS + j] -= smu[i];
    }
    __syncthreads();
    const int q = (nb + 3) / 4;
    const int i0 = part * q, i1 = min(nb, i0 + q);
    for (int k = 0; k < K; ++k) {
      if (jc >= k && jc < K) {
        float p = 0.f;
        for (int i = i0; i < i1; ++i) p += Bm[i * RS + k] * Bm[i * RS + jc];
        red[part][jc] = p;
      }
      __syncthreads();
      const float sig2 = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
      float beta = 0.f, v0 = 0.f, alpha = 0.f, w = 0.f;
      const bool active = sig2 > 0.f;
      if (active) {
        const float x0 = Rm[k * RS + k];
        const float nrm = sqrtf(x0 * x0 + sig2);
        alpha = x0 >= 0.f ? -nrm : nrm;
        v0 = x0 - alpha;
        beta = 2.0f / (v0 * v0 + sig2);
        if (jc > k && jc < K)
          w = v0 * Rm[k * RS + jc] + (((red[0][jc] + red[1][jc]) + red[2][jc]) + red[3][jc]);
      }
      __syncthreads();
      if (active) {
        if (jc > k && jc < K) {
          const float bw = beta * w;
          for (int i = i0; i < i1; ++i) Bm[i * RS + jc] -= bw * Bm[i * RS + k];
          if (part == 0) Rm[k * RS + jc] -= bw * v0;
        }
        if (jc == k && part == 0) Rm[k * RS + k] = alpha;
      }
      __syncthreads();
    }
  }

  // ---- 3: one-sided Jacobi on the columns of R, V accumulated
  for (int e = tid; e < K; e += WT) Vm[e * RS + e] = 1.0f;
  __syncthreads();
  const int Kp = K + (K & 1);
  const int npairs = Kp / 2;
  const int pr = tid >> 3, sub = tid & 7;
  const float tol = (float)K * 5.9604644775390625e-08f;
  int sweeps = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // three flag slots: this sweep writes sw%3, the next one is cleared now,
    // and the slot read at the end of the previous sweep is left alone
    if (tid == 0) sflag[(sw + 1) % 3] = 0;
    for (int round = 0; round < Kp - 1; ++round) {
      int a = -1, b = -1;
      if (pr < npairs) {
        a = pr == 0 ? 0 : 1 + ((pr - 1 + round) % (Kp - 1));
        int m2 = Kp - 1 - pr;
        b = m2 == 0 ? 0 : 1 + ((m2 - 1 + round) % (Kp - 1));
      }
      const bool valid = pr < npairs && a < K && b < K;
      float al = 0.f, be = 0.f, ga = 0.f;
      if (valid)
        for (int i = sub; i < K; i += 8) {
          float x = Rm[i * RS + a], y = Rm[i * RS + b];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
      // butterfly over the 8 lanes of the pair: identical sums in every lane
      for (int o = 1; o < 8; o <<= 1) {
        al += __shfl_xor(al, o, 64);
        be += __shfl_xor(be, o, 64);
        ga += __shfl_xor(ga, o, 64);
      }
      if (valid && ga != 0.f && fabsf(ga) > tol * sqrtf(al) * sqrtf(be)) {
        const double zeta = ((double)be - (double)al) / (2.0 * (double)ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const float c = (float)cs, s = (float)(cs * t);
        for (int i = sub; i < K; i += 8) {
          float x = Rm[i * RS + a], y = Rm[i * RS + b];
          Rm[i * RS + a] = c * x - s * y;
          Rm[i * RS + b] = s * x + c * y;
          float vx = Vm[i * RS + a], vy = Vm[i * RS + b];
          Vm[i * RS + a] = c * vx - s * vy;
          Vm[i * RS + b] = s * vx + c * vy;
        }
        if (sub == 0) sflag[sw % 3] = 1;
      }
      __syncthreads();
    }
    sweeps = sw + 1;
    if (sflag[sw % 3] == 0) break;
  }
  __syncthreads();

  // ---- 4: singular values and WNNM factors
  if (tid < K) {
    float s2 = 0.f;
    for (int i = 0; i < K; ++i) s2 += Rm[i * RS + tid] * Rm[i * RS + tid];
    const float s = sqrtf(s2);
    const float shat = sqrtf(fmaxf(s * s - (float)K * sigma * sigma, 0.f));
    const float tau = wc * sqrtf((float)K) * sigma * sigma / (shat + weps);
    const float sn = fmaxf(s - tau, 0.f);
    ssig[tid] = s;
    swt[tid] = s > 0.f ? (s - sn) / s : 0.f;
  }
  __syncthreads();
  if (sv && tid < K) {
    const float s = ssig[tid];
    int rank = 0;
    for (int i = 0; i < K; ++i) rank += (ssig[i] > s || (ssig[i] == s && i < tid)) ? 1 : 0;
    sv[(size_t)g * K + rank] = s;
  }
  if (tid == 0 && st) atomicMax(&st->sweeps_max, sweeps);
  // W = V diag(w) V^T into Rm
  for (int e = tid; e < K * K; e += WT) {
    const int a = e / K, b = e - a * K;
    float acc = 0.f;
    for (int i = 0; i < K; ++i) acc += Vm[a * RS + i] * swt[i] * Vm[b * RS + i];
    Rm[a * RS + b] = acc;
  }
  __syncthreads();

  // ---- 5: X = Y - Yc W, residual accumulated in FP64
  for (int d0 = 0; d0 < D; d0 += BR) {
    const int nb = min(BR, D - d0);
    load_chunk(G, xp, spos, d0, nb, Bm, smu);
    for (int e = tid; e < nb * K; e += WT) {
      const int i = e % nb, j = e / nb;
      const float mu = smu[i];
      double res = 0.0;
      for (int k = 0; k < K; ++k) res += (double)(Bm[i * RS + k] - mu) * (double)Rm[k * RS + j];
      xhat[((size_t)g * K + j) * D + d0 + i] = (float)((double)Bm[i * RS + j] - res);
    }
    __syncthreads();
  }
}

}  // namespace

void launch_wnnm(const glr_plan* pl, const float* xp, const int32_t* idx, float sigma,
                 float* xhat, float* sv, DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_wnnm, dim3(pl->N), dim3(WT), 0, s, xp, pl->H, pl->W, pl->P, pl->Cp, pl->D,
                     idx, pl->K, sigma, pl->wnnm_c, pl->wnnm_eps, 30, xhat, sv, st);
}
