// Sensing operators and data-fidelity updates (eq. 2-5; GAP / ADMM).
// All kernels are elementwise or per-row/per-column and bound by HBM traffic.
#include "common.h"
#include "internal.h"

namespace {

constexpr int TPB = 256;

inline int nblk(size_t n, int tpb = TPB) { return (int)((n + tpb - 1) / tpb); }

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}


// ---------------------------------------------------------------- CACTI (eq. 2)
// y = sum_t A_t x_t, summed in frame order.
__global__ void k_cacti_forward(const float* __restrict__ x, const uint8_t* __restrict__ m,
                                float* __restrict__ y, int F, int HW) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  float acc = 0.f;
  for (int t = 0; t < F; ++t)
    if (m[(size_t)t * HW + p]) acc += x[(size_t)t * HW + p];
  y[p] = acc;
}

__global__ void k_cacti_adjoint(const float* __restrict__ y, const uint8_t* __restrict__ m,
                                float* __restrict__ x, int F, int HW) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  float v = y[p];
  for (int t = 0; t < F; ++t) x[(size_t)t * HW + p] = m[(size_t)t * HW + p] ? v : 0.f;
}

// x0 = Phi^T (y / R~), R = sum_t A_t, zeros of R replaced by 1.
__global__ void k_cacti_init(const float* __restrict__ y, const uint8_t* __restrict__ m,
                             float* __restrict__ x, int F, int HW) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  int R = 0;
  for (int t = 0; t < F; ++t) R += m[(size_t)t * HW + p] ? 1 : 0;
  float v = y[p] / (float)(R ? R : 1);
  for (int t = 0; t < F; ++t) x[(size_t)t * HW + p] = m[(size_t)t * HW + p] ? v : 0.f;
}

// GAP: x_bar = x + Phi^T((y - Phi x) / R~).  In-place safe.
// Accelerated GAP (yacc non-null): the measurement is replaced by the
// accumulated one, ya = yacc + (y - Phi x), x_bar = x + Phi^T((ya - Phi x) / R~);
// ya is written back when wacc != 0.
__device__ __forceinline__ float gap_target(float yv, float phi, float* yacc, int p, int wacc) {
  if (!yacc) return yv;
  const float ya = yacc[p] + (yv - phi);
  if (wacc) yacc[p] = ya;
  return ya;
}

__global__ void k_cacti_gap(const float* x, const float* __restrict__ y,
                            const uint8_t* __restrict__ m, float* xo, int F, int HW, float* yacc,
                            int wacc) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  float phi = 0.f;
  int R = 0;
  for (int t = 0; t < F; ++t)
    if (m[(size_t)t * HW + p]) {
      phi += x[(size_t)t * HW + p];
      ++R;
    }
  const float yt = gap_target(y[p], phi, yacc, p, wacc);
  float upd = (yt - phi) / (float)(R ? R : 1);
  for (int t = 0; t < F; ++t) {
    size_t i = (size_t)t * HW + p;
    xo[i] = x[i] + (m[i] ? upd : 0.f);
  }
}

// ---------------------------------------------------------------- MSFA (eq. 4-5)
__device__ __forceinline__ int msfa_band(int r, int c) { return 4 * (r & 3) + (c & 3); }

__global__ void k_msfa_forward(const float* __restrict__ x, float* __restrict__ y, int H, int W) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  y[p] = x[(size_t)msfa_band(r, c) * H * W + p];
}

__global__ void k_msfa_adjoint(const float* __restrict__ y, float* __restrict__ x, int H, int W) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  int b = msfa_band(r, c);
  float v = y[p];
  for (int k = 0; k < 16; ++k) x[(size_t)k * H * W + p] = (k == b) ? v : 0.f;
}

// Replication start: band b = 4*rb + cb takes the sample at (rb, cb) of each 4x4 cell.
__global__ void k_msfa_init(const float* __restrict__ y, float* __restrict__ x, int H, int W) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  int r0 = r & ~3, c0 = c & ~3;
  for (int b = 0; b < 16; ++b) x[(size_t)b * H * W + p] = y[(r0 + (b >> 2)) * W + c0 + (b & 3)];
}

// GAP with Phi Phi^T = I: only the measured band of each pixel moves.
__global__ void k_msfa_gap(const float* x, const float* __restrict__ y, float* xo, int H, int W,
                           float* yacc, int wacc) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  int b = msfa_band(r, c);
  const float yt = gap_target(y[p], x[(size_t)b * H * W + p], yacc, p, wacc);
  for (int k = 0; k < 16; ++k) {
    size_t i = (size_t)k * H * W + p;
    float v = x[i];
    xo[i] = (k == b) ? v + (yt - v) : v;
  }
}

// ---------------------------------------------------------------- FFT (eq. 3)
// Radix-2 Stockham autosort FFT in LDS.  Twiddles exp(-+2 pi i k / n) from
// sincospif on exact dyadic arguments.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One workgroup per row of length n (power of two).  With in2, the row
// transformed is in + beta in2 (the ADMM data step's z - u, fused).
__global__ void k_fft_rows(const float2* in, const float2* in2, float beta, float2* out, int n,
                           int inverse, float scale) {
  extern __shared__ float2 sm[];
  float2* a = sm;
  float2* b = sm + n;
  float2* tw = sm + 2 * n;
  const size_t row = blockIdx.x;
  const int half = n >> 1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float2 v = in[row * n + i];
    if (in2) {
      const float2 w = in2[row * n + i];
      v = make_float2(1.0f * v.x + beta * w.x, 1.0f * v.y + beta * w.y);
    }
    a[i] = v;
  }
  for (int i = threadIdx.x; i < half; i += blockDim.x) {
    float s, c;
    sincospif(-2.0f * (float)i / (float)n, &s, &c);
    tw[i] = make_float2(c, inverse ? -s : s);
  }
  __syncthreads();
  for (int ns = 1; ns < n; ns <<= 1) {
    const int tstride = n / (2 * ns);
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      int k = j & (ns - 1);
      float2 x0 = a[j];
      float2 x1 = cmul(a[j + half], tw[k * tstride]);
      int o = ((j - k) << 1) + k;
      b[o] = make_float2(x0.x + x1.x, x0.y + x1.y);
      b[o + ns] = make_float2(x0.x - x1.x, x0.y - x1.y);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    out[row * n + i] = make_float2(a[i].x * scale, a[i].y * scale);
}

// k-space part of the ADMM x-update: (M y + rho F(z - u)) / (M + rho).
__device__ __forceinline__ float2 admm_kspace(float2 f, bool m, float2 yv, float rho) {
  const float2 yy = m ? yv : make_float2(0.f, 0.f);
  const float den = (m ? 1.f : 0.f) + rho;
  return make_float2((yy.x + rho * f.x) / den, (yy.y + rho * f.y) / den);
}

// One workgroup per `cb` adjacent columns of an n-row array with row stride W.
// Fused epilogues of the ADMM loop (each optional): with ky, the k-space
// update above (lines: the sampled-line mask); with pu, also vp = planar
// form of (result + pu) in [2][n][W].
__global__ void k_fft_cols(float2* data, int n, int W, int cb, int inverse, float scale,
                           const float2* __restrict__ ky, const uint8_t* __restrict__ lines,
                           float rho, const float2* __restrict__ pu, float* __restrict__ vp) {
  extern __shared__ float2 sm[];
  float2* a = sm;
  float2* b = sm + (size_t)n * cb;
  float2* tw = sm + (size_t)2 * n * cb;
  const int c0 = blockIdx.x * cb;
  const int half = n >> 1;
  for (int t = threadIdx.x; t < n * cb; t += blockDim.x) {
    int r = t / cb, cc = t - r * cb;
    a[t] = data[(size_t)r * W + c0 + cc];
  }
  for (int i = threadIdx.x; i < half; i += blockDim.x) {
    float s, c;
    sincospif(-2.0f * (float)i / (float)n, &s, &c);
    tw[i] = make_float2(c, inverse ? -s : s);
  }
  __syncthreads();
  for (int ns = 1; ns < n; ns <<= 1) {
    const int tstride = n / (2 * ns);
    for (int t = threadIdx.x; t < half * cb; t += blockDim.x) {
      int j = t / cb, cc = t - j * cb;
      int k = j & (ns - 1);
      float2 x0 = a[j * cb + cc];
      float2 x1 = cmul(a[(j + half) * cb + cc], tw[k * tstride]);
      int o = ((j - k) << 1) + k;
      b[o * cb + cc] = make_float2(x0.x + x1.x, x0.y + x1.y);
      b[(o + ns) * cb + cc] = make_float2(x0.x - x1.x, x0.y - x1.y);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  const size_t HW = (size_t)n * W;
  for (int t = threadIdx.x; t < n * cb; t += blockDim.x) {
    int r = t / cb, cc = t - r * cb;
    const size_t p = (size_t)r * W + c0 + cc;
    float2 v = make_float2(a[t].x * scale, a[t].y * scale);
    if (ky) v = admm_kspace(v, lines[r] != 0, ky[p], rho);
    data[p] = v;
    if (pu) {
      const float2 w = pu[p];
      vp[p] = 1.0f * v.x + 1.0f * w.x;
      vp[HW + p] = 1.0f * v.y + 1.0f * w.y;
    }
  }
}

__global__ void k_kspace_mask(const float2* __restrict__ in, const uint8_t* __restrict__ lines,
                              float2* __restrict__ out, int H, int W) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  out[p] = lines[p / W] ? in[p] : make_float2(0.f, 0.f);
}

__global__ void k_cplx_axpby(const float2* a, const float2* b, float2* out, float alpha,
                             float beta, int n) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float2 u = a[p], v = b[p];
  out[p] = make_float2(alpha * u.x + beta * v.x, alpha * u.y + beta * v.y);
}

// z <- complex form of the planar zp, then u <- u + x - z
__global__ void k_admm_dual(float2* u, const float2* __restrict__ x, const float* __restrict__ zp,
                            float2* __restrict__ z, int n) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float2 c = make_float2(zp[p], zp[n + p]);
  z[p] = c;
  float2 a = u[p], b = x[p];
  u[p] = make_float2((a.x + b.x) - c.x, (a.y + b.y) - c.y);
}

__global__ void k_to_planar(const float2* __restrict__ z, float* __restrict__ p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 v = z[i];
  p[i] = v.x;
  p[n + i] = v.y;
}

__global__ void k_from_planar(const float* __restrict__ p, float2* __restrict__ z, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  z[i] = make_float2(p[i], p[n + i]);
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n)), dim3(TPB), 0, s, p, v, n);
}
void launch_cacti_forward(const float* x, const uint8_t* m, float* y, int F, int HW, hipStream_t s) {
  hipLaunchKernelGGL(k_cacti_forward, dim3(nblk(HW)), dim3(TPB), 0, s, x, m, y, F, HW);
}
void launch_cacti_adjoint(const float* y, const uint8_t* m, float* x, int F, int HW, hipStream_t s) {
  hipLaunchKernelGGL(k_cacti_adjoint, dim3(nblk(HW)), dim3(TPB), 0, s, y, m, x, F, HW);
}
void launch_cacti_init(const float* y, const uint8_t* m, float* x, int F, int HW, hipStream_t s) {
  hipLaunchKernelGGL(k_cacti_init, dim3(nblk(HW)), dim3(TPB), 0, s, y, m, x, F, HW);
}
void launch_cacti_gap(const float* x, const float* y, const uint8_t* m, float* xo, int F, int HW,
                      float* yacc, int wacc, hipStream_t s) {
  hipLaunchKernelGGL(k_cacti_gap, dim3(nblk(HW)), dim3(TPB), 0, s, x, y, m, xo, F, HW, yacc,
                     wacc);
}
void launch_msfa_forward(const float* x, float* y, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_msfa_forward, dim3(nblk((size_t)H * W)), dim3(TPB), 0, s, x, y, H, W);
}
void launch_msfa_adjoint(const float* y, float* x, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_msfa_adjoint, dim3(nblk((size_t)H * W)), dim3(TPB), 0, s, y, x, H, W);
}
void launch_msfa_init(const float* y, float* x, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_msfa_init, dim3(nblk((size_t)H * W)), dim3(TPB), 0, s, y, x, H, W);
}
void launch_msfa_gap(const float* x, const float* y, float* xo, int H, int W, float* yacc,
                     int wacc, hipStream_t s) {
  hipLaunchKernelGGL(k_msfa_gap, dim3(nblk((size_t)H * W)), dim3(TPB), 0, s, x, y, xo, H, W, yacc,
                     wacc);
}

// Orthonormal 2-D DFT: rows then columns, each scaled by 1/sqrt(length).
void launch_fft2d(const float2* in, float2* out, int H, int W, int inverse, hipStream_t s,
                  const FftFuse* f) {
  const FftFuse none{};
  if (!f) f = &none;
  size_t lds_r = (size_t)(2 * W + W / 2) * sizeof(float2);
  hipLaunchKernelGGL(k_fft_rows, dim3(H), dim3(TPB), lds_r, s, in, f->in2, f->beta, out, W,
                     inverse, 1.0f / sqrtf((float)W));
  int cb = 1;
  while (cb * 2 <= 16 && (size_t)(cb * 2) * H * 2 * sizeof(float2) + (size_t)H / 2 * sizeof(float2) <= 48 * 1024 &&
         W % (cb * 2) == 0)
    cb *= 2;
  size_t lds_c = ((size_t)2 * H * cb + H / 2) * sizeof(float2);
  hipLaunchKernelGGL(k_fft_cols, dim3(W / cb), dim3(TPB), lds_c, s, out, H, W, cb, inverse,
                     1.0f / sqrtf((float)H), f->ky, f->lines, f->rho, f->pu, f->vp);
}
void launch_kspace_mask(const float2* in, const uint8_t* lines, float2* out, int H, int W,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_kspace_mask, dim3(nblk((size_t)H * W)), dim3(TPB), 0, s, in, lines, out, H, W);
}
void launch_cplx_axpby(const float2* a, const float2* b, float2* out, float alpha, float beta,
                       int n, hipStream_t s) {
  hipLaunchKernelGGL(k_cplx_axpby, dim3(nblk(n)), dim3(TPB), 0, s, a, b, out, alpha, beta, n);
}
void launch_admm_dual(float2* u, const float2* x, const float* zp, float2* z, int n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_admm_dual, dim3(nblk(n)), dim3(TPB), 0, s, u, x, zp, z, n);
}
void launch_to_planar(const float2* z, float* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_planar, dim3(nblk(n)), dim3(TPB), 0, s, z, p, n);
}
void launch_from_planar(const float* p, float2* z, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_from_planar, dim3(nblk(n)), dim3(TPB), 0, s, p, z, n);
}

// ---------------------------------------------------------------- surrogate judge
namespace {
__global__ void k_fill_f32(float* p, float v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_stride_keys(const int32_t* __restrict__ keys, int n, int stride,
                              int32_t* __restrict__ sub) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i * stride < n) sub[i] = keys[i * stride];
}
constexpr int JB = 256, JN = 512;
// part[blk] = (sum over covered pixels and channels of (a - b)^2, of b^2,
// count of non-finite a anywhere)
__global__ void __launch_bounds__(JB)
k_judge_part(const float* __restrict__ a, const float* __restrict__ b,
             const int32_t* __restrict__ cover, int C, int HW, float* __restrict__ part) {
  __shared__ float s0[JB], s1[JB], s2[JB];
  float n = 0.f, d = 0.f, bad = 0.f;
  const size_t tot = (size_t)C * HW;
  for (size_t i = (size_t)blockIdx.x * JB + threadIdx.x; i < tot; i += (size_t)JN * JB) {
    const float av = a[i], bv = b[i];
    if (!isfinite(av)) bad += 1.f;
    if (cover[i % HW] > 0) {
      const float e = av - bv;
      n = fmaf(e, e, n);
      d = fmaf(bv, bv, d);
    }
  }
  s0[threadIdx.x] = n;
  s1[threadIdx.x] = d;
  s2[threadIdx.x] = bad;
  __syncthreads();
  for (int o = JB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s0[0];
    part[3 * blockIdx.x + 1] = s1[0];
    part[3 * blockIdx.x + 2] = s2[0];
  }
}
__global__ void k_judge_final(const float* __restrict__ part, float* __restrict__ delta) {
  if (threadIdx.x != 0) return;
  double n = 0.0, d = 0.0, bad = 0.0;
  for (int k = 0; k < JN; ++k) {
    n += part[3 * k];
    d += part[3 * k + 1];
    bad += part[3 * k + 2];
  }
  const bool inf = bad > 0.0 || !(d > 0.0) || !isfinite(n);
  delta[0] = inf ? __int_as_float(0x7f800000) : (float)(sqrt(n) / sqrt(d));
}
}  // namespace

void launch_fill_f32(float* p, float v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}
void launch_stride_keys(const int32_t* keys, int n, int stride, int32_t* sub, hipStream_t s) {
  const int m = (n + stride - 1) / stride;
  hipLaunchKernelGGL(k_stride_keys, dim3((m + 255) / 256), dim3(256), 0, s, keys, n, stride, sub);
}
void launch_judge(const float* a, const float* b, const int32_t* cover, int C, int HW,
                  float* part, float* delta, hipStream_t s) {
  hipLaunchKernelGGL(k_judge_part, dim3(JN), dim3(JB), 0, s, a, b, cover, C, HW, part);
  hipLaunchKernelGGL(k_judge_final, dim3(1), dim3(64), 0, s, part, delta);
}
