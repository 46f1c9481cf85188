// Residual CNN surrogate of the GLR prior step: x_out = x + f(x, sigma),
// f = five 3x3 convolutions (2 -> 64 -> 64 -> 64 -> 64 -> 1, zero padding,
// ReLU after the first four), BF16 weights and activations, FP32 sums.
//
// Layouts: activations NHWC bf16 [B][h][w][C] (C = 16 for the packed
// network input, channels 2..15 zero; 64 for hidden layers).  Parameters:
// one flat FP32 vector W1 [64][2][3][3], b1 [64], ..., W5 [1][64][3][3], b5.
// Packed weights (bf16): forward Wf_l [9][64 co][CIP] (tap = 3 dy + dx),
// data-gradient Wd_l [9][64 ci][64 co] with the taps flipped, W5 [9][64];
// followed by the FP32 biases.
//
// Hidden layers run as implicit GEMMs on v_mfma_f32_32x32x16_bf16:
//  forward / data gradient: M = 128 pixels of an image row (4 waves x 32),
//    N = 64 output channels, K = 9 taps x input channels; the block walks
//    down RB rows with a 3-row halo ring in LDS, weights resident in LDS;
//  weight gradient: M = 64 output channels, N = input channels, K = pixels
//    (64-pixel row segments, both operands transposed into LDS so the
//    pixel dimension is contiguous; three copies of the input shifted by
//    dx keep every fragment read 16-byte aligned); per-block partial sums
//    are reduced in a fixed order (no atomics).
// The 64 -> 1 output layer and its gradients are VALU kernels.
#include <cmath>

#include "common.h"
#include "internal.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int CH = 64;

__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);        // round to nearest even
}
__device__ __forceinline__ float from_bf16(uint16_t u) {
  return __uint_as_float((uint32_t)u << 16);
}

// ---------------------------------------------------------------- input / weights
// in16[p][0] = x[p], in16[p][1] = sigma[b], channels 2..15 = 0 (bf16)
__global__ void k_pack_input(const float* __restrict__ x, const float* __restrict__ sigma, int HW,
                             size_t P, uint16_t* __restrict__ in16) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int b = (int)(p / HW);
  uint4 v0 = make_uint4(0, 0, 0, 0), v1 = make_uint4(0, 0, 0, 0);
  v0.x = (uint32_t)to_bf16(x[p]) | ((uint32_t)to_bf16(sigma[b]) << 16);
  uint4* o = reinterpret_cast<uint4*>(in16 + p * 16);
  o[0] = v0;
  o[1] = v1;
}

// Packed weight offsets (bf16 elements) and bias offsets (floats after them).
struct Pack {
  static constexpr size_t wf1 = 0;                            // [9][64][16]
  static constexpr size_t wf2 = wf1 + 9 * 64 * 16;            // [9][64][64] x3
  static constexpr size_t wd2 = wf2 + 3 * 9 * 64 * 64;        // [9][64][64] x3
  static constexpr size_t w5 = wd2 + 3 * 9 * 64 * 64;         // [9][64]
  static constexpr size_t nbf = w5 + 9 * 64;
  static constexpr size_t bias_bytes_off = (nbf * 2 + 255) / 256 * 256;
  static constexpr size_t nbias = 4 * 64 + 1;
  static constexpr size_t bytes = bias_bytes_off + (nbias * 4 + 255) / 256 * 256;
};
// flat parameter offsets
__host__ __device__ constexpr size_t poff_w(int l) {
  return l == 0 ? 0 : (l == 1 ? 1216 : (l == 2 ? 38144 : (l == 3 ? 75072 : 112000)));
}
__host__ __device__ constexpr size_t poff_b(int l) {
  return l == 0 ? 1152 : (l == 1 ? 38080 : (l == 2 ? 75008 : (l == 3 ? 111936 : 112576)));
}
constexpr int NPARAM = 112577;

__global__ void k_pack_weights(const float* __restrict__ th, uint16_t* __restrict__ pk,
                               float* __restrict__ bias) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // forward packs
  if (i < 9 * 64 * 16) {                                       // layer 1
    const int t = i / (64 * 16), co = (i / 16) % 64, ci = i % 16;
    const float w = ci < 2 ? th[poff_w(0) + (co * 2 + ci) * 9 + t] : 0.f;
    pk[Pack::wf1 + i] = to_bf16(w);
  }
  if (i < 3 * 9 * 64 * 64) {
    const int l = 1 + i / (9 * 64 * 64), r = i % (9 * 64 * 64);
    const int t = r / (64 * 64), a = (r / 64) % 64, c = r % 64;
    // forward: [t][co = a][ci = c] = W[a][c][t]
    pk[Pack::wf2 + i] = to_bf16(th[poff_w(l) + ((size_t)a * 64 + c) * 9 + t]);
    // data gradient: [t][ci = a][co = c] = W[c][a][8 - t]
    pk[Pack::wd2 + i] = to_bf16(th[poff_w(l) + ((size_t)c * 64 + a) * 9 + (8 - t)]);
  }
  if (i < 9 * 64) {
    const int t = i / 64, c = i % 64;
    pk[Pack::w5 + i] = to_bf16(th[poff_w(4) + c * 9 + t]);
  }
  if (i < 4 * 64) bias[i] = th[poff_b(i / 64) + i % 64];
  if (i == 0) bias[256] = th[poff_b(4)];
}

// ---------------------------------------------------------------- conv (MFMA)
constexpr int TW = 128;          // pixels per block row segment
constexpr int RB = 8;            // rows per block

// MODE 0: out = bf16(relu(acc + bias[co])); MODE 1: out = bf16(acc * (mask > 0))
template <int CIP, int MODE>
__global__ void __launch_bounds__(256)
k_conv_mfma(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
            const float* __restrict__ bias, const uint16_t* __restrict__ mask, int B, int h,
            int w, uint16_t* __restrict__ out) {
  constexpr int CS = CIP + 8;                 // LDS row stride (bf16)
  constexpr int HW_ = TW + 2;                 // halo row length
  constexpr int NK = CIP / 16;                // K chunks per tap
  __shared__ __align__(16) uint16_t Wl[9 * 64 * CS];
  __shared__ __align__(16) uint16_t Hr[3 * HW_ * CS];

  const int ntc = (w + TW - 1) / TW;
  const int nrb = (h + RB - 1) / RB;
  int bid = blockIdx.x;
  const int ct = bid % ntc;
  bid /= ntc;
  const int rb = bid % nrb;
  const int b = bid / nrb;
  const int c0 = ct * TW, r0 = rb * RB, r1 = min(h, r0 + RB);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lhi = lane >> 5;

  // weights -> LDS (16 B per thread step)
  for (int e = tid; e < 9 * 64 * (CIP / 8); e += 256) {
    const int row = e / (CIP / 8), part = e % (CIP / 8);
    *reinterpret_cast<uint4*>(Wl + row * CS + part * 8) =
        *reinterpret_cast<const uint4*>(wpk + (size_t)row * CIP + part * 8);
  }
  auto load_row = [&](int rr) {               // image row rr -> ring slot
    uint16_t* dst = Hr + ((rr + 3) % 3) * HW_ * CS;
    for (int e = tid; e < HW_ * (CIP / 8); e += 256) {
      const int cc = e / (CIP / 8), part = e % (CIP / 8);
      const int col = c0 + cc - 1;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (rr >= 0 && rr < h && col >= 0 && col < w)
        v = *reinterpret_cast<const uint4*>(in + (((size_t)b * h + rr) * w + col) * CIP + part * 8);
      *reinterpret_cast<uint4*>(dst + cc * CS + part * 8) = v;
    }
  };
  load_row(r0 - 1);
  load_row(r0);
  for (int r = r0; r < r1; ++r) {
    load_row(r + 1);
    __syncthreads();
    f32x16 acc[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[nt][q] = 0.f;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const uint16_t* hrow = Hr + ((r + dy - 1 + 3) % 3) * HW_ * CS;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int t = dy * 3 + dx;
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          const int ko = kc * 16 + lhi * 8;
          const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                               hrow + (wave * 32 + l32 + dx) * CS + ko));
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            const bf16x8 bb = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                  Wl + (t * 64 + nt * 32 + l32) * CS + ko));
            acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[nt], 0, 0, 0);
          }
        }
      }
    }
    // epilogue
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int co = nt * 32 + l32;
      const float bv = MODE == 0 ? bias[co] : 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int px = wave * 32 + 8 * (q >> 2) + 4 * lhi + (q & 3);
        const int col = c0 + px;
        if (col < w) {
          const size_t o = (((size_t)b * h + r) * w + col) * CH + co;
          float v = acc[nt][q];
          if (MODE == 0) {                    // ReLU that keeps NaN (a NaN weight must show)
            v = v + bv;
            v = (v > 0.f || v != v) ? v : 0.f;
          }
          else v = from_bf16(mask[o]) > 0.f ? v : 0.f;
          out[o] = to_bf16(v);
        }
      }
    }
    __syncthreads();                          // ring slot of row r-1 is reused next
  }
}

// ---------------------------------------------------------------- output layer (VALU)
// out[p] = x[p] + b5 + sum_{tap, c} W5[tap][c] a4[p + tap][c]
__global__ void k_conv_out(const uint16_t* __restrict__ a4, const uint16_t* __restrict__ pk,
                           const float* __restrict__ bias, const float* __restrict__ x, int B,
                           int h, int w, float* __restrict__ out) {
  __shared__ float w5[9 * 64];
  for (int i = threadIdx.x; i < 9 * 64; i += blockDim.x) w5[i] = from_bf16(pk[Pack::w5 + i]);
  __syncthreads();
  const size_t P = (size_t)B * h * w;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int col = (int)(p % w), row = (int)((p / w) % h);
  const size_t b = p / ((size_t)h * w);
  float z = bias[256];
  for (int dy = 0; dy < 3; ++dy) {
    const int rr = row + dy - 1;
    if (rr < 0 || rr >= h) continue;
    for (int dx = 0; dx < 3; ++dx) {
      const int cc = col + dx - 1;
      if (cc < 0 || cc >= w) continue;
      const uint16_t* src = a4 + ((b * h + rr) * w + cc) * CH;
      const float* wt = w5 + (dy * 3 + dx) * 64;
      for (int c8 = 0; c8 < 64; c8 += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(src + c8);
        const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          z = fmaf(wt[c8 + 2 * k], __uint_as_float(u[k] << 16), z);
          z = fmaf(wt[c8 + 2 * k + 1], __uint_as_float(u[k] & 0xffff0000u), z);
        }
      }
    }
  }
  out[p] = x[p] + z;
}

// ---------------------------------------------------------------- loss
constexpr int RED = 256;          // threads of the reduction kernels

// dy[p] = 2 (out - tgt) / n; part[blk] = sum over the block's pixels of (out - tgt)^2
__global__ void __launch_bounds__(RED)
k_loss(const float* __restrict__ out, const float* __restrict__ tgt, size_t P,
       float* __restrict__ dy, float* __restrict__ part) {
  __shared__ float sh[RED];
  float s = 0.f;
  const float sc = 2.0f / (float)P;
  for (size_t p = (size_t)blockIdx.x * RED + threadIdx.x; p < P; p += (size_t)gridDim.x * RED) {
    const float r = out[p] - tgt[p];
    dy[p] = sc * r;
    s = fmaf(r, r, s);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = RED / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[0] = scale * sum of part[0..n) (fixed order)
__global__ void k_sum(const float* __restrict__ part, int n, float scale, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = (float)(s * scale);
  }
}

// ---------------------------------------------------------------- output layer backward
// dz4[q][c] = bf16( (sum_tap W5[tap][c] dy[q - tap]) * (a4[q][c] > 0) )
__global__ void k_out_bwd_data(const float* __restrict__ dy, const uint16_t* __restrict__ pk,
                               const uint16_t* __restrict__ a4, int B, int h, int w,
                               uint16_t* __restrict__ dz) {
  __shared__ float w5[9 * 64];
  for (int i = threadIdx.x; i < 9 * 64; i += blockDim.x) w5[i] = from_bf16(pk[Pack::w5 + i]);
  __syncthreads();
  const size_t P = (size_t)B * h * w;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  const int col = (int)(q % w), row = (int)((q / w) % h);
  const size_t b = q / ((size_t)h * w);
  float g[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dyy = t / 3, dxx = t % 3;
    const int rr = row - dyy + 1, cc = col - dxx + 1;       // q = p + tap  =>  p = q - tap
    g[t] = (rr >= 0 && rr < h && cc >= 0 && cc < w) ? dy[(b * h + rr) * w + cc] : 0.f;
  }
  for (int c = 0; c < 64; ++c) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) s = fmaf(w5[t * 64 + c], g[t], s);
    const float m = from_bf16(a4[q * CH + c]);
    dz[q * CH + c] = to_bf16(m > 0.f ? s : 0.f);
  }
}

// per block: part[blk][t*64 + c] = sum over the block's pixels p of dy[p] a4[p + tap][c];
// part[blk][576] = sum dy[p]
constexpr int OBP = 2048;        // pixels per block
__global__ void __launch_bounds__(RED)
k_out_bwd_weight(const float* __restrict__ dy, const uint16_t* __restrict__ a4, int B, int h,
                 int w, float* __restrict__ part) {
  const size_t P = (size_t)B * h * w;
  const size_t p0 = (size_t)blockIdx.x * OBP;
  const size_t p1 = min(P, p0 + OBP);
  float acc[3] = {0.f, 0.f, 0.f};
  float sdy = 0.f;
  for (size_t p = p0; p < p1; ++p) {
    const float d = dy[p];
    if (threadIdx.x == 0) sdy += d;
    const int col = (int)(p % w), row = (int)((p / w) % h);
    const size_t b = p / ((size_t)h * w);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int e = threadIdx.x + k * RED;
      if (e < 576) {
        const int t = e / 64, c = e % 64;
        const int rr = row + t / 3 - 1, cc = col + t % 3 - 1;
        if (rr >= 0 && rr < h && cc >= 0 && cc < w)
          acc[k] = fmaf(d, from_bf16(a4[((b * h + rr) * w + cc) * CH + c]), acc[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int e = threadIdx.x + k * RED;
    if (e < 576) part[(size_t)blockIdx.x * 577 + e] = acc[k];
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * 577 + 576] = sdy;
}

// ---------------------------------------------------------------- weight gradient (MFMA)
constexpr int WT = 64;           // pixels per weight-gradient tile (row segment)

// part[blk][t][co][ci] (FP32) = sum over the block's tiles of dz[p][co] a[p + tap][ci];
// bpart[blk][co] = sum dz[p][co]
template <int CIP>
__global__ void __launch_bounds__(256)
k_wgrad_mfma(const uint16_t* __restrict__ dz, const uint16_t* __restrict__ a, int B, int h, int w,
             float* __restrict__ part, float* __restrict__ bpart) {
  constexpr int PS = WT + 8;                  // LDS pixel stride (bf16)
  constexpr int NT = CIP >= 32 ? CIP / 32 : 1;   // N tiles of 32 input channels
  constexpr int NTILE = 9 * 2 * NT;           // (tap, M tile, N tile) output tiles
  constexpr int TPW = (NTILE + 3) / 4;        // tiles per wave
  __shared__ __align__(16) uint16_t Zt[64 * PS];
  __shared__ __align__(16) uint16_t At[3 * 3 * (NT * 32) * PS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int nseg = (w + WT - 1) / WT;
  const long long ntiles = (long long)B * h * nseg;

  f32x16 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[i][q] = 0.f;
  float bsum = 0.f;                           // thread co < 64: bias gradient

  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int seg = (int)(tile % nseg);
    const long long br = tile / nseg;
    const int row = (int)(br % h);
    const int b = (int)(br / h);
    const int c0 = seg * WT;
    __syncthreads();                          // previous tile's reads are done
    // Zt[co][px] = dz[row][c0 + px][co]
    for (int e = tid; e < WT * 8; e += 256) {
      const int px = e / 8, part8 = e % 8;
      const int col = c0 + px;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (col < w) v = *reinterpret_cast<const uint4*>(dz + (((size_t)b * h + row) * w + col) * CH + part8 * 8);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Zt[(part8 * 8 + 2 * k) * PS + px] = (uint16_t)(u[k] & 0xffffu);
        Zt[(part8 * 8 + 2 * k + 1) * PS + px] = (uint16_t)(u[k] >> 16);
      }
    }
    // At[dx][dy][ci][px] = a[row + dy - 1][c0 + px + dx - 1][ci] (zero outside)
    for (int e = tid; e < 3 * (WT + 2) * (CIP / 8); e += 256) {
      const int dy = e / ((WT + 2) * (CIP / 8));
      const int rem = e % ((WT + 2) * (CIP / 8));
      const int cc = rem / (CIP / 8), part8 = rem % (CIP / 8);
      const int rr = row + dy - 1, col = c0 + cc - 1;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (rr >= 0 && rr < h && col >= 0 && col < w)
        v = *reinterpret_cast<const uint4*>(a + (((size_t)b * h + rr) * w + col) * CIP + part8 * 8);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int px = cc - dx;               // input column cc serves pixel px for shift dx
        if (px < 0 || px >= WT) continue;
        uint16_t* dst = At + ((dx * 3 + dy) * (NT * 32)) * PS + px;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          dst[(part8 * 8 + 2 * k) * PS] = (uint16_t)(u[k] & 0xffffu);
          dst[(part8 * 8 + 2 * k + 1) * PS] = (uint16_t)(u[k] >> 16);
        }
      }
    }
    if (CIP < NT * 32) {                      // zero the padded channels
      for (int e = tid; e < 9 * (NT * 32 - CIP) * WT; e += 256) {
        const int px = e % WT, r2 = e / WT;
        const int ci = CIP + r2 % (NT * 32 - CIP), td = r2 / (NT * 32 - CIP);
        At[(td * (NT * 32) + ci) * PS + px] = 0;
      }
    }
    __syncthreads();
    if (tid < 64) {
      float s = 0.f;
      for (int px = 0; px < WT; ++px) s += from_bf16(Zt[tid * PS + px]);
      bsum += s;
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int ot = wave + 4 * i;
      if (ot < NTILE) {
        const int t = ot / (2 * NT), mt = (ot / NT) % 2, nt = ot % NT;
        const int dy = t / 3, dx = t % 3;
#pragma unroll
        for (int k0 = 0; k0 < WT; k0 += 16) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                Zt + (mt * 32 + l32) * PS + k0 + lhi * 8));
          const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                At + ((dx * 3 + dy) * (NT * 32) + nt * 32 + l32) * PS + k0 + lhi * 8));
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
        }
      }
    }
  }
  // partials: acc tile (co = mt*32 + i, ci = nt*32 + j)
  float* pb = part + (size_t)blockIdx.x * 9 * 64 * CIP;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int ot = wave + 4 * i;
    if (ot < NTILE) {
      const int t = ot / (2 * NT), mt = (ot / NT) % 2, nt = ot % NT;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int co = mt * 32 + 8 * (q >> 2) + 4 * lhi + (q & 3);
        const int ci = nt * 32 + l32;
        if (ci < CIP) pb[((size_t)t * 64 + co) * CIP + ci] = acc[i][q];
      }
    }
  }
  if (tid < 64) bpart[(size_t)blockIdx.x * 64 + tid] = bsum;
}

// grad (canonical layer layout) = sum over blocks (fixed order) of the partials
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ bpart,
                               int nblk, int CIP, int ci_real, float* __restrict__ gW,
                               float* __restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e over [co][ci_real][9]
  const int n = 64 * ci_real * 9;
  if (e < n) {
    const int co = e / (ci_real * 9), ci = (e / 9) % ci_real, t = e % 9;
    float s = 0.f;
    for (int k = 0; k < nblk; ++k) s += part[((size_t)k * 9 + t) * 64 * CIP + (size_t)co * CIP + ci];
    gW[e] = s;
  }
  if (e < 64) {
    float s = 0.f;
    for (int k = 0; k < nblk; ++k) s += bpart[(size_t)k * 64 + e];
    gb[e] = s;
  }
}

__global__ void k_out_reduce(const float* __restrict__ part, int nblk, float* __restrict__ g) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 577) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += part[(size_t)k * 577 + e];
  if (e < 576) {
    const int t = e / 64, c = e % 64;
    g[poff_w(4) + c * 9 + t] = s;
  } else {
    g[poff_b(4)] = s;
  }
}

// ---------------------------------------------------------------- Adam
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] = th[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------- host side
size_t cnn_packed_bytes() { return Pack::bytes; }
int cnn_param_count() { return NPARAM; }

// workspace layout for (B, h, w)
struct CnnWs {
  size_t in16, act[4], dy, dz[2], wpart, bpart, opart, lpart, grad_tmp, total;
  int nblk_w, nblk_o, nblk_l;
};

static CnnWs cnn_layout(int B, int h, int w, int train) {
  CnnWs L{};
  const size_t P = (size_t)B * h * w;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) / 256 * 256; return o; };
  L.in16 = take(P * 16 * 2);
  const int nact = train ? 4 : 2;
  for (int i = 0; i < 4; ++i) L.act[i] = i < nact ? take(P * CH * 2) : L.act[i - 2];
  L.nblk_w = 256;
  L.nblk_o = (int)((P + OBP - 1) / OBP);
  L.nblk_l = 512;
  if (train) {
    L.dy = take(P * 4);
    L.dz[0] = take(P * CH * 2);
    L.dz[1] = take(P * CH * 2);
    L.wpart = take((size_t)L.nblk_w * 9 * 64 * 64 * 4);
    L.bpart = take((size_t)L.nblk_w * 64 * 4);
    L.opart = take((size_t)L.nblk_o * 577 * 4);
    L.lpart = take((size_t)L.nblk_l * 4);
  }
  L.total = off;
  return L;
}

size_t cnn_workspace_bytes(int B, int h, int w, int train) { return cnn_layout(B, h, w, train).total; }

void cnn_pack(const float* params, void* packed, hipStream_t s) {
  uint16_t* pk = (uint16_t*)packed;
  float* bias = (float*)((char*)packed + Pack::bias_bytes_off);
  hipLaunchKernelGGL(k_pack_weights, dim3((3 * 9 * 64 * 64 + 255) / 256), dim3(256), 0, s, params,
                     pk, bias);
}

static void conv_grid(int B, int h, int w, dim3& g) {
  g = dim3((unsigned)((size_t)B * ((h + RB - 1) / RB) * ((w + TW - 1) / TW)));
}

// forward through layer 4 (activations in ws), then the output layer into out
static void cnn_forward_impl(const void* packed, const float* x, const float* sigma, float* out,
                             int B, int h, int w, char* ws, const CnnWs& L, hipStream_t s) {
  const uint16_t* pk = (const uint16_t*)packed;
  const float* bias = (const float*)((const char*)packed + Pack::bias_bytes_off);
  const size_t P = (size_t)B * h * w;
  uint16_t* in16 = (uint16_t*)(ws + L.in16);
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, x, sigma,
                     h * w, P, in16);
  dim3 g;
  conv_grid(B, h, w, g);
  uint16_t* a[4];
  for (int i = 0; i < 4; ++i) a[i] = (uint16_t*)(ws + L.act[i]);
  hipLaunchKernelGGL((k_conv_mfma<16, 0>), g, dim3(256), 0, s, in16, pk + Pack::wf1, bias,
                     (const uint16_t*)nullptr, B, h, w, a[0]);
  for (int l = 1; l < 4; ++l)
    hipLaunchKernelGGL((k_conv_mfma<64, 0>), g, dim3(256), 0, s, a[l - 1],
                       pk + Pack::wf2 + (size_t)(l - 1) * 9 * 64 * 64, bias + 64 * l,
                       (const uint16_t*)nullptr, B, h, w, a[l]);
  hipLaunchKernelGGL(k_conv_out, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, a[3], pk,
                     bias, x, B, h, w, out);
}

void cnn_forward(const void* packed, const float* x, const float* sigma, float* out, int B, int h,
                 int w, void* ws, hipStream_t s) {
  const CnnWs L = cnn_layout(B, h, w, 0);
  cnn_forward_impl(packed, x, sigma, out, B, h, w, (char*)ws, L, s);
}

// loss (device scalar) and the gradient of all parameters (flat, canonical)
void cnn_loss_grad(const void* packed, const float* x, const float* sigma, const float* tgt,
                   int B, int h, int w, float* loss, float* grad, float* out_tmp, void* wsv,
                   hipStream_t s) {
  char* ws = (char*)wsv;
  const CnnWs L = cnn_layout(B, h, w, 1);
  const uint16_t* pk = (const uint16_t*)packed;
  const size_t P = (size_t)B * h * w;
  cnn_forward_impl(packed, x, sigma, out_tmp, B, h, w, ws, L, s);
  float* dy = (float*)(ws + L.dy);
  float* lpart = (float*)(ws + L.lpart);
  hipLaunchKernelGGL(k_loss, dim3(L.nblk_l), dim3(RED), 0, s, out_tmp, tgt, P, dy, lpart);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, lpart, L.nblk_l, 1.0f / (float)P, loss);
  uint16_t* a[4];
  for (int i = 0; i < 4; ++i) a[i] = (uint16_t*)(ws + L.act[i]);
  uint16_t* in16 = (uint16_t*)(ws + L.in16);
  uint16_t* dz[2] = {(uint16_t*)(ws + L.dz[0]), (uint16_t*)(ws + L.dz[1])};
  // output layer
  float* opart = (float*)(ws + L.opart);
  hipLaunchKernelGGL(k_out_bwd_weight, dim3(L.nblk_o), dim3(RED), 0, s, dy, a[3], B, h, w, opart);
  hipLaunchKernelGGL(k_out_reduce, dim3(3), dim3(256), 0, s, opart, L.nblk_o, grad);
  hipLaunchKernelGGL(k_out_bwd_data, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, dy, pk,
                     a[3], B, h, w, dz[0]);
  // hidden layers 4..1: dz[cur] = gradient of layer l's pre-activation
  float* wpart = (float*)(ws + L.wpart);
  float* bpart = (float*)(ws + L.bpart);
  dim3 g;
  conv_grid(B, h, w, g);
  int cur = 0;
  for (int l = 3; l >= 0; --l) {
    const uint16_t* ain = l == 0 ? in16 : a[l - 1];
    if (l == 0)
      hipLaunchKernelGGL(k_wgrad_mfma<16>, dim3(L.nblk_w), dim3(256), 0, s, dz[cur], ain, B, h, w,
                         wpart, bpart);
    else
      hipLaunchKernelGGL(k_wgrad_mfma<64>, dim3(L.nblk_w), dim3(256), 0, s, dz[cur], ain, B, h, w,
                         wpart, bpart);
    const int cir = l == 0 ? 2 : 64;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((64 * cir * 9 + 255) / 256), dim3(256), 0, s, wpart,
                       bpart, L.nblk_w, l == 0 ? 16 : 64, cir, grad + poff_w(l), grad + poff_b(l));
    if (l > 0) {
      hipLaunchKernelGGL((k_conv_mfma<64, 1>), g, dim3(256), 0, s, dz[cur],
                         pk + Pack::wd2 + (size_t)(l - 1) * 9 * 64 * 64, (const float*)nullptr,
                         a[l - 1], B, h, w, dz[cur ^ 1]);
      cur ^= 1;
    }
  }
}

void cnn_adam(float* params, float* m, float* v, const float* grad, int step, float lr,
              void* packed, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, step)));
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, params, m, v, grad,
                     NPARAM, lr, (float)b1, (float)b2, c1, c2, 1e-8f);
  cnn_pack(params, packed, s);
}
