// Key (exemplar) patch detection: corner points instead of a uniform grid
// (Method section, Fig. 1a).  Reading: an integer Harris detector on a u8
// detection image.  Only the quantiser uses floating point (IEEE FP32 with no
// contraction: the file is built with -ffp-contract=off); everything after it
// is exact integer arithmetic, so the keys are reproducible bit for bit.
#include "common.h"
#include "internal.h"

namespace {

constexpr int TPB = 256;
inline int nblk(size_t n) { return (int)((n + TPB - 1) / TPB); }

// q = floor((sum_c clamp(rint(255 x_c), 0, 255) + C/2) / C)
__global__ void k_quant_real(const float* __restrict__ x, int C, int HW, uint8_t* __restrict__ q) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  int s = 0;
  for (int c = 0; c < C; ++c) {
    float v = rintf(255.0f * x[(size_t)c * HW + p]);
    v = fminf(fmaxf(v, 0.0f), 255.0f);
    s += (int)v;
  }
  q[p] = (uint8_t)((s + C / 2) / C);
}

constexpr int MAXB = 256;         // blocks of the magnitude maximum (one partial each)
static_assert(MAXB <= TPB, "one partial per thread of a block");

// block maximum of a TPB-thread block (all threads get it)
__device__ __forceinline__ uint32_t block_max_u32(uint32_t b, uint32_t* red) {
  for (int o = 32; o > 0; o >>= 1) b = max(b, (uint32_t)__shfl_xor((int)b, o, 64));
  if (lane_id() == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  uint32_t m = red[0];
  for (int i = 1; i < TPB / 64; ++i) m = max(m, red[i]);
  return m;
}

// largest squared magnitude (non-negative floats order like their bit
// patterns): one partial maximum per block, over a grid-stride range
__global__ void k_mag2_max(const float* __restrict__ xp, int HW, uint32_t* __restrict__ part) {
  __shared__ uint32_t red[TPB / 64];
  uint32_t b = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += gridDim.x * blockDim.x) {
    const float re = xp[p], im = xp[HW + p];
    b = max(b, __float_as_uint(re * re + im * im));
  }
  const uint32_t m = block_max_u32(b, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// q = clamp(rint(255 * (m * (1/max m))), 0, 255); all zero if max m == 0.
// Every block folds the nb <= TPB partial maxima itself.
__global__ void k_quant_cplx(const float* __restrict__ xp, int HW, const uint32_t* __restrict__ part,
                             int nb, uint8_t* __restrict__ q) {
  __shared__ uint32_t red[TPB / 64];
  const uint32_t mx = block_max_u32(threadIdx.x < nb ? part[threadIdx.x] : 0u, red);
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  float m_max = __uint_as_float(mx);
  if (!(m_max > 0.0f)) {
    q[p] = 0;
    return;
  }
  float s = __fdiv_rn(1.0f, m_max);
  float re = xp[p], im = xp[HW + p];
  float m = re * re + im * im;
  float v = rintf(255.0f * (m * s));
  v = fminf(fmaxf(v, 0.0f), 255.0f);
  q[p] = (uint8_t)v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Sobel with replicate borders; products gx^2, gy^2, gx*gy.
__global__ void k_sobel(const uint8_t* __restrict__ q, int H, int W, int* __restrict__ gxx,
                        int* __restrict__ gyy, int* __restrict__ gxy) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  int rm = clampi(r - 1, 0, H - 1), rp = clampi(r + 1, 0, H - 1);
  int cm = clampi(c - 1, 0, W - 1), cp = clampi(c + 1, 0, W - 1);
  auto Q = [&](int rr, int cc) { return (int)q[rr * W + cc]; };
  int gx = (Q(rm, cp) + 2 * Q(r, cp) + Q(rp, cp)) - (Q(rm, cm) + 2 * Q(r, cm) + Q(rp, cm));
  int gy = (Q(rp, cm) + 2 * Q(rp, c) + Q(rp, cp)) - (Q(rm, cm) + 2 * Q(rm, c) + Q(rm, cp));
  gxx[p] = gx * gx;
  gyy[p] = gy * gy;
  gxy[p] = gx * gy;
}

// 5x5 binomial structure tensor (replicate borders) and R25 = 25 det - tr^2.
__global__ void k_harris(const int* __restrict__ gxx, const int* __restrict__ gyy,
                         const int* __restrict__ gxy, int H, int W, long long* __restrict__ r25) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  int r = p / W, c = p - r * W;
  const int w5[5] = {1, 4, 6, 4, 1};
  int sxx = 0, syy = 0, sxy = 0;
  for (int a = 0; a < 5; ++a) {
    int rr = clampi(r + a - 2, 0, H - 1);
    for (int b = 0; b < 5; ++b) {
      int cc = clampi(c + b - 2, 0, W - 1);
      int w = w5[a] * w5[b];
      int i = rr * W + cc;
      sxx += w * gxx[i];
      syy += w * gyy[i];
      sxy += w * gxy[i];
    }
  }
  long long A = sxx, B = syy, X = sxy;
  r25[p] = 25 * (A * B - X * X) - (A + B) * (A + B);
}

// 3x3 non-maximum suppression under (R25 desc, pixel index asc), neighbours
// inside the image; flag per top-left grid position of a domain centre.
__global__ void k_nms(const long long* __restrict__ R, int H, int W, int P, uint8_t* __restrict__ flag) {
  const int o = (P - 1) / 2;
  const int Hc = H - P + 1, Wc = W - P + 1;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Hc * Wc) return;
  int gr = t / Wc, gc = t - gr * Wc;
  int r = gr + o, c = gc + o;
  long long v = R[(size_t)r * W + c];
  bool keep = v > 0;
  for (int dr = -1; dr <= 1; ++dr)
    for (int dc = -1; dc <= 1; ++dc) {
      if (dr == 0 && dc == 0) continue;
      int rr = r + dr, cc = c + dc;
      if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
      long long nb = R[(size_t)rr * W + cc];
      bool earlier = dr < 0 || (dr == 0 && dc < 0);
      keep = keep && (earlier ? (v > nb) : (v >= nb));
    }
  flag[t] = keep ? 1 : 0;
}

constexpr int SEL_T = 1024;
constexpr int RUN = 64;           // consecutive positions per thread per scan step

// number of non-zero bytes of a word whose bytes are 0 or 1
__device__ __forceinline__ int ones4(uint32_t w) { return (int)((w * 0x01010101u) >> 24); }

// Ordered compaction of the positions t < n with flag[t] != 0 (flags are 0
// or 1) into list[]; optionally records their scores.  Each thread takes 64
// consecutive flags, read as four 16-byte words.  Returns the count
// (block-uniform).
__device__ int ordered_compact(const uint8_t* __restrict__ flag, int n, int32_t* __restrict__ list,
                               int cap, long long* __restrict__ vals,
                               const long long* __restrict__ R, int W, int Wc, int o,
                               int* scan_sh) {
  int S = 0;
  for (int base = 0; base < n; base += SEL_T * RUN) {
    const int t0 = base + threadIdx.x * RUN;
    uint32_t w[RUN / 4];
    if (t0 + RUN <= n) {
#pragma unroll
      for (int q = 0; q < RUN / 16; ++q) {
        const uint4 v = *reinterpret_cast<const uint4*>(flag + t0 + 16 * q);
        w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < RUN / 4; ++q) {
        uint32_t x = 0u;
        for (int b = 0; b < 4; ++b) {
          const int t = t0 + 4 * q + b;
          if (t < n) x |= (uint32_t)flag[t] << (8 * b);
        }
        w[q] = x;
      }
    }
    int c = 0;
#pragma unroll
    for (int q = 0; q < RUN / 4; ++q) c += ones4(w[q]);
    int tot;
    const int pre = block_excl_scan(c, scan_sh, &tot);
    int wr = S + pre;
    if (c > 0)
      for (int q = 0; q < RUN / 4; ++q)
        for (int b = 0; b < 4; ++b)
          if ((w[q] >> (8 * b)) & 0xffu) {
            const int t = t0 + 4 * q + b;
            if (wr < cap) {
              list[wr] = t;
              if (vals) {
                const int gr = t / Wc, gc = t - gr * Wc;
                vals[wr] = R[(size_t)(gr + o) * W + gc + o];
              }
            }
            ++wr;
          }
    S += tot;
  }
  return S;
}

constexpr int SEL_R = 4;          // survivor scores held in registers per thread

// Single workgroup: ordered selection of the best N survivors by
// (R25 desc, position asc), uniform raster fill, ascending key list.
// `flag` holds the NMS survivors on entry (and, when there are fewer than N,
// the survivors plus the raster fill on exit).
__global__ void __launch_bounds__(SEL_T) k_select(uint8_t* __restrict__ flag,
                                                  const long long* __restrict__ R, int H, int W,
                                                  int P, int N, int32_t* __restrict__ slist,
                                                  long long* __restrict__ sval,
                                                  int32_t* __restrict__ keys, DevStats* st) {
  __shared__ int scan_sh[SEL_T / 64 + 1];
  __shared__ int hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_remaining, s_top;
  __shared__ unsigned long long s_mn[SEL_T / 64], s_mx[SEL_T / 64];
  const int o = (P - 1) / 2;
  const int Hc = H - P + 1, Wc = W - P + 1;
  const int Ncand = Hc * Wc;
  const int tid = threadIdx.x;
  // A. ordered list of survivors, then their scores: survivor i = tid +
  //    k SEL_T is read by this thread (all reads in flight together) and kept
  //    in registers when S <= SEL_T SEL_R, else written to sval
  const int S = ordered_compact(flag, Ncand, slist, Ncand, nullptr, R, W, Wc, o, scan_sh);
  __syncthreads();
  const bool in_reg = S <= SEL_T * SEL_R;
  unsigned long long rv[SEL_R];
  if (S > N) {
    for (int base = 0; base < S; base += SEL_T * SEL_R) {
      int pos[SEL_R];
#pragma unroll
      for (int k = 0; k < SEL_R; ++k) {
        const int i = base + k * SEL_T + tid;
        pos[k] = i < S ? slist[i] : -1;
      }
#pragma unroll
      for (int k = 0; k < SEL_R; ++k) {
        const int t = pos[k] < 0 ? 0 : pos[k];
        const int gr = t / Wc, gc = t - gr * Wc;
        rv[k] = pos[k] < 0 ? 0ull : (unsigned long long)R[(size_t)(gr + o) * W + gc + o];
      }
      if (!in_reg)
#pragma unroll
        for (int k = 0; k < SEL_R; ++k) {
          const int i = base + k * SEL_T + tid;
          if (i < S) sval[i] = (long long)rv[k];
        }
    }
    if (!in_reg) __syncthreads();
  }
  // visits every survivor score of this thread (i ascending per thread)
  auto each = [&](auto&& f) {
    if (in_reg) {
#pragma unroll
      for (int k = 0; k < SEL_R; ++k) {
        const int i = k * SEL_T + tid;
        if (i < S) f(rv[k]);
      }
    } else {
      for (int i = tid; i < S; i += SEL_T) f((unsigned long long)sval[i]);
    }
  };
  // B. radix select of the N-th largest score v* (scores are positive): the
  //    bits above the highest bit in which the survivors' scores differ are
  //    common, the rest is resolved in digits of up to 8 bits, most
  //    significant first; need_eq = how many survivors equal to v* are taken
  if (S > N) {
    unsigned long long mn = ~0ull, mx = 0ull;
    each([&](unsigned long long v) {
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
    });
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      const unsigned long long a = __shfl_xor(mn, o2, 64), b = __shfl_xor(mx, o2, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    if ((tid & 63) == 0) {
      s_mn[tid >> 6] = mn;
      s_mx[tid >> 6] = mx;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long a = s_mn[0], b = s_mx[0];
      for (int i = 1; i < SEL_T / 64; ++i) {
        a = s_mn[i] < a ? s_mn[i] : a;
        b = s_mx[i] > b ? s_mx[i] : b;
      }
      const int top = a == b ? -1 : 63 - __builtin_clzll(a ^ b);
      s_prefix = top < 0 ? a : (top == 63 ? 0ull : a & ~((2ull << top) - 1ull));
      s_remaining = N;
      s_top = top;
    }
    __syncthreads();
    for (int top = s_top; top >= 0;) {
      const int shift = top >= 7 ? top - 7 : 0;
      const unsigned long long hmask = top == 63 ? 0ull : ~((2ull << top) - 1ull);
      if (tid < 256) hist[tid] = 0;
      __syncthreads();
      const unsigned long long prefix = s_prefix;
      each([&](unsigned long long v) {
        if ((v & hmask) == (prefix & hmask)) atomicAdd(&hist[(v >> shift) & 255u], 1);
      });
      __syncthreads();
      if (tid < 64) {
        // wave 0: lane l owns bins 255-4l .. 252-4l (descending), so a prefix
        // sum over lanes counts the scores above each bin
        const int rem = s_remaining;
        const int b0 = 255 - 4 * tid;
        const int c0 = hist[b0], c1 = hist[b0 - 1], c2 = hist[b0 - 2], c3 = hist[b0 - 3];
        const int tot = c0 + c1 + c2 + c3;
        const int incl = wave_incl_scan(tot);
        const int excl = incl - tot;
        if (excl < rem && rem <= incl) {
          int digit, above;
          const int r = rem - excl;
          if (r <= c0) { digit = b0; above = excl; }
          else if (r <= c0 + c1) { digit = b0 - 1; above = excl + c0; }
          else if (r <= c0 + c1 + c2) { digit = b0 - 2; above = excl + c0 + c1; }
          else { digit = b0 - 3; above = excl + c0 + c1 + c2; }
          s_prefix = prefix | ((unsigned long long)digit << shift);
          s_remaining = rem - above;
        }
      }
      __syncthreads();
      top = shift - 1;
    }
    const unsigned long long vstar = s_prefix;
    const int need_eq = s_remaining;
    // C. keep the survivors above v* and the first need_eq equal to it (the
    //    lowest positions); they are the key list, in ascending position
    int eq_seen = 0, sel_seen = 0;
    for (int k = 0; k * SEL_T < S; ++k) {
      const int i = k * SEL_T + tid;
      unsigned long long v = 0ull;
      if (in_reg) {
#pragma unroll
        for (int q = 0; q < SEL_R; ++q)
          if (q == k) v = rv[q];
      } else if (i < S) {
        v = (unsigned long long)sval[i];
      }
      const int is_eq = (i < S && v == vstar) ? 1 : 0;
      int tot;
      const int pre = block_excl_scan(is_eq, scan_sh, &tot);
      const int sel = (i < S && (v > vstar || (is_eq && eq_seen + pre < need_eq))) ? 1 : 0;
      int tsel;
      const int spre = block_excl_scan(sel, scan_sh, &tsel);
      if (sel) keys[sel_seen + spre] = slist[i];
      eq_seen += tot;
      sel_seen += tsel;
    }
    if (tid == 0 && st) st->keys_selected = N;
    return;
  }
  if (tid == 0 && st) st->keys_selected = S;
  if (S == N) {
    for (int i = tid; i < S; i += SEL_T) keys[i] = slist[i];
    return;
  }
  // D. uniform raster fill (step s, then step 1) of positions not chosen
  int need = N - S;
  {
    int s = 1;
    while ((long long)s * s * N < (long long)Ncand) ++s;
    for (int pass = 0; pass < 2 && need > 0; ++pass) {
      const int step = pass == 0 ? s : 1;
      const int nr = (Hc + step - 1) / step, nc = (Wc + step - 1) / step;
      const int tot_pos = nr * nc;
      for (int base = 0; base < tot_pos && need > 0; base += SEL_T) {
        const int i = base + tid;
        int t = -1;
        if (i < tot_pos) t = (i / nc) * step * Wc + (i % nc) * step;
        const int cand = (t >= 0 && !flag[t]) ? 1 : 0;
        int tot;
        const int pre = block_excl_scan(cand, scan_sh, &tot);
        if (cand && pre < need) flag[t] = 1;
        need -= tot < need ? tot : need;
      }
    }
  }
  __syncthreads();
  // E. ascending key list (exactly N chosen positions)
  ordered_compact(flag, Ncand, keys, N, nullptr, R, W, Wc, o, scan_sh);
}

}  // namespace

// ---------------------------------------------------------------- edge maps
// The paper's matching score (eq. 6-8) correlates binary edge maps.  Reading:
// per real channel, the quantised channel image q_c = clamp(rint(255 x_c))
// (complex data: the detector's single quantised squared-magnitude image),
// the detector's integer Sobel (replicate borders), and rising and falling
// edges thresholded at th = ceil(max |g| / 10) over the whole stack:
// E[4c + 0] = [gx > th], E[4c + 1] = [-gx > th], E[4c + 2] = [gy > th],
// E[4c + 3] = [-gy > th] (gx along columns, gy along rows).

// per-channel quantisation q[p] = clamp(rint(255 x[p]), 0, 255) of n values
__global__ void k_quant_chan(const float* __restrict__ x, size_t n, uint8_t* __restrict__ q) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float v = rintf(255.0f * x[p]);
  q[p] = (uint8_t)fminf(fmaxf(v, 0.0f), 255.0f);
}

// Sobel of every channel image of q [Ce][H][W]: gx, gy (|g| <= 1020) and the
// largest |g| of the stack (one atomic per block; *gmax cleared before)
__global__ void k_edge_grad(const uint8_t* __restrict__ q, int Ce, int H, int W,
                            int16_t* __restrict__ gxo, int16_t* __restrict__ gyo,
                            uint32_t* __restrict__ gmax) {
  __shared__ uint32_t red[TPB / 64];
  const size_t HW = (size_t)H * W;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t m = 0;
  if (p < HW * Ce) {
    const int ch = (int)(p / HW);
    const int pix = (int)(p - (size_t)ch * HW);
    const int r = pix / W, c = pix - r * W;
    const int rm = clampi(r - 1, 0, H - 1), rp = clampi(r + 1, 0, H - 1);
    const int cm = clampi(c - 1, 0, W - 1), cp = clampi(c + 1, 0, W - 1);
    const uint8_t* qc = q + (size_t)ch * HW;
    auto Q = [&](int rr, int cc) { return (int)qc[rr * W + cc]; };
    const int gx = (Q(rm, cp) + 2 * Q(r, cp) + Q(rp, cp)) - (Q(rm, cm) + 2 * Q(r, cm) + Q(rp, cm));
    const int gy = (Q(rp, cm) + 2 * Q(rp, c) + Q(rp, cp)) - (Q(rm, cm) + 2 * Q(rm, c) + Q(rm, cp));
    gxo[p] = (int16_t)gx;
    gyo[p] = (int16_t)gy;
    m = (uint32_t)max(abs(gx), abs(gy));
  }
  m = block_max_u32(m, red);
  if (threadIdx.x == 0 && m > 0) atomicMax(gmax, m);
}

__global__ void k_edge_maps(const int16_t* __restrict__ gx, const int16_t* __restrict__ gy,
                            int Ce, size_t HW, const uint32_t* __restrict__ gmax,
                            float* __restrict__ E) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW * Ce) return;
  const int th = (int)((gmax[0] + 9u) / 10u);
  const size_t ch = p / HW, pix = p - ch * HW;
  const int x = gx[p], y = gy[p];
  float* e = E + 4 * ch * HW + pix;
  e[0] = x > th ? 1.f : 0.f;
  e[HW] = -x > th ? 1.f : 0.f;
  e[2 * HW] = y > th ? 1.f : 0.f;
  e[3 * HW] = -y > th ? 1.f : 0.f;
}

// keys[i] = (step (i / nc)) Wc + step (i % nc), nc = ceil(Wc / step): the
// uniform exemplar grid, ascending
__global__ void k_uniform_keys(int32_t* __restrict__ keys, int n, int Wc, int step, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = i / nc, b = i - a * nc;
  keys[i] = a * step * Wc + b * step;
}

void launch_edges(const glr_plan* pl, const float* xp, char* ws, float* E, hipStream_t s) {
  const int H = pl->H, W = pl->W;
  const size_t HW = (size_t)H * W;
  const int Ce = pl->is_complex ? 1 : pl->Cp;
  uint8_t* q = (uint8_t*)(ws + pl->ws.eq);
  int16_t* gx = (int16_t*)(ws + pl->ws.egx);
  int16_t* gy = gx + (size_t)Ce * HW;
  uint32_t* gmax = (uint32_t*)(ws + pl->ws.emax);
  launch_fill_u32(gmax, 0u, 1, s);
  if (pl->is_complex) {
    uint32_t* part = (uint32_t*)(ws + pl->ws.red);
    const int nb = std::min(nblk(HW), MAXB);
    hipLaunchKernelGGL(k_mag2_max, dim3(nb), dim3(TPB), 0, s, xp, (int)HW, part);
    hipLaunchKernelGGL(k_quant_cplx, dim3(nblk(HW)), dim3(TPB), 0, s, xp, (int)HW, part, nb, q);
  } else {
    hipLaunchKernelGGL(k_quant_chan, dim3(nblk(HW * Ce)), dim3(TPB), 0, s, xp, HW * Ce, q);
  }
  hipLaunchKernelGGL(k_edge_grad, dim3(nblk(HW * Ce)), dim3(TPB), 0, s, q, Ce, H, W, gx, gy, gmax);
  hipLaunchKernelGGL(k_edge_maps, dim3(nblk(HW * Ce)), dim3(TPB), 0, s, gx, gy, Ce, HW, gmax, E);
}

void launch_uniform_keys(const glr_plan* pl, int32_t* keys, int step, hipStream_t s) {
  const int nr = (pl->Hc + step - 1) / step, nc = (pl->Wc + step - 1) / step;
  const int n = nr * nc;
  hipLaunchKernelGGL(k_uniform_keys, dim3((n + 255) / 256), dim3(256), 0, s, keys, n, pl->Wc,
                     step, nc);
}

void launch_detect(const glr_plan* pl, const float* xp, char* ws, int32_t* keys, int n_sel,
                   hipStream_t s) {
  const int H = pl->H, W = pl->W, HW = H * W;
  uint8_t* q = (uint8_t*)(ws + pl->ws.q);
  int* gxx = (int*)(ws + pl->ws.gxx);
  int* gyy = (int*)(ws + pl->ws.gyy);
  int* gxy = (int*)(ws + pl->ws.gxy);
  long long* r25 = (long long*)(ws + pl->ws.r25);
  uint8_t* flag = (uint8_t*)(ws + pl->ws.cflag);
  int32_t* slist = (int32_t*)(ws + pl->ws.slist);
  long long* sval = (long long*)(ws + pl->ws.sval);
  DevStats* st = (DevStats*)(ws + pl->ws.stats);
  if (pl->is_complex) {
    uint32_t* part = (uint32_t*)(ws + pl->ws.red);      // [MAXB]
    const int nb = std::min(nblk(HW), MAXB);
    hipLaunchKernelGGL(k_mag2_max, dim3(nb), dim3(TPB), 0, s, xp, HW, part);
    hipLaunchKernelGGL(k_quant_cplx, dim3(nblk(HW)), dim3(TPB), 0, s, xp, HW, part, nb, q);
  } else {
    hipLaunchKernelGGL(k_quant_real, dim3(nblk(HW)), dim3(TPB), 0, s, xp, pl->Cp, HW, q);
  }
  hipLaunchKernelGGL(k_sobel, dim3(nblk(HW)), dim3(TPB), 0, s, q, H, W, gxx, gyy, gxy);
  hipLaunchKernelGGL(k_harris, dim3(nblk(HW)), dim3(TPB), 0, s, gxx, gyy, gxy, H, W, r25);
  hipLaunchKernelGGL(k_nms, dim3(nblk((size_t)pl->Ncand)), dim3(TPB), 0, s, r25, H, W, pl->P, flag);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(SEL_T), 0, s, flag, r25, H, W, pl->P, n_sel, slist,
                     sval, keys, st);
}
