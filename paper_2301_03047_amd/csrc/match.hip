// Global patch matching (eq. 8 candidate grid; Im2Col + matrix product as the
// acceleration of the paper's matching convolution): every key patch against
// every stride-1 image patch, as one contraction on MFMA.
//
// Both forms work on mean-centred patches: with a = k - mu_k 1 and
// pbar = p - mu_p 1 (FP32) and dmu = mu_k - mu_p, the exact identity
//     ||k - p||^2 = ||a||^2 + ||pbar||^2 - 2 <a, pbar> + D dmu^2
//                   + 2 dmu (sum a - sum pbar)
// gives the distance from one centred dot product; its rounding error scales
// with the centred norms (||a|| ||pbar||) instead of the raw ones, which is
// what keeps the certified margin of the top-K pass small on smooth images.
//   FP32 form: <a, pbar> on v_mfma_f32_32x32x2f32;
//   BF16 form: <bf16(a), bf16(pbar)> on v_mfma_f32_32x32x16_bf16 (FP32 sums).
// The candidate operand is never materialised: a 128-candidate tile lies on
// one row of the top-left grid, so for each (channel, dy) the tile's patch
// rows are one image row segment of 128 + P - 1 values staged in LDS.
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- key matrix
// A[g][d] = x[c][r_g + dy][c_g + dx], d = (c*P + dy)*P + dx.  One wave per key.
// Also sets the top-K scan's per-key bounds tsh[0..n_tsh) to +inf, so every
// match call starts from them whatever an earlier call left.
__global__ void k_gather_keys(const float* __restrict__ xp, int H, int W, int P, int D,
                              const int32_t* __restrict__ keys, int N, float* __restrict__ A,
                              uint32_t* __restrict__ tsh, int n_tsh) {
  const int g = blockIdx.x;
  if (g >= N) return;
  if (threadIdx.x == 0 && g < n_tsh) tsh[g] = 0xffffffffu;
  const int Wc = W - P + 1;
  const int t = keys[g];
  const int gr = t / Wc, gc = t - gr * Wc;
  for (int d = threadIdx.x; d < D; d += 64) {
    int c = d / (P * P);
    int rem = d - c * P * P;
    int dy = rem / P, dx = rem - dy * P;
    A[(size_t)g * D + d] = xp[((size_t)c * H + gr + dy) * W + gc + dx];
  }
}

// ---------------------------------------------------------------- FP32 MFMA matcher
constexpr int BM = 128;   // keys per block
constexpr int BN = 128;   // candidates per block (one grid-row segment)
constexpr int CB = 32;    // channels per epilogue pass

// d~ from the centred dot product S (BF16 form, one mean per patch)
__device__ __forceinline__ float centred_dist(float4 km, float4 cm, float S, int D) {
  // km = (||a||^2, mu_k, sum a, ||a||), cm = (mu_p, ||pbar||^2, ||pbar||, sum pbar)
  const float dmu = km.y - cm.x;
  const float base = (km.x + cm.y) - 2.0f * S;
  return (base + ((float)D * dmu) * dmu) + 2.0f * dmu * (km.z - cm.w);
}

// FP32 form: every channel block of n = P^2 elements is centred on its own
// mean.  With a~ = fl(k - mu_kc), p~ = fl(p - mu_pc) per channel c (means
// correctly rounded from FP64 sums) and dmu_c = mu_kc - mu_pc,
//   ||k - p||^2 = ||a~||^2 + ||p~||^2 - 2 <a~, p~> + n sum_c dmu_c^2
// up to the residues of the centring (the channel sums of a~ and p~ and the
// subtraction roundings), which the error bound of the top-K pass covers.
// The kernel adds sum_c (P mu_kc - P mu_pc)^2 with P mu rounded to FP32.
// Removing each channel's own level (a band's brightness, a frame's
// exposure) keeps ||a~||, ||p~||, and with them the rounding error, at the
// scale of the texture.
//
// Key data: Ac[g] = a~ (rows g or kmap[g0+g]), kn[g] = (||a~||^2, h_k, 0,
// ||a~||) with h the norm of the channels' mean |values| (a bound term),
// kc[g][c] = fl(P mu_kc).  Candidate data: pn[j] = ||p~_j||^2, pc[c][j] =
// (mu_pc, fl(P mu_pc)) (channel-major, so lanes of consecutive candidates
// read consecutive entries).
template <int P2>
__global__ void __launch_bounds__(256, 3)
k_match_f32(const float* __restrict__ xp, int H, int W, int P, int Cp,
            const float* __restrict__ Ac, int D, const float4* __restrict__ kn,
            const float* __restrict__ kc, const float* __restrict__ pn,
            const float2* __restrict__ pc, size_t ncand, const int32_t* __restrict__ kmap,
            int g0, int nk, float* __restrict__ dist, size_t ldd) {
  // The K dimension runs in stages of GM patch rows of one channel (GM fixed
  // by P2: the most rows whose staging registers fit three waves per SIMD
  // without spills): one barrier per stage, and the next stage's loads are
  // in flight during a stage's MFMAs.
  constexpr int GM = (P2 == 12 || P2 == 14) ? 1 : (P2 == 6 ? 3 : (P2 >= 10 ? 2 : (P2 <= 2 ? 2 : 4)));
  constexpr int SEG = BN + P2;
  constexpr int AST = GM * P2 + 1;   // odd LDS stride for the key slab
  constexpr int MAIN = 2 * GM * SEG + 2 * BM * AST;
  constexpr int EPI = CB * BM + CB * BN;
  __shared__ __align__(16) float lds[MAIN > EPI ? MAIN : EPI];
  float* const seg0 = lds;                    // [2][GM][SEG] image rows
  float* const As0 = lds + 2 * GM * SEG;      // [2][BM][AST] key slab
  float* const skc = lds;                     // epilogue: [channel of the pass][key]
  float* const spc = lds + CB * BM;           // epilogue: [channel of the pass][candidate]
  __shared__ int krow[BM];
  __shared__ float skn[BM];

  const int Hc = H - P + 1, Wc = W - P + 1;
  const int ntc = (Wc + BN - 1) / BN;
  int b = blockIdx.x;
  const int ct = b % ntc;
  b /= ntc;
  const int r = b % Hc;
  const int kt = b / Hc;
  const int c0 = ct * BN;
  const int kbase = kt * BM;                 // chunk-local key index of the tile

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int SPC = (P + GM - 1) / GM;         // stages per channel
  const int S = Cp * SPC;
  auto key_row = [&](int m) {
    const int g = kbase + m;
    return g < nk ? (kmap ? kmap[g0 + g] : g0 + g) : -1;
  };
  // the epilogue's key and candidate terms are loaded now and staged after
  // the main loop (for up to four channels), so their latency overlaps it
  float knr = 0.f;
  if (tid < BM) {
    const int gg = key_row(tid);
    krow[tid] = gg;
    knr = gg >= 0 ? kn[gg].x : 0.f;
  }
  const bool pre = Cp <= 4;
  float pkc[2] = {0.f, 0.f}, ppc[2] = {0.f, 0.f};
  if (pre) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * 256;
      if (e < Cp * BM) {
        const int c = e / BM, m = e - c * BM;
        const int gg = key_row(m);
        pkc[k] = gg >= 0 ? kc[(size_t)gg * Cp + c] : 0.f;
      }
      if (e < Cp * BN) {
        const int c = e / BN, j = e - c * BN;
        ppc[k] = c0 + j < Wc ? pc[(size_t)c * ncand + (size_t)r * Wc + c0 + j].y : 0.f;
      }
    }
  }
  __syncthreads();

  const int l32 = lane & 31, lhi = lane >> 5;
  const int colA = c0 + wn * 64 + l32, colB = colA + 32;
  const size_t tA = (size_t)r * Wc + colA, tB = tA + 32;
  const float pnA = colA < Wc ? pn[tA] : 0.f, pnB = colB < Wc ? pn[tB] : 0.f;

  // register staging of the next stage
  float rseg[GM];
  constexpr int APT = (BM * GM * P2 + 255) / 256;
  float ra[APT];
  float nb0 = 0.f, nb1 = 0.f;

  auto load_stage = [&](int st) {
    const int ch = st / SPC, dy0 = (st - ch * SPC) * GM;
#pragma unroll
    for (int q = 0; q < GM; ++q) {
      rseg[q] = 0.f;
      if (tid < SEG && dy0 + q < P) {
        const int cc = c0 + tid;
        if (cc < W) rseg[q] = xp[((size_t)ch * H + r + dy0 + q) * W + cc];
      }
    }
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      const int e = tid + u * 256;
      float v = 0.f;
      if (e < BM * GM * P2) {
        const int m = e / (GM * P2), rem = e - m * (GM * P2);
        const int q = rem / P2, dx = rem - q * P2;
        const int gg = krow[m];
        if (dx < P && dy0 + q < P && gg >= 0)
          v = Ac[(size_t)gg * D + (size_t)(ch * P + dy0 + q) * P + dx];
      }
      ra[u] = v;
    }
    if (dy0 == 0) {                          // the channel's candidate means
      nb0 = colA < Wc ? pc[(size_t)ch * ncand + tA].x : 0.f;
      nb1 = colB < Wc ? pc[(size_t)ch * ncand + tB].x : 0.f;
    }
  };
  auto store_stage = [&](int buf) {
    float* sg = seg0 + buf * GM * SEG;
    if (tid < SEG)
#pragma unroll
      for (int q = 0; q < GM; ++q) sg[q * SEG + tid] = rseg[q];
    float* as = As0 + buf * BM * AST;
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      const int e = tid + u * 256;
      if (e < BM * GM * P2) {
        const int m = e / (GM * P2), rem = e - m * (GM * P2);
        as[m * AST + rem] = ra[u];
      }
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

  load_stage(0);
  store_stage(0);
  float mb0 = nb0, mb1 = nb1;                // the current channel's candidate means
  __syncthreads();
  for (int st = 0; st < S; ++st) {
    const int cur = st & 1;
    if (st + 1 < S) load_stage(st + 1);
    const float* sg = seg0 + cur * GM * SEG;
    const float* as = As0 + cur * BM * AST;
    const int rows = min(GM, P - (st % SPC) * GM);
#pragma unroll 1
    for (int q = 0; q < rows; ++q) {
      {
#pragma unroll
        for (int kk = 0; kk < P2 / 2; ++kk) {
          const int dx = 2 * kk + lhi;
          float a0 = as[(wm * 64 + l32) * AST + q * P2 + dx];
          float a1 = as[(wm * 64 + 32 + l32) * AST + q * P2 + dx];
          float b0 = sg[q * SEG + wn * 64 + l32 + dx] - mb0;
          float b1 = sg[q * SEG + wn * 64 + 32 + l32 + dx] - mb1;
          acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
      }
    }
    if (st + 1 < S) store_stage(cur ^ 1);
    if ((st + 1) % SPC == 0) {
      mb0 = nb0;
      mb1 = nb1;
    }
    __syncthreads();
  }

  // epilogue: d~ = ((||a~||^2 + ||p~||^2) - 2 S) + sum_c (P mu_kc - P mu_pc)^2,
  // one 32 x 32 tile at a time, channels in passes of CB (staged once when
  // Cp <= CB)
  auto stage_means = [&](int cb) {
    const int nc = min(CB, Cp - cb);
    for (int e = tid; e < nc * BM; e += 256) {
      const int c = e / BM, m = e - c * BM;
      const int gg = krow[m];
      skc[e] = gg >= 0 ? kc[(size_t)gg * Cp + cb + c] : 0.f;
    }
    for (int e = tid; e < nc * BN; e += 256) {
      const int c = e / BN, j = e - c * BN;
      spc[e] = c0 + j < Wc ? pc[(size_t)(cb + c) * ncand + (size_t)r * Wc + c0 + j].y : 0.f;
    }
  };
  const bool one_pass = Cp <= CB;
  if (tid < BM) skn[tid] = knr;
  if (pre) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * 256;
      if (e < Cp * BM) skc[e] = pkc[k];
      if (e < Cp * BN) spc[e] = ppc[k];
    }
  } else if (one_pass) {
    stage_means(0);
  }
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const float pp = nt ? pnB : pnA;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int i0 = wm * 64 + mt * 32 + 4 * lhi;   // rows i0 + 8 j + h, h < 4
      __builtin_amdgcn_sched_barrier(0);   // read this tile's accumulators only now
      float v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        v[q] = fmaf(-2.0f, acc[mt][nt][q], skn[i0 + 8 * (q >> 2) + (q & 3)] + pp);
      for (int cb = 0; cb < Cp; cb += CB) {
        if (!one_pass) {
          __syncthreads();
          stage_means(cb);
          __syncthreads();
        }
        const int nc = min(CB, Cp - cb);
#pragma unroll 1
        for (int c = 0; c < nc; ++c) {
          const float qv = spc[c * BN + wn * 64 + nt * 32 + l32];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float4 kv = *reinterpret_cast<const float4*>(skc + c * BM + i0 + 8 * j);
            const float d0 = kv.x - qv, d1 = kv.y - qv, d2 = kv.z - qv, d3 = kv.w - qv;
            v[4 * j] = fmaf(d0, d0, v[4 * j]);
            v[4 * j + 1] = fmaf(d1, d1, v[4 * j + 1]);
            v[4 * j + 2] = fmaf(d2, d2, v[4 * j + 2]);
            v[4 * j + 3] = fmaf(d3, d3, v[4 * j + 3]);
          }
        }
      }
      if ((nt ? colB : colA) < Wc) {
        const size_t t = nt ? tB : tA;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int i = i0 + 8 * (q >> 2) + (q & 3);
          if (krow[i] >= 0) dist[(size_t)(kbase + i) * ldd + t] = v[q];
        }
      }
    }
  }
}

// Small-D variant of the same contraction (D' = Cp P P2 <= SD_MAX, Cp <= 4):
// a persistent block keeps its key tile's whole centred slab in LDS and
// streams candidate tiles (one grid-row segment of BN candidates each)
// through it; a tile's image rows, candidate means and norms are loaded
// into registers while the previous tile computes, so a tile costs its
// MFMAs, its epilogue and two barriers.  Same arithmetic and output as
// k_match_f32.
constexpr int SD_MAX = 72;
constexpr int SD_CP = 4;

template <int P2>
__global__ void __launch_bounds__(256, 2)
k_match_f32_slab(const float* __restrict__ xp, int H, int W, int P, int Cp,
                 const float* __restrict__ Ac, int D, const float4* __restrict__ kn,
                 const float* __restrict__ kc, const float* __restrict__ pn,
                 const float2* __restrict__ pc, size_t ncand, const int32_t* __restrict__ kmap,
                 int g0, int nk, int npb, float* __restrict__ dist, size_t ldd) {
  constexpr int SEG = BN + P2;
  constexpr int AST = SD_MAX + 1;            // odd LDS stride of the key slab
  constexpr int NR = SD_MAX / P2;            // image rows per tile (Cp P), at most
  __shared__ float As[BM * AST];
  __shared__ float seg[NR * SEG];
  __shared__ __align__(16) float skc[SD_CP * BM];
  __shared__ float spc[SD_CP * BN];          // fl(P mu_pc) of the tile's candidates
  __shared__ float smu[SD_CP * BN];          // mu_pc
  __shared__ float spn[BN];
  __shared__ int krow[BM];
  __shared__ float skn[BM];

  const int Hc = H - P + 1, Wc = W - P + 1;
  const int ntc = (Wc + BN - 1) / BN;
  const int ntile = Hc * ntc;
  const int kt = blockIdx.x / npb, part = blockIdx.x - kt * npb;
  const int kbase = kt * BM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int NRr = Cp * P;                    // image rows of a tile
  const int DP = Cp * P * P2;                // padded key length in LDS

  // ---- key tile: rows, norms, scaled channel means, centred slab
  if (tid < BM) {
    const int g = kbase + tid;
    const int gg = g < nk ? (kmap ? kmap[g0 + g] : g0 + g) : -1;
    krow[tid] = gg;
    skn[tid] = gg >= 0 ? kn[gg].x : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < Cp * BM; e += 256) {
    const int c = e / BM, m = e - c * BM;
    const int gg = krow[m];
    skc[e] = gg >= 0 ? kc[(size_t)gg * Cp + c] : 0.f;
  }
  for (int e = tid; e < BM * DP; e += 256) {
    const int m = e / DP, rem = e - m * DP;
    const int row = rem / P2, dx = rem - row * P2;  // row = ch P + dy
    const int gg = krow[m];
    As[m * AST + rem] = (dx < P && gg >= 0) ? Ac[(size_t)gg * D + (size_t)row * P + dx] : 0.f;
  }

  // ---- per-tile operands, staged through registers (the rows' elements
  // spread over all threads)
  constexpr int RR = (NR * SEG + 255) / 256;
  float rseg[RR];
  float rmu[2], rpc[2], rpn = 0.f;
  auto fetch = [&](int tile) {
    const int r = tile / ntc, c0 = (tile - r * ntc) * BN;
#pragma unroll
    for (int k = 0; k < RR; ++k) {
      const int e = tid + k * 256;
      const int q = e / SEG, x = e - q * SEG;
      rseg[k] = 0.f;
      if (q < NRr) {
        const int ch = q / P, dy = q - ch * P;
        const int cc = c0 + x;
        if (cc < W) rseg[k] = xp[((size_t)ch * H + r + dy) * W + cc];
      }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * 256;
      rmu[k] = 0.f;
      rpc[k] = 0.f;
      if (e < Cp * BN) {
        const int c = e / BN, j = e - c * BN;
        if (c0 + j < Wc) {
          const float2 v = pc[(size_t)c * ncand + (size_t)r * Wc + c0 + j];
          rmu[k] = v.x;
          rpc[k] = v.y;
        }
      }
    }
    rpn = (tid < BN && c0 + tid < Wc) ? pn[(size_t)r * Wc + c0 + tid] : 0.f;
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < RR; ++k) {
      const int e = tid + k * 256;
      if (e < NRr * SEG) seg[e] = rseg[k];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * 256;
      if (e < Cp * BN) {
        smu[e] = rmu[k];
        spc[e] = rpc[k];
      }
    }
    if (tid < BN) spn[tid] = rpn;
  };

  if (part < ntile) {
    fetch(part);
    stage();
  }
  __syncthreads();
  for (int tile = part; tile < ntile; tile += npb) {
    const int r = tile / ntc, c0 = (tile - r * ntc) * BN;
    const int next = tile + npb;
    if (next < ntile) fetch(next);
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;
    for (int ch = 0; ch < Cp; ++ch) {
      const float mb0 = smu[ch * BN + wn * 64 + l32], mb1 = smu[ch * BN + wn * 64 + 32 + l32];
#pragma unroll 1
      for (int dy = 0; dy < P; ++dy) {
        const int row = ch * P + dy;
        const float* sg = seg + row * SEG;
#pragma unroll
        for (int kk = 0; kk < P2 / 2; ++kk) {
          const int dx = 2 * kk + lhi;
          float a0 = As[(wm * 64 + l32) * AST + row * P2 + dx];
          float a1 = As[(wm * 64 + 32 + l32) * AST + row * P2 + dx];
          float b0 = sg[wn * 64 + l32 + dx] - mb0;
          float b1 = sg[wn * 64 + 32 + l32 + dx] - mb1;
          acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
      }
    }
    // epilogue: d~ = ((||a~||^2 + ||p~||^2) - 2 S) + sum_c (P mu_kc - P mu_pc)^2
    const int colA = c0 + wn * 64 + l32, colB = colA + 32;
    const size_t tA = (size_t)r * Wc + colA, tB = tA + 32;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const float pp = spn[wn * 64 + nt * 32 + l32];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int i0 = wm * 64 + mt * 32 + 4 * lhi;   // rows i0 + 8 j + h, h < 4
        __builtin_amdgcn_sched_barrier(0);
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          v[q] = fmaf(-2.0f, acc[mt][nt][q], skn[i0 + 8 * (q >> 2) + (q & 3)] + pp);
#pragma unroll 1
        for (int c = 0; c < Cp; ++c) {
          const float qv = spc[c * BN + wn * 64 + nt * 32 + l32];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float4 kv = *reinterpret_cast<const float4*>(skc + c * BM + i0 + 8 * j);
            const float d0 = kv.x - qv, d1 = kv.y - qv, d2 = kv.z - qv, d3 = kv.w - qv;
            v[4 * j] = fmaf(d0, d0, v[4 * j]);
            v[4 * j + 1] = fmaf(d1, d1, v[4 * j + 1]);
            v[4 * j + 2] = fmaf(d2, d2, v[4 * j + 2]);
            v[4 * j + 3] = fmaf(d3, d3, v[4 * j + 3]);
          }
        }
        if ((nt ? colB : colA) < Wc) {
          const size_t t = nt ? tB : tA;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int i = i0 + 8 * (q >> 2) + (q & 3);
            if (krow[i] >= 0) dist[(size_t)(kbase + i) * ldd + t] = v[q];
          }
        }
      }
    }
    __syncthreads();                         // every wave is done with this tile
    if (next < ntile) stage();
    __syncthreads();
  }
}

template <int P2>
void launch_match_t(const glr_plan* pl, const float* xp, const float* Ac, const float* kn,
                    const float* kc, const float* pn, const float* pc, const int32_t* kmap,
                    int g0, int nk, float* dist, hipStream_t s) {
  const int Hc = pl->Hc, Wc = pl->Wc;
  const int ntc = (Wc + BN - 1) / BN;
  const int nkt = (nk + BM - 1) / BM;
  if constexpr (P2 >= 4 && P2 <= 8) {
    if (pl->Cp * pl->P * P2 <= SD_MAX && pl->Cp <= SD_CP) {
      // persistent blocks: about two per CU over all key tiles
      const int ntile = Hc * ntc;
      const int npb = std::max(1, std::min(ntile, (2 * 256 + nkt - 1) / nkt));
      hipLaunchKernelGGL(k_match_f32_slab<P2>, dim3((unsigned)(nkt * npb)), dim3(256), 0, s, xp,
                         pl->H, pl->W, pl->P, pl->Cp, Ac, pl->D, (const float4*)kn, kc, pn,
                         (const float2*)pc, (size_t)pl->Ncand, kmap, g0, nk, npb, dist,
                         (size_t)pl->ldd);
      return;
    }
  }
  size_t blocks = (size_t)nkt * Hc * ntc;
  hipLaunchKernelGGL(k_match_f32<P2>, dim3((unsigned)blocks), dim3(256), 0, s, xp, pl->H, pl->W,
                     pl->P, pl->Cp, Ac, pl->D, (const float4*)kn, kc, pn, (const float2*)pc,
                     (size_t)pl->Ncand, kmap, g0, nk, dist, (size_t)pl->ldd);
}

// Per key of the FP32 form (one wave per key): Ac, kn, kc as described at
// k_match_f32.  Channel means from FP64 sums, correctly rounded to FP32.
__global__ void k_key_meta_pc(const float* __restrict__ A, int D, int P, int Cp, int N,
                              float* __restrict__ Ac, float4* __restrict__ kn,
                              float* __restrict__ kc) {
  const int g = blockIdx.x;
  if (g >= N) return;
  const int n = P * P;
  const float* k = A + (size_t)g * D;
  float* ac = Ac + (size_t)g * D;
  const int l = threadIdx.x;
  float an = 0.f, h = 0.f;
  for (int c = 0; c < Cp; ++c) {
    double s = 0.0, sb = 0.0;
    for (int i = l; i < n; i += 64) {
      const double v = k[c * n + i];
      s += v;
      sb += fabs(v);
    }
    for (int o = 32; o > 0; o >>= 1) {
      s += __shfl_xor(s, o, 64);
      sb += __shfl_xor(sb, o, 64);
    }
    const float mu = (float)(s / n);
    for (int i = l; i < n; i += 64) {
      const float a = k[c * n + i] - mu;
      ac[c * n + i] = a;
      an = fmaf(a, a, an);
    }
    if (l == 0) kc[(size_t)g * Cp + c] = (float)P * mu;
    const float ma = (float)(sb / n);
    h = fmaf(ma, ma, h);
  }
  for (int o = 32; o > 0; o >>= 1) an += __shfl_xor(an, o, 64);
  if (l == 0) kn[g] = make_float4(an, sqrtf(h), 0.f, sqrtf(an));
}

// Per candidate of the FP32 form (one thread per candidate): pn[j] = ||p~||^2,
// pc[c][j] = (mu_pc, fl(P mu_pc)), pq[j] = (h_p, ||p~||) for the top-K bound.
__global__ void k_cand_meta_pc(const float* __restrict__ xp, int Cp, int H, int W, int P,
                               float* __restrict__ pn, float2* __restrict__ pc,
                               float2* __restrict__ pq) {
  const int Wc = W - P + 1, Hc = H - P + 1;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t ncand = (size_t)Hc * Wc;
  if (j >= (int)ncand) return;
  const int r = j / Wc, c = j - r * Wc;
  const int n = P * P;
  float sq = 0.f, h = 0.f;
  for (int ch = 0; ch < Cp; ++ch) {
    double s = 0.0, sb = 0.0;
    for (int dy = 0; dy < P; ++dy) {
      const float* row = xp + ((size_t)ch * H + r + dy) * W + c;
      for (int dx = 0; dx < P; ++dx) {
        s += (double)row[dx];
        sb += fabs((double)row[dx]);
      }
    }
    const float mu = (float)(s / n);
    for (int dy = 0; dy < P; ++dy) {
      const float* row = xp + ((size_t)ch * H + r + dy) * W + c;
      for (int dx = 0; dx < P; ++dx) {
        const float v = row[dx] - mu;
        sq = fmaf(v, v, sq);
      }
    }
    pc[(size_t)ch * ncand + j] = make_float2(mu, (float)P * mu);
    const float ma = (float)(sb / n);
    h = fmaf(ma, ma, h);
  }
  pn[j] = sq;
  pq[j] = make_float2(sqrtf(h), sqrtf(sq));
}

// ---------------------------------------------------------------- BF16 form
// Centred form of the same distance (exact identity):
//   a = k - mu_k 1, pbar = p - mu_p 1 (FP32),  dmu = mu_k - mu_p,
//   ||k - p||^2 = ||a||^2 + ||pbar||^2 - 2<a, pbar> + D dmu^2 + 2 dmu (sum a - sum pbar)
// (plus rounding residues of the two subtractions, covered by the error
// bound).  <a, pbar> runs on BF16 MFMA with FP32 accumulation; centring both
// operands shrinks the BF16 rounding error, which scales with ||a|| ||pbar||.

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;        // round to nearest even (finite input)
}

// BF16 operand layout.  A channel's P x P patch block is padded to R rows of
// X = 8 (P <= 8) or 16 (P <= 16) columns and cut into NS = R*X/8 slices of 8
// consecutive columns; slice t = y*(X/8) + dx/8.  One MFMA (K = 16) takes two
// slices, lanes 0-31 the even one and lanes 32-63 the odd one, for the key
// and the candidate alike.  R is P rounded up to even for X = 8, and 12 or
// 16 for X = 16 (padding is zero).
__host__ __device__ constexpr int bf16_slices(int P) {
  return P <= 8 ? P + (P & 1) : (P <= 12 ? 24 : 32);
}

// BF16 value of f (round to nearest even) as a float
__device__ __forceinline__ float bf16_val(float f) { return __uint_as_float(bf16_rne(f) << 16); }

// Per key: kmb[g] = (||a||^2, mu_k, sum a, ||a||) with a = k - mu_k (FP32,
// the values both matchers use) and kre[g] = ||a - bf16(a)|| (the BF16
// operand's rounding residual, for the error bound); with Ab, also
// Ab[g][c][t][0..8) = bf16(a) in the BF16 slice layout (padding zero).  One
// wave per key.
// raw != 0 (the edge-map score): no centring (mu = 0) and kmb = (0, 0, 0,
// ||k||), so the BF16 matcher's epilogue returns -2 <k, p> exactly for 0/1
// vectors.
__global__ void k_key_meta(const float* __restrict__ A, int D, int P, int Cp, int NS, int XS,
                           int N, uint16_t* __restrict__ Ab, float4* __restrict__ kmb,
                           float* __restrict__ kre, int raw) {
  const int g = blockIdx.x;
  if (g >= N) return;
  const float* k = A + (size_t)g * D;
  const int l = threadIdx.x;
  float s = 0.f;
  for (int d = l; d < D; d += 64) s += k[d];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  const float mu = raw ? 0.f : s / (float)D;
  float an = 0.f, sa = 0.f, en = 0.f;
  for (int d = l; d < D; d += 64) {
    const float a = k[d] - mu;
    const float e = a - bf16_val(a);        // exact
    an = fmaf(a, a, an);
    sa += a;
    en = fmaf(e, e, en);
  }
  for (int o = 32; o > 0; o >>= 1) {
    an += __shfl_xor(an, o, 64);
    sa += __shfl_xor(sa, o, 64);
    en += __shfl_xor(en, o, 64);
  }
  if (l == 0) {
    kmb[g] = raw ? make_float4(0.f, 0.f, 0.f, sqrtf(an)) : make_float4(an, mu, sa, sqrtf(an));
    kre[g] = sqrtf(en);
  }
  if (!Ab) return;
  const int row = NS * 8;
  for (int e = l; e < Cp * row; e += 64) {
    const int c = e / row, rem = e - c * row, t = rem >> 3;
    const int y = t / XS, dx = (t - y * XS) * 8 + (rem & 7);
    const float a = (y < P && dx < P) ? k[(c * P + y) * P + dx] - mu : 0.f;
    Ab[(size_t)g * Cp * row + e] = (uint16_t)bf16_rne(a);
  }
}

// Per candidate: cmeta[j] = (mu_p, ||pbar||^2, ||pbar||, sum pbar) with
// pbar = p - mu_p computed in FP32 exactly as the matcher forms its operand;
// cm2[j] = (mu_p, ||pbar||) and cre[j] = ||pbar - bf16(pbar)|| (the residual
// of the matcher's round-to-nearest-even BF16 operand) for the error bound
// of the top-K pass.  One block per 256 candidates of one grid row: each
// channel's P image rows (256 + P - 1 columns) are staged in LDS and every
// thread reads its window from there; the sums run in four partial sums per
// quantity (over dx mod 4, combined in a fixed order), so the additions do
// not form one dependency chain per thread.
constexpr int CMB = 256;                     // candidates per block
__global__ void __launch_bounds__(CMB)
k_cand_meta(const float* __restrict__ xp, int Cp, int H, int W, int P,
            float4* __restrict__ cmeta, float2* __restrict__ cm2, float* __restrict__ cre,
            int raw) {
  __shared__ float tile[16 * (CMB + 15)];    // P <= 16
  const int Wc = W - P + 1;
  const int r = blockIdx.y, c0 = blockIdx.x * CMB, t = threadIdx.x;
  const int TW = CMB + P - 1;
  const int D = Cp * P * P;
  auto stage = [&](int ch) {
    __syncthreads();                         // the previous channel's readers are done
    for (int i = t; i < P * TW; i += CMB) {
      const int dy = i / TW, x = i - dy * TW;
      tile[i] = xp[((size_t)ch * H + r + dy) * W + min(c0 + x, W - 1)];
    }
    __syncthreads();
  };
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < Cp; ++ch) {
    stage(ch);
    for (int dy = 0; dy < P; ++dy) {
      const float* row = tile + dy * TW + t;
      for (int dx = 0; dx < P; dx += 4) {
        s[0] += row[dx];
        if (dx + 1 < P) s[1] += row[dx + 1];
        if (dx + 2 < P) s[2] += row[dx + 2];
        if (dx + 3 < P) s[3] += row[dx + 3];
      }
    }
  }
  const float mu = raw ? 0.f : ((s[0] + s[1]) + (s[2] + s[3])) / (float)D;
  float pn[4] = {0.f, 0.f, 0.f, 0.f}, sp[4] = {0.f, 0.f, 0.f, 0.f}, en[4] = {0.f, 0.f, 0.f, 0.f};
  auto acc = [&](int k, float x) {
    const float v = x - mu;
    const float e = v - bf16_val(v);         // exact
    pn[k] = fmaf(v, v, pn[k]);
    sp[k] += v;
    en[k] = fmaf(e, e, en[k]);
  };
  for (int ch = 0; ch < Cp; ++ch) {
    stage(ch);
    for (int dy = 0; dy < P; ++dy) {
      const float* row = tile + dy * TW + t;
      for (int dx = 0; dx < P; dx += 4) {
        acc(0, row[dx]);
        if (dx + 1 < P) acc(1, row[dx + 1]);
        if (dx + 2 < P) acc(2, row[dx + 2]);
        if (dx + 3 < P) acc(3, row[dx + 3]);
      }
    }
  }
  if (c0 + t >= Wc) return;                  // no block barrier below
  const size_t j = (size_t)r * Wc + c0 + t;
  const float pnt = (pn[0] + pn[1]) + (pn[2] + pn[3]);
  const float spt = (sp[0] + sp[1]) + (sp[2] + sp[3]);
  const float ent = (en[0] + en[1]) + (en[2] + en[3]);
  const float pr = sqrtf(pnt);
  cmeta[j] = raw ? make_float4(0.f, 0.f, pr, 0.f) : make_float4(mu, pnt, pr, spt);
  cm2[j] = make_float2(mu, pr);
  cre[j] = sqrtf(ent);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Candidates per block of the BF16 matcher: 256 (each wave 64 keys x 128
// candidates, four 32 x 32 tiles per key tile) while the operand buffers fit
// LDS (NS <= 8), else 128.
__host__ __device__ constexpr int bf16_nt(int NS) { return NS <= 8 ? 4 : 2; }

// BF16 MFMA matcher: 128 keys x 64 NT candidates per block (one grid-row
// segment), one channel (NS slices of the padded patch block) per step.
// The candidate operand is built in LDS per step from the staged image rows:
// Bs[t][j][0..8) = bf16(x[c][r+y][c0+j+dx] - mu_p(j)) for slice t = (y, dx/8);
// a thread builds four consecutive candidates of one slice from three
// 16-byte reads of the row (their eight-value windows overlap).  Bs rows
// get 16 bytes of padding after every 16 candidates, so the stores (lanes
// four candidates apart) and the fragment reads (consecutive candidates)
// are both free of bank conflicts.
template <int NS>
__global__ void __launch_bounds__(256, 2)
k_match_bf16(const float* __restrict__ xp, int H, int W, int P, int Cp,
             const uint16_t* __restrict__ Ab, const float4* __restrict__ kmb,
             const float4* __restrict__ cmeta, int g0, int nk, float* __restrict__ dist,
             size_t ldd) {
  constexpr int NT = bf16_nt(NS);         // 32-candidate tiles per wave
  constexpr int BNB = 64 * NT;            // candidates per block
  constexpr int XS = NS > 8 ? 2 : 1;      // slices per patch row
  constexpr int RP = NS / XS;             // padded rows
  constexpr int ROWB = NS * 8;            // bf16 per key and channel
  constexpr int AST = ROWB + 8;           // LDS row stride of the key slab (bf16)
  constexpr int SEGW = BNB + 8 * XS;      // staged image row length (multiple of 4)
  constexpr int NAU = ROWB / 16;          // uint4 per thread for the key slab (2 threads/key)
  constexpr int NSEG = (RP * SEGW + 255) / 256;
  constexpr int QW = BNB / 4;             // four-candidate groups per slice
  __shared__ __align__(16) uint16_t As[BM * AST];
  __shared__ __align__(16) uint16_t Bs[NS * BNB * 8 + NS * BNB / 2];
  __shared__ __align__(16) float seg[RP * SEGW];
  __shared__ __align__(16) float mup[BNB];
  __shared__ float4 skm[BM];

  const int Hc = H - P + 1, Wc = W - P + 1;
  const int ntc = (Wc + BNB - 1) / BNB;
  int b = blockIdx.x;
  const int ct = b % ntc;
  b /= ntc;
  const int r = b % Hc;
  const int kt = b / Hc;
  const int c0 = ct * BNB;
  const int kbase = kt * BM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int D = Cp * P * P;

  for (int j = tid; j < BNB; j += 256) {
    const int col = c0 + j;
    mup[j] = col < Wc ? cmeta[(size_t)r * Wc + col].x : 0.f;
  }
  if (tid < BM) {
    const int g = kbase + tid;
    skm[tid] = g < nk ? kmb[g0 + g] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  uint4 ra[NAU];
  float rs[NSEG];
  const int akey = tid >> 1, ahalf = tid & 1;
  auto load_stage = [&](int ch) {
    const int g = kbase + akey;
#pragma unroll
    for (int u = 0; u < NAU; ++u) {
      ra[u] = make_uint4(0, 0, 0, 0);
      if (g < nk)
        ra[u] = *reinterpret_cast<const uint4*>(Ab + ((size_t)(g0 + g) * Cp + ch) * ROWB +
                                                ahalf * (ROWB / 2) + u * 8);
    }
#pragma unroll
    for (int u = 0; u < NSEG; ++u) {
      const int e = tid + u * 256;
      float v = 0.f;
      if (e < RP * SEGW) {
        const int y = e / SEGW, cc = c0 + (e - y * SEGW);
        if (y < P && cc < W) v = xp[((size_t)ch * H + r + y) * W + cc];
      }
      rs[u] = v;
    }
  };

  f32x16 acc[2][NT];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

  load_stage(0);
  for (int ch = 0; ch < Cp; ++ch) {
#pragma unroll
    for (int u = 0; u < NAU; ++u)
      *reinterpret_cast<uint4*>(As + akey * AST + ahalf * (ROWB / 2) + u * 8) = ra[u];
#pragma unroll
    for (int u = 0; u < NSEG; ++u) {
      const int e = tid + u * 256;
      if (e < RP * SEGW) seg[e] = rs[u];
    }
    __syncthreads();
    // padding entries (dx >= P, or rows y >= P, staged as zeros) take
    // finite values here and meet zeros in the key slices
#pragma unroll
    for (int w = tid; w < NS * QW; w += 256) {
      const int t = w / QW, j0 = 4 * (w - t * QW);
      const int y = t / XS, xb = (t - y * XS) * 8;
      const float4* src = reinterpret_cast<const float4*>(seg + y * SEGW + j0 + xb);
      const float4 f0 = src[0], f1 = src[1], f2 = src[2];
      const float f[12] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w,
                           f2.x, f2.y, f2.z, f2.w};
      const float4 m4 = *reinterpret_cast<const float4*>(mup + j0);
      const float mm[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        uint32_t wd[4];
#pragma unroll
        for (int h = 0; h < 4; ++h)
          wd[h] = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                      (f32x2){f[u + 2 * h] - mm[u], f[u + 2 * h + 1] - mm[u]},
                      bf16x2));   // round to nearest even
        const int row = t * BNB + j0 + u;
        *reinterpret_cast<uint4*>(Bs + row * 8 + (row >> 4) * 8) =
            make_uint4(wd[0], wd[1], wd[2], wd[3]);
      }
    }
    __syncthreads();
    if (ch + 1 < Cp) load_stage(ch + 1);
#pragma unroll
    for (int kk = 0; kk < NS / 2; ++kk) {
      const int t = 2 * kk + lhi;
      bf16x8 a[2], bb[NT];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        a[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                    As + (wm * 64 + mt * 32 + l32) * AST + t * 8));
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int row = t * BNB + wn * (32 * NT) + nt * 32 + l32;
        bb[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                     Bs + row * 8 + (row >> 4) * 8));
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], bb[nt], acc[mt][nt], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: d~ = ||a||^2 + ||pbar||^2 - 2 S + D dmu^2 + 2 dmu (sum a - sum pbar)
  const bool all_keys = kbase + BM <= nk;   // block-uniform: no per-row test
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int col = c0 + wn * (32 * NT) + nt * 32 + l32;
    if (col >= Wc) continue;
    const size_t t = (size_t)r * Wc + col;
    const float4 cm = cmeta[t];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = wm * 64 + mt * 32 + 8 * (q >> 2) + 4 * lhi + (q & 3);
        const int g = kbase + i;
        if (all_keys || g < nk)
          dist[(size_t)g * ldd + t] = centred_dist(skm[i], cm, acc[mt][nt][q], D);
      }
  }
}

// Double-buffered BF16 matcher for patch sides up to 8 (NS <= 8 slices per
// channel): 256 keys x 256 candidates per block, eight waves, each a 64 x 128
// tile (2 x 4 MFMA 32 x 32 tiles).  Per channel the key slab (As) and the
// candidate operand (Bs) are staged in one of two LDS buffers while the MFMAs
// read the other, with one barrier per channel.  The candidate operand is
// built from registers: wave t (t < NS) builds slice t (patch row t) of the
// 256 candidates, lane l the four candidates 4l..4l+3 from three 16-byte
// reads of image row r + t (columns c0 + 4l .. c0 + 4l + 11; the eight-value
// windows of the four candidates overlap).  The loads for channel ch + 2 are
// issued once channel ch + 1 is staged, a whole channel of MFMAs ahead of
// their use.  The channel loop is unrolled by two so both buffers have static
// addresses and the staging of one buffer can be scheduled between the MFMAs
// that read the other.  Same operand layout, slice order and epilogue as
// k_match_bf16 (the same MFMA sequence per output).
constexpr int DBM = 256;                  // keys per block (double-buffered form)
constexpr int DBN = 256;                  // candidates per block

// Instruction order of one channel step (LDS reads of the first two
// k-steps, then per k-step its eight MFMAs with the next k-step's reads and a
// share of the staging work between them), so the staging of the other
// buffer runs in the shadow of the MFMAs and at most two k-steps of operands
// are live.
template <int NS>
__device__ __forceinline__ void sched_db_step() {
  constexpr int KS = NS / 2;
  __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);          // DS reads, k-step 0
  if (KS > 1) __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);      // VALU (operand build)
      if (i == 3 && kk + 2 < KS) __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
      if (i & 1) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // DS write
      if (kk == KS - 1 && (i & 1) == 0) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
  }
}

template <int NS, bool VEC4>
__global__ void __launch_bounds__(512, 1)
k_match_bf16_db(const float* __restrict__ xp, int H, int W, int P, int Cp,
                const uint16_t* __restrict__ Ab, const float4* __restrict__ kmb,
                const float4* __restrict__ cmeta, int g0, int nk, float* __restrict__ dist,
                size_t ldd) {
  static_assert(NS <= 8 && (NS & 1) == 0, "double-buffered matcher: P <= 8");
  constexpr int NT = 4;                     // 32-candidate tiles per wave
  constexpr int ROWB = NS * 8;              // bf16 per key and channel
  constexpr int AST = ROWB + 8;             // LDS row stride of the key slab (bf16)
  constexpr int NAU = NS / 2;               // uint4 per thread of the key slab (2 threads/key)
  constexpr int ASZ = DBM * AST;
  constexpr int BSZ = NS * DBN * 8 + NS * DBN / 2;
  __shared__ __align__(16) uint16_t As0[ASZ];
  __shared__ __align__(16) uint16_t As1[ASZ];
  __shared__ __align__(16) uint16_t Bs0[BSZ];
  __shared__ __align__(16) uint16_t Bs1[BSZ];
  __shared__ float4 skm[DBM];

  const int Hc = H - P + 1, Wc = W - P + 1;
  const int ntc = (Wc + DBN - 1) / DBN;
  int b = blockIdx.x;
  const int ct = b % ntc;
  b /= ntc;
  const int r = b % Hc;
  const int kt = b / Hc;
  const int c0 = ct * DBN;
  const int kbase = kt * DBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int D = Cp * P * P;

  if (tid < DBM) {
    const int g = kbase + tid;
    skm[tid] = g < nk ? kmb[g0 + g] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // the builder's four candidates and their means (constant over channels)
  const int cb = c0 + 4 * lane;
  float mu[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) mu[u] = cb + u < Wc ? cmeta[(size_t)r * Wc + cb + u].x : 0.f;
  const bool builder = NS == 8 || wave < NS;   // all eight waves build when NS = 8
  const bool row_ok = wave < P;             // padding rows (P odd) are zeros
  const int akey = tid >> 1, ahalf = tid & 1;
  const bool key_ok = kbase + akey < nk;
  const uint16_t* asrc = Ab + (size_t)(g0 + (key_ok ? kbase + akey : 0)) * Cp * ROWB +
                         ahalf * (ROWB / 2);
  const size_t HW = (size_t)H * W;
  const float* bsrc = xp + (size_t)(r + (row_ok ? wave : 0)) * W;

  // Loads are always issued in bounds; what must read as zero (keys past
  // nk, columns past W, padding rows, channels past Cp: an odd Cp is rounded
  // up to even) is cleared by bit masks when staged, so the loads have no
  // consumer before the next staging and every step stays one block.
  uint4 ra[NAU];
  float4 rb[3];
  uint32_t km, rm[3];
  const uint32_t kmask = key_ok ? 0xffffffffu : 0u;
  const uint32_t rmask = row_ok ? 0xffffffffu : 0u;
  auto load = [&](int ch) {
    const uint32_t cm_ok = ch < Cp ? 0xffffffffu : 0u;
    km = kmask & cm_ok;
    ch = min(ch, Cp - 1);
#pragma unroll
    for (int u = 0; u < NAU; ++u)
      ra[u] = *reinterpret_cast<const uint4*>(asrc + (size_t)ch * ROWB + u * 8);
    if (builder) {
      const float* row = bsrc + (size_t)ch * HW;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int cm = cb + 4 * m;
        if (VEC4) {
          // W % 4 == 0 and cm % 4 == 0: the group is wholly inside the row
          // or wholly past its end (then read in bounds and cleared)
          rb[m] = *reinterpret_cast<const float4*>(row + min(cm, W - 4));
          rm[m] = cm < W ? rmask & cm_ok : 0u;
        } else {
          // columns past W read the row's last value; the builder's
          // candidates that use them lie past Wc and are never stored
          rb[m] = make_float4(row[min(cm, W - 1)], row[min(cm + 1, W - 1)],
                              row[min(cm + 2, W - 1)], row[min(cm + 3, W - 1)]);
          rm[m] = rmask & cm_ok;
        }
      }
    }
  };
  // LDS byte offsets: one per-lane base per operand, the rest immediates.
  // Candidate row q of slice t sits at 16 (q' + q' / 16), q' = t DBN + q.
  const int a_st = (akey * AST + ahalf * (ROWB / 2)) * 2;
  const int bq = wave * DBN + 4 * lane;                 // builder: rows bq .. bq + 3
  const int b_st = 16 * (bq + (bq >> 4));
  const int a_rd = ((wm * 64 + l32) * AST + lhi * 8) * 2;
  const int bl = lhi * DBN + wn * (32 * NT) + l32;     // fragment row of t = lhi, nt = 0
  const int b_rd = 16 * (bl + (bl >> 4));
  auto stage = [&](uint16_t* As, uint16_t* Bs) {
    char* Ab8 = reinterpret_cast<char*>(As) + a_st;
    char* Bb8 = reinterpret_cast<char*>(Bs) + b_st;
#pragma unroll
    for (int u = 0; u < NAU; ++u)
      *reinterpret_cast<uint4*>(Ab8 + 16 * u) =
          make_uint4(ra[u].x & km, ra[u].y & km, ra[u].z & km, ra[u].w & km);
    if (builder) {
      auto cl = [](float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) & m); };
      const float f[12] = {cl(rb[0].x, rm[0]), cl(rb[0].y, rm[0]), cl(rb[0].z, rm[0]),
                           cl(rb[0].w, rm[0]), cl(rb[1].x, rm[1]), cl(rb[1].y, rm[1]),
                           cl(rb[1].z, rm[1]), cl(rb[1].w, rm[1]), cl(rb[2].x, rm[2]),
                           cl(rb[2].y, rm[2]), cl(rb[2].z, rm[2]), cl(rb[2].w, rm[2])};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        uint32_t wd[4];
#pragma unroll
        for (int h = 0; h < 4; ++h)
          wd[h] = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                      (f32x2){f[u + 2 * h] - mu[u], f[u + 2 * h + 1] - mu[u]},
                      bf16x2));   // round to nearest even
        // rows bq + u share bq's 16-row group (bq is a multiple of 4)
        *reinterpret_cast<uint4*>(Bb8 + 16 * u) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
      }
    }
  };

  f32x16 acc[2][NT];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

  auto mfma = [&](const uint16_t* As, const uint16_t* Bs) {
    const char* Ar8 = reinterpret_cast<const char*>(As) + a_rd;
    const char* Br8 = reinterpret_cast<const char*>(Bs) + b_rd;
#pragma unroll
    for (int kk = 0; kk < NS / 2; ++kk) {
      bf16x8 a[2], bb[NT];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        a[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                    Ar8 + 2 * (mt * 32 * AST + 2 * kk * 8)));
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)   // slice 2 kk + lhi, rows + 2 kk DBN + 32 nt
        bb[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                     Br8 + 16 * ((2 * kk * DBN + nt * 32) + (2 * kk * DBN + nt * 32) / 16)));
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], bb[nt], acc[mt][nt], 0, 0, 0);
    }
  };

  // channel ch is read from buffer ch & 1; the loop runs over an even
  // channel count (a zero channel pads an odd Cp) so that each iteration is
  // one straight-line block and the accumulators stay in place
  const int Cp2 = Cp + (Cp & 1);
  load(0);
  stage(As0, Bs0);
  load(1);
  __syncthreads();
  for (int ch = 0; ch < Cp2; ch += 2) {
    mfma(As0, Bs0);
    stage(As1, Bs1);
    load(ch + 2);
    sched_db_step<NS>();
    __syncthreads();
    mfma(As1, Bs1);
    stage(As0, Bs0);
    load(ch + 3);
    sched_db_step<NS>();
    __syncthreads();
  }

  // epilogue: d~ = ||a||^2 + ||pbar||^2 - 2 S + D dmu^2 + 2 dmu (sum a - sum pbar)
  // (the arithmetic of centred_dist).  Key terms are read once per output
  // row, candidate terms once per column; each row's four 32-candidate runs
  // are stored from one row pointer.
  const int colb = c0 + wn * (32 * NT) + l32;
  float4 cmv[NT];
  bool cok[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int col = colb + nt * 32;
    cok[nt] = col < Wc;
    cmv[nt] = cmeta[(size_t)r * Wc + (cok[nt] ? col : 0)];
  }
  float* dbase = dist + (size_t)r * Wc + colb;
  const int nrow = min(DBM, nk - kbase);     // rows of this key tile that exist
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = wm * 64 + mt * 32 + 8 * (q >> 2) + 4 * lhi + (q & 3);
      if (i >= nrow) continue;
      const float4 km = skm[i];
      float* drow = dbase + (size_t)(kbase + i) * ldd;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const float4 cm = cmv[nt];
        const float dmu = km.y - cm.x;
        const float base = (km.x + cm.y) - 2.0f * acc[mt][nt][q];
        const float d = (base + ((float)D * dmu) * dmu) + 2.0f * dmu * (km.z - cm.w);
        if (cok[nt]) drow[nt * 32] = d;
      }
    }
}

template <int NS>
void launch_match_bf16_db(const glr_plan* pl, const float* xp, const uint16_t* Ab,
                          const float* kmb, const float* cmeta, int g0, int nk, float* dist,
                          hipStream_t s) {
  const int ntc = (pl->Wc + DBN - 1) / DBN;
  const int nkt = (nk + DBM - 1) / DBM;
  const size_t blocks = (size_t)nkt * pl->Hc * ntc;
  if ((pl->W & 3) == 0)
    hipLaunchKernelGGL((k_match_bf16_db<NS, true>), dim3((unsigned)blocks), dim3(512), 0, s, xp,
                       pl->H, pl->W, pl->P, pl->Cp, Ab, (const float4*)kmb, (const float4*)cmeta,
                       g0, nk, dist, (size_t)pl->ldd);
  else
    hipLaunchKernelGGL((k_match_bf16_db<NS, false>), dim3((unsigned)blocks), dim3(512), 0, s, xp,
                       pl->H, pl->W, pl->P, pl->Cp, Ab, (const float4*)kmb, (const float4*)cmeta,
                       g0, nk, dist, (size_t)pl->ldd);
}

template <int NS>
void launch_match_bf16_t(const glr_plan* pl, const float* xp, const uint16_t* Ab,
                         const float* kmb, const float* cmeta, int g0, int nk, float* dist,
                         hipStream_t s) {
  constexpr int BNB = 64 * bf16_nt(NS);
  const int ntc = (pl->Wc + BNB - 1) / BNB;
  const int nkt = (nk + BM - 1) / BM;
  const size_t blocks = (size_t)nkt * pl->Hc * ntc;
  hipLaunchKernelGGL(k_match_bf16<NS>, dim3((unsigned)blocks), dim3(256), 0, s, xp, pl->H, pl->W,
                     pl->P, pl->Cp, Ab, (const float4*)kmb, (const float4*)cmeta, g0, nk, dist,
                     (size_t)pl->ldd);
}
}  // namespace

void launch_gather_keys(const glr_plan* pl, const float* xp, const int32_t* keys, float* A,
                        uint32_t* tsh, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_keys, dim3(pl->N), dim3(64), 0, s, xp, pl->H, pl->W, pl->P, pl->D,
                     keys, pl->N, A, tsh, std::min(pl->n_chunk, pl->N));
}

int bf16_key_row(int P) { return bf16_slices(P) * 8; }

void launch_key_meta(const glr_plan* pl, const float* A, uint16_t* Ab, float* kmb, float* kre,
                     int raw, hipStream_t s) {
  const int NS = bf16_slices(pl->P);
  hipLaunchKernelGGL(k_key_meta, dim3(pl->N), dim3(64), 0, s, A, pl->D, pl->P, pl->Cp, NS,
                     NS > 8 ? 2 : 1, pl->N, Ab, (float4*)kmb, kre, raw);
}

void launch_cand_meta(const glr_plan* pl, const float* xp, float* cmeta, float* cm2, float* cre,
                      int raw, hipStream_t s) {
  const int Wc = pl->W - pl->P + 1, Hc = pl->H - pl->P + 1;
  hipLaunchKernelGGL(k_cand_meta, dim3((Wc + CMB - 1) / CMB, Hc), dim3(CMB), 0, s, xp, pl->Cp,
                     pl->H, pl->W, pl->P, (float4*)cmeta, (float2*)cm2, cre, raw);
}

void launch_key_meta_pc(const glr_plan* pl, const float* A, float* Ac, float* kn, float* kc,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_key_meta_pc, dim3(pl->N), dim3(64), 0, s, A, pl->D, pl->P, pl->Cp, pl->N,
                     Ac, (float4*)kn, kc);
}

void launch_cand_meta_pc(const glr_plan* pl, const float* xp, float* pn, float* pc, float* pq,
                         hipStream_t s) {
  const int n = pl->Ncand;
  hipLaunchKernelGGL(k_cand_meta_pc, dim3((n + 255) / 256), dim3(256), 0, s, xp, pl->Cp, pl->H,
                     pl->W, pl->P, pn, (float2*)pc, (float2*)pq);
}

void launch_match_f32(const glr_plan* pl, const float* xp, const float* Ac, const float* kn,
                      const float* kc, const float* pn, const float* pc, const int32_t* kmap,
                      int g0, int nk, float* dist, hipStream_t s) {
#define GLR_MATCH_CASE(c, p2) \
  case c: launch_match_t<p2>(pl, xp, Ac, kn, kc, pn, pc, kmap, g0, nk, dist, s); break;
  switch ((pl->P + 1) / 2) {
    GLR_MATCH_CASE(1, 2)
    GLR_MATCH_CASE(2, 4)
    GLR_MATCH_CASE(3, 6)
    GLR_MATCH_CASE(4, 8)
    GLR_MATCH_CASE(5, 10)
    GLR_MATCH_CASE(6, 12)
    GLR_MATCH_CASE(7, 14)
    default: launch_match_t<16>(pl, xp, Ac, kn, kc, pn, pc, kmap, g0, nk, dist, s); break;
  }
#undef GLR_MATCH_CASE
}

void launch_match_bf16(const glr_plan* pl, const float* xp, const uint16_t* Ab, const float* kmb,
                       const float* cmeta, int g0, int nk, float* dist, hipStream_t s) {
  switch (bf16_slices(pl->P)) {
    case 2: launch_match_bf16_db<2>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
    case 4: launch_match_bf16_db<4>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
    case 6: launch_match_bf16_db<6>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
    case 8: launch_match_bf16_db<8>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
    case 24: launch_match_bf16_t<24>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
    default: launch_match_bf16_t<32>(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s); break;
  }
}
