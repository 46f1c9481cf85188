// Global patch matching (eq. 8 candidate grid; Im2Col + matrix product as the
// acceleration of the paper's matching convolution): every key patch against
// every stride-1 image patch, as one contraction
//     d~[g][j] = ||k_g||^2 - 2 <k_g, p_j> + ||p_j||^2
// on MFMA.  The candidate operand is never materialised: a 128-candidate
// tile lies on one row of the top-left grid, so for each (channel, dy) the
// tile's patch rows are one image row segment of 128 + P - 1 values staged in
// LDS, and the MFMA B fragment for (candidate j, dx) is segment[j + dx].
#include "common.h"
#include "internal.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- key matrix
// A[g][d] = x[c][r_g + dy][c_g + dx], d = (c*P + dy)*P + dx;
// kmeta[g] = (||k_g||^2, ||k_g||).  One wave per key; the norm is a per-lane
// strided sum followed by a fixed butterfly (deterministic).
__global__ void k_gather_keys(const float* __restrict__ xp, int H, int W, int P, int D,
                              const int32_t* __restrict__ keys, int N, float* __restrict__ A,
                              float2* __restrict__ kmeta) {
  const int g = blockIdx.x;
  if (g >= N) return;
  const int Wc = W - P + 1;
  const int t = keys[g];
  const int gr = t / Wc, gc = t - gr * Wc;
  float acc = 0.f;
  for (int d = threadIdx.x; d < D; d += 64) {
    int c = d / (P * P);
    int rem = d - c * P * P;
    int dy = rem / P, dx = rem - dy * P;
    float v = xp[((size_t)c * H + gr + dy) * W + gc + dx];
    A[(size_t)g * D + d] = v;
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) kmeta[g] = make_float2(acc, sqrtf(acc));
}

// ---------------------------------------------------------------- candidate norms
// pnorm[j] = ||p_j||^2 summed in d order; prt[j] = sqrt(pnorm[j]).
__global__ void k_cand_norms(const float* __restrict__ xp, int Cp, int H, int W, int P,
                             float* __restrict__ pnorm, float* __restrict__ prt) {
  const int Wc = W - P + 1, Hc = H - P + 1;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Hc * Wc) return;
  int r = j / Wc, c = j - r * Wc;
  float acc = 0.f;
  for (int ch = 0; ch < Cp; ++ch)
    for (int dy = 0; dy < P; ++dy) {
      const float* row = xp + ((size_t)ch * H + r + dy) * W + c;
      for (int dx = 0; dx < P; ++dx) acc += row[dx] * row[dx];
    }
  pnorm[j] = acc;
  prt[j] = sqrtf(acc);
}

// ---------------------------------------------------------------- FP32 MFMA matcher
constexpr int BM = 128;   // keys per block
constexpr int BN = 128;   // candidates per block (one grid-row segment)

// P2 = P rounded up to even (the K=2 step of v_mfma_f32_32x32x2f32).
template <int P2>
__global__ void __launch_bounds__(256)
k_match_f32(const float* __restrict__ xp, int H, int W, int P, int Cp,
            const float* __restrict__ A, int D, const float2* __restrict__ kmeta,
            const float* __restrict__ pnorm, int g0, int nk, float* __restrict__ dist,
            size_t ldd) {
  constexpr int SEG = BN + P2;
  constexpr int AST = P2 + 1;   // odd LDS stride for the key slab
  __shared__ float seg[2][SEG];
  __shared__ float As[2][BM * AST];

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
  const int S = Cp * P;                      // (channel, dy) stages

  // register staging of the next stage
  float rseg = 0.f;
  constexpr int APT = (BM * P2 + 255) / 256;
  float ra[APT];

  auto load_stage = [&](int s) {
    const int ch = s / P, dy = s - ch * P;
    const float* row = xp + ((size_t)ch * H + r + dy) * W;
    if (tid < SEG) {
      int cc = c0 + tid;
      rseg = (cc < W) ? row[cc] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      int e = tid + u * 256;
      float v = 0.f;
      if (e < BM * P2) {
        int m = e / P2, dx = e - m * P2;
        int g = kbase + m;
        if (dx < P && g < nk) v = A[(size_t)(g0 + g) * D + (size_t)s * P + dx];
      }
      ra[u] = v;
    }
  };
  auto store_stage = [&](int buf) {
    if (tid < SEG) seg[buf][tid] = rseg;
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      int e = tid + u * 256;
      if (e < BM * P2) {
        int m = e / P2, dx = e - m * P2;
        As[buf][m * AST + dx] = ra[u];
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
  __syncthreads();
  const int l32 = lane & 31, lhi = lane >> 5;
  for (int s = 0; s < S; ++s) {
    const int cur = s & 1;
    if (s + 1 < S) load_stage(s + 1);
#pragma unroll
    for (int kk = 0; kk < P2 / 2; ++kk) {
      const int dx = 2 * kk + lhi;
      float a0 = As[cur][(wm * 64 + l32) * AST + dx];
      float a1 = As[cur][(wm * 64 + 32 + l32) * AST + dx];
      float b0 = seg[cur][wn * 64 + l32 + dx];
      float b1 = seg[cur][wn * 64 + 32 + l32 + dx];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (s + 1 < S) store_stage(cur ^ 1);
    __syncthreads();
  }

  // epilogue: d~ = (||k||^2 - 2 S) + ||p||^2
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int col = c0 + wn * 64 + nt * 32 + l32;
      const bool cok = col < Wc;
      const size_t t = (size_t)r * Wc + col;
      const float pn = cok ? pnorm[t] : 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = wm * 64 + mt * 32 + 8 * (q >> 2) + 4 * lhi + (q & 3);
        const int g = kbase + i;
        if (cok && g < nk) {
          const float kn = kmeta[g0 + g].x;
          dist[(size_t)g * ldd + t] = (kn - 2.0f * acc[mt][nt][q]) + pn;
        }
      }
    }
}

template <int P2>
void launch_match_t(const glr_plan* pl, const float* xp, const float* A, const float* kmeta,
                    const float* pnorm, int g0, int nk, float* dist, hipStream_t s) {
  const int Hc = pl->Hc, Wc = pl->Wc;
  const int ntc = (Wc + BN - 1) / BN;
  const int nkt = (nk + BM - 1) / BM;
  size_t blocks = (size_t)nkt * Hc * ntc;
  hipLaunchKernelGGL(k_match_f32<P2>, dim3((unsigned)blocks), dim3(256), 0, s, xp, pl->H, pl->W,
                     pl->P, pl->Cp, A, pl->D, (const float2*)kmeta, pnorm, g0, nk, dist,
                     (size_t)pl->ldd);
}

}  // namespace

void launch_gather_keys(const glr_plan* pl, const float* xp, const int32_t* keys, float* A,
                        float* kmeta, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_keys, dim3(pl->N), dim3(64), 0, s, xp, pl->H, pl->W, pl->P, pl->D,
                     keys, pl->N, A, (float2*)kmeta);
}

void launch_cand_norms(const glr_plan* pl, const float* xp, float* pnorm, float* prt,
                       hipStream_t s) {
  int n = pl->Ncand;
  hipLaunchKernelGGL(k_cand_norms, dim3((n + 255) / 256), dim3(256), 0, s, xp, pl->Cp, pl->H,
                     pl->W, pl->P, pnorm, prt);
}

void launch_match_f32(const glr_plan* pl, const float* xp, const float* A, const float* kmeta,
                      const float* pnorm, int g0, int nk, float* dist, hipStream_t s) {
  switch ((pl->P + 1) / 2) {
    case 1: launch_match_t<2>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 2: launch_match_t<4>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 3: launch_match_t<6>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 4: launch_match_t<8>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 5: launch_match_t<10>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 6: launch_match_t<12>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    case 7: launch_match_t<14>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
    default: launch_match_t<16>(pl, xp, A, kmeta, pnorm, g0, nk, dist, s); break;
  }
}
