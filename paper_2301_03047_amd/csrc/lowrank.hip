// Low-rank step: WNNM shrinkage of every patch group (the rank-minimisation
// objective of the Method section, solved by weighted nuclear-norm
// minimisation [Gu et al. 2014]).
//
// One wave per group Y (D x K, column j = member patch j); lane j owns
// column j and keeps it in registers:
//  1. rows are streamed in chunks of up to 64 (each lane loads one row and
//     its mean; Yc = Y - mu 1^T in FP32); the Gram matrix G = Yc^T Yc is
//     accumulated on FP64 MFMA (16 x 16 tiles of its upper triangle) and
//     factored by an FP64 Cholesky, R^T R = G: R is the QR factor of Yc up
//     to row signs;
//  2. one-sided Jacobi on the columns of R^T (odd-even transposition
//     ordering, partner columns moved between lanes by DPP, rotation angles
//     computed in FP64); the converged columns are sigma_i v_i with v_i the
//     right singular vectors of R, hence of Yc, so V is read off them
//     without accumulating rotations;
//  3. WNNM: sigma_hat = sqrt(max(s^2 - K sigma^2, 0)),
//     tau = c sqrt(K) sigma^2 / (sigma_hat + eps), s' = max(s - tau, 0),
//     w = (s - s') / s; for weighted aggregation the group's weight
//     1 / max(r, 1), r the number of s' > 0;
//  4. X = Y - Yc W, W = V diag(w) V^T: the residual sum_i (s_i - s'_i) u_i v_i^T
//     accumulated in FP64 (sigma = 0 gives w = 0, W = 0, X = Y exactly).
// The Gram matrix, its factor, the rotation angles and the residual use
// FP64; the data and the Jacobi iteration FP32.
// The group rows are read from a channel-interleaved copy of the iterate,
// xi[(r*W + c)*Cp + ch], made once per step, and taken in the output order
// e = (dy*P + dx)*Cp + ch (the row order does not change the factorisation):
// one member's patch row over all channels is then one contiguous run, and a
// 64-row chunk of one member is 256 consecutive bytes.
// Estimates are written per member patch in (dy, dx, channel) order:
// xhat[(g*K + j)*D + (dy*P + dx)*Cp + c], staged through LDS.
#include "common.h"
#include "internal.h"

#include <type_traits>

namespace {

constexpr int LS = 65;           // LDS stride (conflict-free column/row access)
constexpr int BR = 64;           // rows per streamed chunk

// xi[(p)*Cp + c] = xp[c*HW + p]: the channel-interleaved copy the group
// loads read (one thread per output element: coalesced writes; the reads of
// a block touch Cp short runs that the next blocks reuse from L2)
__global__ void k_interleave(const float* __restrict__ xp, int Cp, size_t HW,
                             float* __restrict__ xi) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= HW * Cp) return;
  const size_t p = o / Cp;
  const int c = (int)(o - p * Cp);
  xi[o] = xp[(size_t)c * HW + p];
}


// Lane i < nb loads row e = d0+i (output order (dy P + dx) Cp + c) of Y from
// the interleaved copy xi into B[i][0..K) (raw values) and its mean; spos
// holds the members' top-left pixels r W + c.
// Row stride RS (LS by default); with kpad > K the entries K..kpad-1 of a
// row are zeroed.  With tr, the chunk is stored transposed, B[u*RS + i]
// (member-major).
__device__ __forceinline__ void load_rows(const float* __restrict__ xi, const int* spos, int d0,
                                          int nb, int K, int P, int W, int Cp, float* B,
                                          float* smu, int RS = LS, int kpad = 0,
                                          bool tr = false) {
  const int i = threadIdx.x;
  if (i < nb) {
    const int e = d0 + i, pix = e / Cp, c = e - pix * Cp;
    const int dy = pix / P;
    const size_t o = ((size_t)dy * W + (pix - dy * P)) * Cp + c;
    // all of a row's loads in flight at once: the 64 member positions come
    // in 16-byte LDS reads (entries past K repeat the last member; their
    // values are not stored); the sum runs in member order
    int sp[64];
#pragma unroll
    for (int u = 0; u < 64; u += 4) {
      const int4 t = *reinterpret_cast<const int4*>(spos + u);
      sp[u] = t.x; sp[u + 1] = t.y; sp[u + 2] = t.z; sp[u + 3] = t.w;
    }
    float v[64];
#pragma unroll
    for (int u = 0; u < 64; ++u) v[u] = xi[o + (size_t)sp[u] * Cp];
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 64; ++u)
      if (u < K) {
        B[tr ? u * RS + i : i * RS + u] = v[u];
        s += v[u];
      }
    for (int j = K; j < kpad; ++j) B[tr ? j * RS + i : i * RS + j] = 0.f;
    smu[i] = s / (float)K;
  }
  __syncthreads();
}

// FP64 Jacobi rotation annihilating gamma for column norms a1 (first) and a2:
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (a2 - a1) / (2 gamma),
// written with one division; c = 1/sqrt(1 + t^2), s = c t.
// FP64 reciprocal and reciprocal square root from the hardware estimates
// plus one Newton step: the estimates are within about 2^-24 relative
// (largest error over 2^20 inputs spread over 2^-40..2^40 on gfx950), so the
// step leaves an error near 2^-48, far below the FP32 rounding the rotation
// is applied with.
__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return r * fma(-x, r, 2.0);
}
__device__ __forceinline__ double rsq64(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x, r * r, 1.5);
}

// Rotation of the column pair (a, b) with squared norms a1, a2 and inner
// product ga that makes them orthogonal (Hestenes): zeta = (a2 - a1) / (2 ga),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2),
// s = c t; computed in FP64 in the overflow-free form below.  Needs ga != 0.
__device__ __forceinline__ double jacobi_angle(float a1, float a2, float ga, float& c, float& s) {
  const double d = (double)a2 - (double)a1;
  const double g2 = 2.0 * (double)ga;
  const double sg = ((d >= 0.0) == (g2 >= 0.0)) ? 1.0 : -1.0;     // sign(zeta), zeta = 0 -> +1
  const double q = d * d + g2 * g2;
  const double t = sg * fabs(g2) * rcp64(fabs(d) + q * rsq64(q));
  const double cs = rsq64(1.0 + t * t);
  c = (float)cs;
  s = (float)(cs * t);
  return t;
}

// A double held by lane k (uniform k), read as two 32-bit halves.
__device__ __forceinline__ double bcast64(double v, int k) {
  const long long x = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), k);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The value held by lane ^ 1 (a DPP quad permutation: no LDS traffic).
__device__ __forceinline__ float lane_xor1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
}

// The value held by lane src4 / 4 (ds_bpermute: the LDS crossbar moves the
// values, no LDS memory and no VALU work; one instruction where the odd-round
// pattern lane +- 1 would take two DPP shifts and a select).
__device__ __forceinline__ float lane_read(float v, int src4) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src4, __builtin_bit_cast(int, v)));
}

// LDS ordering between lanes of the one wave that runs a group.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


template <int N>
__device__ __forceinline__ void store_vec(float* dst, const float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; i += 4)
    *reinterpret_cast<float4*>(dst + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
}
template <int N>
__device__ __forceinline__ void load_vec(float (&v)[N], const float* src) {
#pragma unroll
  for (int i = 0; i < N; i += 4) {
    const float4 t = *reinterpret_cast<const float4*>(src + i);
    v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
  }
}

template <int KP>
__global__ void __launch_bounds__(64)
k_wnnm(const float* __restrict__ xi, int H, int W, int P, int D, const int32_t* __restrict__ idx,
       int K, float sigma_h, const float* __restrict__ sigp, float wc, float weps,
       int max_sweeps, float* __restrict__ xhat,
       float* __restrict__ sv, DevStats* st, int32_t* __restrict__ zbuf, int zn, int bump,
       float* __restrict__ gw) {
  constexpr int XS = KP + 4;       // row stride of the column-exchange buffer (16-byte rows)
  constexpr int TS = 68;           // row stride of W and of the member-major chunk (64 + 4)
  constexpr int BLN = 64 * (XS > LS ? XS : LS);
  static_assert(KP * TS <= BLN, "W and the member-major chunk fit a buffer");
  static_assert(2 * BLN * 4 >= 64 * 64 * 8, "the Gram matrix fits the two buffers");
  // Rl: R columns (Rl[j*LS + i]); exchange rows; W columns.  Bl: chunk rows
  // (stride XS); then exchange rows and V rows with stride XS.  Both together
  // first hold the FP64 Gram matrix.
  __shared__ __align__(16) float RB[2 * BLN];
  float* const Rl = RB;
  float* const Bl = RB + BLN;
  __shared__ __align__(16) double srow[64];     // one row of the Cholesky factor
  __shared__ float smu[64];
  __shared__ __align__(16) int spos[64];
  __shared__ float sw[64];
  __shared__ float ssig[64];

  const int g = blockIdx.x;
  const int lane = threadIdx.x;
  const int Wc = W - P + 1;
  const int Cp = D / (P * P);
  // side duties of the step, folded in to save launches: clear the
  // aggregation's counters (read only by the kernels after this one) and
  // count the prior step
  for (int i = g * 64 + lane; i < zn; i += gridDim.x * 64) zbuf[i] = 0;
  if (bump && g == 0 && lane == 0) st->steps += 1;

  {
    // lanes past K repeat the last member's position (K <= 64)
    const int t = idx[(size_t)g * K + min(lane, K - 1)];
    const int r = t / Wc, c = t - r * Wc;
    spos[lane] = r * W + c;
  }
  for (int i = 0; i < 64; ++i) Rl[lane * LS + i] = 0.f;
  __syncthreads();

  // ---- 1. Gram matrix G = Yc^T Yc in FP64 over the streamed rows (FP64
  // MFMA on the 16 x 16 tiles of its upper triangle; the FP32 centred values
  // and their products are exact in FP64), then its Cholesky
  // factor R (R^T R = G, upper triangular, column j in lane j; a pivot <= 0,
  // which only a numerically dependent column gives, leaves a zero row).  R
  // equals the QR factor of Yc up to the signs of its rows, so it has the
  // same singular values and right singular vectors.  R is handed to the
  // Jacobi phase in FP32, scaled by the power of two 2^fe that brings its
  // largest entry into [1, 2) (phases 2-3 work on the scaled factor; the
  // singular values are scaled back before the shrinkage, and phase 4 reads
  // the raw rows).
  int fe = 0;
  {
    // FP64 MFMA (16 x 16 x 4): tile (I, J) of G, I <= J, sums four rows per
    // step; lane (m, kq) = (lane % 16, lane / 16) holds row kq of the step
    // for member 16 I + m, the A operand of tile row I and the B operand of
    // tile column I alike, so one LDS read serves every tile of the step
    constexpr int NTI = KP / 16;
    constexpr int NTL = NTI * (NTI + 1) / 2;
    using f64x4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    f64x4 gacc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) gacc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int gm = lane & 15, gk = lane >> 4;
    for (int d0 = 0; d0 < D; d0 += BR) {
      const int nb = min(BR, D - d0);
      const int nb4 = (nb + 3) & ~3;
      // members K..KP-1 of each row are zeros, so the products need no mask
      load_rows(xi, spos, d0, nb, K, P, W, Cp, Bl, smu, XS, KP);
      // centre the chunk in place (lane i: row i), once for all lanes; rows
      // nb..nb4-1 (the last step's rows past the chunk) are zeros
      if (lane < nb) {
        const float mu = smu[lane];
        for (int u = 0; u < K; ++u) Bl[lane * XS + u] -= mu;
      } else if (lane < nb4) {
        for (int u = 0; u < KP; ++u) Bl[lane * XS + u] = 0.f;
      }
      __syncthreads();
      for (int i0 = 0; i0 < nb4; i0 += 4) {
        double v[NTI];
#pragma unroll
        for (int I = 0; I < NTI; ++I) v[I] = (double)Bl[(i0 + gk) * XS + 16 * I + gm];
        int t = 0;
#pragma unroll
        for (int I = 0; I < NTI; ++I)
#pragma unroll
          for (int J = I; J < NTI; ++J, ++t)
            gacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[I], v[J], gacc[t], 0, 0, 0);
      }
      __syncthreads();
    }
    // lane (m, kq) holds G[16 I + kq + 4 i][16 J + m], i < 4; both triangles
    // are stored (entries at or past KP are never read)
    double* G = reinterpret_cast<double*>(RB);
    int t = 0;
#pragma unroll
    for (int I = 0; I < NTI; ++I)
#pragma unroll
      for (int J = I; J < NTI; ++J, ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * I + gk + 4 * i, col = 16 * J + gm;
          G[row * 64 + col] = gacc[t][i];
          if (I != J) G[col * 64 + row] = gacc[t][i];
        }
  }
  __syncthreads();
  {
    const double* G = reinterpret_cast<const double*>(RB);
    double cj[KP];
#pragma unroll
    for (int i = 0; i < KP; ++i) cj[i] = G[i * 64 + lane];
    __syncthreads();                             // RB is rewritten below
    // columns k >= K are zero (G is zero there): their steps change nothing
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const double dkk = bcast64(cj[k], k);
      const double rkk = dkk > 0.0 ? sqrt(dkk) : 0.0;
      const double inv = rkk > 0.0 ? 1.0 / rkk : 0.0;
      cj[k] = lane == k ? rkk : cj[k] * inv;     // row k of R (lanes > k), its pivot
      srow[lane] = cj[k];
      wave_sync();
      // Schur update of the trailing entries; entries below a lane's
      // diagonal are left as they fall and cleared below
#pragma unroll
      for (int i = k + 1; i < KP; ++i) cj[i] = fma(-srow[i], cj[k], cj[i]);
      wave_sync();
    }
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      if (i > lane || lane >= K) cj[i] = 0.0;
      mx = fmax(mx, fabs(cj[i]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (mx > 0.0) {
      int e;
      frexp(mx, &e);                             // mx = f 2^e, f in [0.5, 1)
      fe = max(min(1 - e, 126), -126);
    }
    for (int i = 0; i < 64; ++i) Rl[lane * LS + i] = i < KP ? (float)ldexp(cj[i], fe) : 0.f;
  }
  __syncthreads();

  // ---- 2. one-sided Jacobi on the columns of M = R^T: lane i holds row i of R
  float m[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) m[k] = (lane < K && k < K) ? Rl[k * LS + lane] : 0.f;
  const int Kp = K + (K & 1);
  const float tol = (float)K * 5.9604644775390625e-08f;
  // a sweep whose rotations all had |cos| <= sqrt(tol) / 2 leaves
  // off-diagonal terms of order tol / 4 (cyclic Jacobi converges
  // quadratically), below the threshold: the sweep that would only confirm
  // convergence is skipped
  const float tol_last = 0.5f * sqrtf(tol);
  int sweeps = 0;
  // Each column is held as sc * m: a rotation scales the pair by c and
  // updates m with one FMA per entry (m' = o + f m, f = +-t sc / sc_o); the
  // scale is folded back into m at the start of every sweep (within a sweep
  // it shrinks by at most 2^-Kp/2, far from underflow).
  const float tol2 = tol * tol, tol_last2 = tol_last * tol_last;
  float sc = 1.f;
  int cid = lane;                              // the column of M this lane holds
  for (int swp = 0; swp < max_sweeps; ++swp) {
    bool big = false;
#pragma unroll
    for (int k = 0; k < KP; ++k) m[k] *= sc;
    sc = 1.f;
    // squared column norm, exact at the start of a sweep; within the sweep a
    // rotation updates it in closed form (||a'||^2 = a1 - t g, ||b'||^2 =
    // a2 + t g), which only steers the angles: the singular values are
    // recomputed from the columns at the end
    float al;
    {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int k = 0; k < KP; k += 4) {
        a0 = fmaf(m[k], m[k], a0);
        a1 = fmaf(m[k + 1], m[k + 1], a1);
        a2 = fmaf(m[k + 2], m[k + 2], a2);
        a3 = fmaf(m[k + 3], m[k + 3], a3);
      }
      al = (a0 + a1) + (a2 + a3);
    }
    // odd-even transposition ordering: even rounds pair lanes (2i, 2i+1),
    // odd rounds (2i+1, 2i+2); after its rotation a pair's two columns trade
    // lanes, so in Kp rounds every column passes every other exactly once
    // (the ordering is equivalent to the cyclic one).  Even rounds take the
    // partner column by a DPP quad permutation (lanes at or past Kp hold zero
    // columns that stay zero); odd rounds by ds_bpermute, each unpaired lane
    // reading its own column and keeping it (f = 0: m' = o = m).
    // (an even and an odd round per iteration, so the rotated columns stay
    // in the registers the exchange wrote, with no copy per round)
    auto round = [&](auto oddc) {
      constexpr bool odd = decltype(oddc)::value;
      const int q = odd ? ((lane & 1) ? lane + 1 : lane - 1) : (lane ^ 1);
      const bool paired = lane < Kp && q >= 0 && q < Kp;
      float o[KP];
      float be, osc;
      int ocid;
      if constexpr (odd) {
        const int src4 = (paired ? q : lane) << 2;
#pragma unroll
        for (int k = 0; k < KP; ++k) o[k] = lane_read(m[k], src4);
        be = lane_read(al, src4);
        osc = lane_read(sc, src4);
        ocid = __builtin_bit_cast(int, lane_read(__builtin_bit_cast(float, cid), src4));
      } else {
#pragma unroll
        for (int k = 0; k < KP; ++k) o[k] = lane_xor1(m[k]);
        be = lane_xor1(al);
        osc = lane_xor1(sc);
        ocid = __builtin_bit_cast(int, lane_xor1(__builtin_bit_cast(float, cid)));
      }
      float gp[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < KP; ++k) gp[k & 7] = fmaf(m[k], o[k], gp[k & 7]);
      // same products, order and scales in both lanes of a pair
      const float ga = ((((gp[0] + gp[1]) + (gp[2] + gp[3])) + ((gp[4] + gp[5]) + (gp[6] + gp[7])))) *
                       (sc * osc);
      const bool first = lane < q;
      const float n1 = first ? al : be;          // norm^2 of the lower lane's column
      const float n2 = first ? be : al;
      const float gg = ga * ga, nn = n1 * n2;
      const bool act = paired && ga != 0.f && gg > tol2 * nn;
      // the lower lane takes the other column's update c (b + t a), the upper
      // lane c (a - t b): new m = o + f m, new scale c times the partner's
      float c = 1.f, f = 0.f, tf = 0.f;
      if (act) {
        float s;
        tf = (float)jacobi_angle(n1, n2, ga, c, s);
        f = (first ? tf : -tf) * (sc * __builtin_amdgcn_rcpf(osc));   // rcp within 1 ulp
      }
      if (!odd && !paired) f = 1.f;              // o is 0 here: m stays
#pragma unroll
      for (int k = 0; k < KP; ++k) m[k] = fmaf(f, m[k], o[k]);
      if (paired) {
        // the tracked norm only steers the next angles (FP32 is enough;
        // every sweep starts from the exact norms)
        al = fmaxf(first ? fmaf(tf, ga, n2) : fmaf(-tf, ga, n1), 0.f);
        sc = c * osc;
        cid = ocid;
      }
      big = big || (act && gg > tol_last2 * nn);
    };
    for (int r = 0; r < Kp; r += 2) {
      round(std::false_type{});
      round(std::true_type{});
    }
    sweeps = swp + 1;
    if (__ballot(big) == 0) break;
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) m[k] *= sc;
  __syncthreads();

  // ---- 3. singular values, WNNM factors, V into LDS (V[k][i] = column i / sigma_i)
  // (the noise level comes from the device when an inner iteration estimated it)
  const float sigma = sigp ? sigp[0] : sigma_h;
  float s2a = 0.f, s2b = 0.f;
#pragma unroll
  for (int k = 0; k < KP; k += 2) {
    s2a = fmaf(m[k], m[k], s2a);
    s2b = fmaf(m[k + 1], m[k + 1], s2b);
  }
  const float ss = sqrtf(s2a + s2b);           // singular value of the scaled group
  const float s = ldexpf(ss, -fe);
  // the columns sit in lanes 0..Kp-1 in some order; for odd K one of them
  // is the zero padding column (cid == K), whose w is 0 and which is left
  // out of the singular-value list
  bool kept = false;
  if (lane < Kp) {
    const float shat = sqrtf(fmaxf(s * s - (float)K * sigma * sigma, 0.f));
    const float tau = wc * sqrtf((float)K) * sigma * sigma / (shat + weps);
    const float sn = fmaxf(s - tau, 0.f);
    ssig[lane] = cid < K ? ss : -1.f;
    sw[lane] = s > 0.f ? (s - sn) / s : 0.f;
    kept = cid < K && sn > 0.f;
  }
  // aggregation weight of the group: 1 / max(r, 1), r = singular values kept
  const int rk = __popcll(__ballot(kept));
  if (gw && lane == 0) gw[g] = 1.0f / (float)(rk > 0 ? rk : 1);
  // V rows and columns past K (past Kp) are written as zeros: the products
  // below run over all KP entries, and 0 times stale LDS contents could be NaN
  if (lane < KP) {
    const float inv = (lane < Kp && ss > 0.f) ? 1.0f / ss : 0.f;
#pragma unroll
    for (int k = 0; k < KP; ++k) Bl[k * XS + lane] = (lane < Kp && k < K) ? m[k] * inv : 0.f;
  }
  __syncthreads();
  if (sv && lane < Kp && cid < K) {
    int rank = 0;
    for (int i = 0; i < Kp; ++i) rank += (ssig[i] > ss || (ssig[i] == ss && i < lane)) ? 1 : 0;
    sv[(size_t)g * K + rank] = s;
  }
  if (lane == 0 && st) {
    atomicMax(&st->sweeps_max, sweeps);
    atomicAdd(&st->sweeps_sum, (unsigned long long)sweeps);
  }
  // W[a][b] = sum_i w_i V[a][i] V[b][i]; lane b holds w_i V[b][i] and builds
  // column b of W into Rl[a*TS + b] (W row-major, 16-byte rows of 64)
  {
    float vb[KP];
    load_vec(vb, Bl + lane * XS);
#pragma unroll
    for (int i = 0; i < KP; ++i) vb[i] = (lane < K && i < Kp) ? vb[i] * sw[i] : 0.f;
    if (lane < K)
      for (int a = 0; a < K; ++a) {
        float va[KP];
        load_vec(va, Bl + a * XS);
        float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
        for (int i = 0; i < KP; i += 4) {
          c0 = fmaf(va[i], vb[i], c0);
          c1 = fmaf(va[i + 1], vb[i + 1], c1);
          c2 = fmaf(va[i + 2], vb[i + 2], c2);
          c3 = fmaf(va[i + 3], vb[i + 3], c3);
        }
        Rl[a * TS + lane] = (c0 + c1) + (c2 + c3);
      }
    // rows and columns of W past K are zero
    for (int a = K; a < KP; ++a) Rl[a * TS + lane] = 0.f;
    if (lane >= K)
      for (int a = 0; a < K; ++a) Rl[a * TS + lane] = 0.f;
  }
  __syncthreads();
  {
    double ws = 0.0;
    for (int a = 0; a < K; ++a) ws += (double)Rl[a * TS + lane];
    srow[lane] = ws;                           // column sums of W (FP64)
  }
  __syncthreads();

  // ---- 4. X = Y - Yc W (residual in FP64), per streamed chunk of rows held
  // member-major (Bl[u*TS + i] = Y[i][u]): the product Y W runs on FP64 MFMA
  // (16 x 16 x 4) over 16-row by 16-member tiles, the A operand Y[16 R + m]
  // [a0 + k] and the B operand W[a0 + k][16 C + n] of lane (m or n, k) =
  // (lane % 16, lane / 16) read from LDS; then
  // sum_a (y_a - mu) w_a = sum_a y_a w_a - mu sum_a w_a (FP64; W and the
  // chunk are zero past K) and each lane writes its four rows of a member
  // (rows past nb hold stale values, and only their own outputs, which are
  // not stored)
  {
    constexpr int NTI = KP / 16;
    using f64x4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    const int gm = lane & 15, gk = lane >> 4;
    double wsc[NTI];
#pragma unroll
    for (int C = 0; C < NTI; ++C) wsc[C] = srow[16 * C + gm];
    for (int d0 = 0; d0 < D; d0 += BR) {
      const int nb = min(BR, D - d0);
      load_rows(xi, spos, d0, nb, K, P, W, Cp, Bl, smu, TS, KP, true);
      f64x4 o[4][NTI];
#pragma unroll
      for (int R = 0; R < 4; ++R)
#pragma unroll
        for (int C = 0; C < NTI; ++C) o[R][C] = f64x4{0.0, 0.0, 0.0, 0.0};
      for (int a0 = 0; a0 < KP; a0 += 4) {
        double ya[4], wb[NTI];
#pragma unroll
        for (int R = 0; R < 4; ++R) ya[R] = (double)Bl[(a0 + gk) * TS + 16 * R + gm];
#pragma unroll
        for (int C = 0; C < NTI; ++C) wb[C] = (double)Rl[(a0 + gk) * TS + 16 * C + gm];
#pragma unroll
        for (int R = 0; R < 4; ++R)
#pragma unroll
          for (int C = 0; C < NTI; ++C)
            o[R][C] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[R], wb[C], o[R][C], 0, 0, 0);
      }
      // lane (n, k) holds rows 16 R + k + 4 i of member 16 C + n, i < 4
#pragma unroll
      for (int C = 0; C < NTI; ++C) {
        const int j = 16 * C + gm;
        if (j >= K) continue;
        float* outp = xhat + ((size_t)g * K + j) * D + d0;
#pragma unroll
        for (int R = 0; R < 4; ++R)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * R + gk + 4 * i;
            const double r = o[R][C][i] - (double)smu[row] * wsc[C];
            if (row < nb) outp[row] = (float)((double)Bl[j * TS + row] - r);
          }
      }
      __syncthreads();
    }
  }
}

// Complex-Hermitian form for complex data.  The interleaved image holds Re
// and Im of a pixel as channels 0 and 1, so rows 2t and 2t+1 of the real
// group are Re and Im of row t of the complex group Z (P^2 x K, t = dy P + dx,
// D = 2 P^2).  The steps of k_wnnm in complex arithmetic:
//  1. G = Zc^H Zc in FP64: Re G is the Gram matrix of the real rows (first
//     pass over the rows), Im G[a][b] = sum_t (Re z_a Im z_b - Im z_a Re z_b)
//     pairs each row with its partner row (second pass); the Cholesky factor
//     R^H R = G is upper triangular with a real diagonal (rank-deficient G,
//     K > P^2, leaves zero or rounding-sized rows);
//  2. one-sided Jacobi on the columns of M = R^H (lane i holds the conjugate
//     of row i of R): for a pair (a, b) with a^H b = |g| e^{i phi}, b turned
//     by e^{-i phi} has a real inner product with a and the real rotation
//     applies; the lower lane takes c (b + t e^{i phi} a), the upper
//     c (a - t e^{-i phi} b).  The converged columns are sigma_i v_i with v_i
//     the right singular vectors of R, hence of Zc;
//  3. the WNNM factors of the real form (K the member count), and
//     W = V diag(w) V^H (Hermitian);
//  4. X = Z - Zc W in complex FP64.
template <int KP>
__global__ void __launch_bounds__(64)
k_wnnm_cplx(const float* __restrict__ xi, int H, int W, int P, int D,
            const int32_t* __restrict__ idx, int K, float sigma_h, const float* __restrict__ sigp,
            float wc, float weps, int max_sweeps, float* __restrict__ xhat,
            float* __restrict__ sv, DevStats* st, int32_t* __restrict__ zbuf, int zn, int bump,
            float* __restrict__ gw) {
  constexpr int XS = KP + 4;       // row stride of the streamed chunk and of V
  constexpr int TS = 68;           // row stride of W and of the member-major chunk
  constexpr int CH = 64 * XS;      // the chunk (64 rows), phase 1
  constexpr int NG = 4 * KP * KP;  // Re G and Im G in FP64, phase 1
  constexpr int NV = 2 * KP * XS;  // Re V and Im V, then the member-major chunk
  constexpr int NW = 2 * KP * TS;  // Re W and Im W
  constexpr int NR = 2 * KP * LS;  // Re R and Im R columns
  constexpr int N1 = CH + NG > NV + NW ? CH + NG : NV + NW;
  constexpr int NB = N1 > NR ? N1 : NR;
  static_assert(KP * TS <= NV, "the member-major chunk fits the V buffer");
  static_assert(KP % 8 == 0, "8 x 8 blocks");
  __shared__ __align__(16) float RB[NB];
  __shared__ __align__(16) double srr[64];      // a row of R; the column sums of W
  __shared__ __align__(16) double sri[64];
  __shared__ float smu[64];
  __shared__ __align__(16) int spos[64];
  __shared__ float sw[64];
  __shared__ float ssig[64];
  float* const Bl = RB;
  double* const Gr = reinterpret_cast<double*>(RB + CH);
  double* const Gi = Gr + KP * KP;
  float* const Rr = RB;
  float* const Ri = RB + KP * LS;
  float* const Vr = RB;
  float* const Vi = RB + KP * XS;
  float* const Wr = RB + NV;
  float* const Wi = RB + NV + KP * TS;

  const int g = blockIdx.x;
  const int lane = threadIdx.x;
  const int Wc = W - P + 1;
  for (int i = g * 64 + lane; i < zn; i += gridDim.x * 64) zbuf[i] = 0;
  if (bump && g == 0 && lane == 0) st->steps += 1;
  {
    const int t = idx[(size_t)g * K + min(lane, K - 1)];
    const int r = t / Wc, c = t - r * Wc;
    spos[lane] = r * W + c;
  }
  __syncthreads();

  // ---- 1. G = Zc^H Zc (lane (bi, bj): the 8 x 8 block at 8 bi, 8 bj)
  int fe = 0;
  {
    const int bi = lane >> 3, bj = lane & 7;
    for (int pass = 0; pass < 2; ++pass) {
      double acc[8][8];
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[p][q] = 0.0;
      for (int d0 = 0; d0 < D; d0 += BR) {
        const int nb = min(BR, D - d0);              // even: D is, and BR
        // members K..KP-1 are zeros (no masks below); blocks at or past KP
        // read other rows' values, and their entries of G are not stored
        load_rows(xi, spos, d0, nb, K, P, W, 2, Bl, smu, XS, KP);
        if (lane < nb) {
          const float mu = smu[lane];
          for (int u = 0; u < K; ++u) Bl[lane * XS + u] -= mu;
        }
        __syncthreads();
#pragma unroll 2
        for (int i = 0; i < nb; ++i) {
          // Re G: row with itself; Im G: a Re row times its Im row, an Im row
          // times minus its Re row
          const int ib = pass ? (i ^ 1) : i;
          const double sg = (pass && (i & 1)) ? -1.0 : 1.0;
          float a[8], b[8];
          load_vec(a, Bl + i * XS + 8 * bi);
          load_vec(b, Bl + ib * XS + 8 * bj);
          double ya[8], yb[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            ya[t] = (double)a[t];
            yb[t] = sg * (double)b[t];
          }
#pragma unroll
          for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[p][q] = fma(ya[p], yb[q], acc[p][q]);
        }
        __syncthreads();
      }
      double* G = pass ? Gi : Gr;
      if (8 * bi < KP && 8 * bj < KP) {
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
          for (int q = 0; q < 8; ++q) G[(8 * bi + p) * KP + 8 * bj + q] = acc[p][q];
      }
    }
  }
  __syncthreads();
  {
    // lane j: column j of G, then of R (R[k][j] = conj(R[k][j]) of M's row)
    double cr[KP], ci[KP];
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      cr[i] = lane < KP ? Gr[i * KP + lane] : 0.0;
      ci[i] = lane < KP ? Gi[i * KP + lane] : 0.0;
    }
    __syncthreads();                             // RB is rewritten below
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const double dkk = bcast64(cr[k], k);      // the pivot is real
      const double rkk = dkk > 0.0 ? sqrt(dkk) : 0.0;
      const double inv = rkk > 0.0 ? 1.0 / rkk : 0.0;
      cr[k] = lane == k ? rkk : cr[k] * inv;
      ci[k] = lane == k ? 0.0 : ci[k] * inv;
      srr[lane] = cr[k];
      sri[lane] = ci[k];
      wave_sync();
      // G'[i][j] -= conj(R[k][i]) R[k][j]
#pragma unroll
      for (int i = k + 1; i < KP; ++i) {
        const double ar = srr[i], ai = sri[i];
        cr[i] = fma(-ar, cr[k], fma(-ai, ci[k], cr[i]));
        ci[i] = fma(-ar, ci[k], fma(ai, cr[k], ci[i]));
      }
      wave_sync();
    }
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      if (i > lane || lane >= K) {
        cr[i] = 0.0;
        ci[i] = 0.0;
      }
      mx = fmax(mx, fmax(fabs(cr[i]), fabs(ci[i])));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (mx > 0.0) {
      int e;
      frexp(mx, &e);
      fe = max(min(1 - e, 126), -126);
    }
    if (lane < KP)
      for (int i = 0; i < KP; ++i) {
        Rr[lane * LS + i] = (float)ldexp(cr[i], fe);
        Ri[lane * LS + i] = (float)ldexp(ci[i], fe);
      }
  }
  __syncthreads();

  // ---- 2. one-sided Jacobi on the columns of M = R^H
  float mr[KP], mi[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const bool in = lane < K && k < K;
    mr[k] = in ? Rr[k * LS + lane] : 0.f;
    mi[k] = in ? -Ri[k * LS + lane] : 0.f;
  }
  const int Kp = K + (K & 1);
  const float tol = (float)K * 5.9604644775390625e-08f;
  const float tol_last = 0.5f * sqrtf(tol);
  const float tol2 = tol * tol, tol_last2 = tol_last * tol_last;
  int sweeps = 0;
  float sc = 1.f;
  int cid = lane;
  for (int swp = 0; swp < max_sweeps; ++swp) {
    bool big = false;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      mr[k] *= sc;
      mi[k] *= sc;
    }
    sc = 1.f;
    float al;
    {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int k = 0; k < KP; k += 2) {
        a0 = fmaf(mr[k], mr[k], a0);
        a1 = fmaf(mi[k], mi[k], a1);
        a2 = fmaf(mr[k + 1], mr[k + 1], a2);
        a3 = fmaf(mi[k + 1], mi[k + 1], a3);
      }
      al = (a0 + a1) + (a2 + a3);
    }
    auto round = [&](auto oddc) {
      constexpr bool odd = decltype(oddc)::value;
      const int q = odd ? ((lane & 1) ? lane + 1 : lane - 1) : (lane ^ 1);
      const bool paired = lane < Kp && q >= 0 && q < Kp;
      float orr[KP], oi[KP];
      float be, osc;
      int ocid;
      if constexpr (odd) {
        const int src4 = (paired ? q : lane) << 2;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          orr[k] = lane_read(mr[k], src4);
          oi[k] = lane_read(mi[k], src4);
        }
        be = lane_read(al, src4);
        osc = lane_read(sc, src4);
        ocid = __builtin_bit_cast(int, lane_read(__builtin_bit_cast(float, cid), src4));
      } else {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          orr[k] = lane_xor1(mr[k]);
          oi[k] = lane_xor1(mi[k]);
        }
        be = lane_xor1(al);
        osc = lane_xor1(sc);
        ocid = __builtin_bit_cast(int, lane_xor1(__builtin_bit_cast(float, cid)));
      }
      // Re(m^H o) is symmetric in the pair; the two cross sums trade places
      // between the lanes, so both lanes form Im(a^H b) (a the lower lane's
      // column) from the same products in the same order
      float gp[4] = {0.f, 0.f, 0.f, 0.f}, s1p[4] = {0.f, 0.f, 0.f, 0.f},
            s2p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        gp[k & 3] = fmaf(mr[k], orr[k], gp[k & 3]);
        gp[k & 3] = fmaf(mi[k], oi[k], gp[k & 3]);
        s1p[k & 3] = fmaf(mr[k], oi[k], s1p[k & 3]);
        s2p[k & 3] = fmaf(mi[k], orr[k], s2p[k & 3]);
      }
      const bool first = lane < q;
      const float scl = sc * osc;
      const float gr = ((gp[0] + gp[1]) + (gp[2] + gp[3])) * scl;
      const float s1 = (s1p[0] + s1p[1]) + (s1p[2] + s1p[3]);
      const float s2 = (s2p[0] + s2p[1]) + (s2p[2] + s2p[3]);
      const float gi = (first ? s1 - s2 : s2 - s1) * scl;
      const float n1 = first ? al : be;
      const float n2 = first ? be : al;
      const float gg = fmaf(gr, gr, gi * gi), nn = n1 * n2;
      const bool act = paired && gg > tol2 * nn && gg > 0.f;
      float c = 1.f, fr = 0.f, fi = 0.f, tf = 0.f, ga = 0.f;
      if (act) {
        const double gd = sqrt((double)gr * gr + (double)gi * gi);
        ga = (float)gd;
        float sn;
        tf = (float)jacobi_angle(n1, n2, ga, c, sn);
        const float ig = (float)(1.0 / gd);
        const float ratio = sc * __builtin_amdgcn_rcpf(osc);
        fr = (first ? tf : -tf) * (gr * ig) * ratio;
        fi = tf * (gi * ig) * ratio;
      }
      if (!odd && !paired) fr = 1.f;            // even rounds: o is 0 here, m stays
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const float xr = mr[k], xm = mi[k];
        mr[k] = fmaf(fr, xr, fmaf(-fi, xm, orr[k]));
        mi[k] = fmaf(fr, xm, fmaf(fi, xr, oi[k]));
      }
      if (paired) {
        al = fmaxf(first ? fmaf(tf, ga, n2) : fmaf(-tf, ga, n1), 0.f);
        sc = c * osc;
        cid = ocid;
      }
      big = big || (act && gg > tol_last2 * nn);
    };
    for (int r = 0; r < Kp; r += 2) {
      round(std::false_type{});
      round(std::true_type{});
    }
    sweeps = swp + 1;
    if (__ballot(big) == 0) break;
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    mr[k] *= sc;
    mi[k] *= sc;
  }
  __syncthreads();

  // ---- 3. singular values, WNNM factors, V (V[k][i] = column i / sigma_i)
  const float sigma = sigp ? sigp[0] : sigma_h;
  float s2a = 0.f, s2b = 0.f;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    s2a = fmaf(mr[k], mr[k], s2a);
    s2b = fmaf(mi[k], mi[k], s2b);
  }
  const float ss = sqrtf(s2a + s2b);
  const float s = ldexpf(ss, -fe);
  bool kept = false;
  if (lane < Kp) {
    const float shat = sqrtf(fmaxf(s * s - (float)K * sigma * sigma, 0.f));
    const float tau = wc * sqrtf((float)K) * sigma * sigma / (shat + weps);
    const float sn = fmaxf(s - tau, 0.f);
    ssig[lane] = cid < K ? ss : -1.f;
    sw[lane] = s > 0.f ? (s - sn) / s : 0.f;
    kept = cid < K && sn > 0.f;
  }
  const int rk = __popcll(__ballot(kept));
  if (gw && lane == 0) gw[g] = 1.0f / (float)(rk > 0 ? rk : 1);
  if (lane < KP) {
    const float inv = (lane < Kp && ss > 0.f) ? 1.0f / ss : 0.f;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const bool in = lane < Kp && k < K;
      Vr[k * XS + lane] = in ? mr[k] * inv : 0.f;
      Vi[k * XS + lane] = in ? mi[k] * inv : 0.f;
    }
  }
  __syncthreads();
  if (sv && lane < Kp && cid < K) {
    int rank = 0;
    for (int i = 0; i < Kp; ++i) rank += (ssig[i] > ss || (ssig[i] == ss && i < lane)) ? 1 : 0;
    sv[(size_t)g * K + rank] = s;
  }
  if (lane == 0 && st) {
    atomicMax(&st->sweeps_max, sweeps);
    atomicAdd(&st->sweeps_sum, (unsigned long long)sweeps);
  }
  // W[a][b] = sum_i w_i V[a][i] conj(V[b][i]); lane b holds w_i conj(V[b][i])
  {
    const int b = min(lane, KP - 1);
    float vbr[KP], vbi[KP];
    load_vec(vbr, Vr + b * XS);
    load_vec(vbi, Vi + b * XS);
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      const float w = (lane < K && i < Kp) ? sw[i] : 0.f;
      vbr[i] *= w;
      vbi[i] *= -w;
    }
    if (lane < K)
      for (int a = 0; a < K; ++a) {
        float var[KP], vai[KP];
        load_vec(var, Vr + a * XS);
        load_vec(vai, Vi + a * XS);
        float r0 = 0.f, r1 = 0.f, i0 = 0.f, i1 = 0.f;
#pragma unroll
        for (int i = 0; i < KP; i += 2) {
          r0 = fmaf(var[i], vbr[i], fmaf(-vai[i], vbi[i], r0));
          r1 = fmaf(var[i + 1], vbr[i + 1], fmaf(-vai[i + 1], vbi[i + 1], r1));
          i0 = fmaf(var[i], vbi[i], fmaf(vai[i], vbr[i], i0));
          i1 = fmaf(var[i + 1], vbi[i + 1], fmaf(vai[i + 1], vbr[i + 1], i1));
        }
        Wr[a * TS + lane] = r0 + r1;
        Wi[a * TS + lane] = i0 + i1;
      }
    for (int a = K; a < KP; ++a) {
      Wr[a * TS + lane] = 0.f;
      Wi[a * TS + lane] = 0.f;
    }
    if (lane >= K)
      for (int a = 0; a < K; ++a) {
        Wr[a * TS + lane] = 0.f;
        Wi[a * TS + lane] = 0.f;
      }
  }
  __syncthreads();
  {
    double a0 = 0.0, a1 = 0.0;
    for (int a = 0; a < K; ++a) {
      a0 += (double)Wr[a * TS + lane];
      a1 += (double)Wi[a * TS + lane];
    }
    srr[lane] = a0;
    sri[lane] = a1;
  }
  __syncthreads();

  // ---- 4. X = Z - Zc W per streamed chunk, member-major (Bl[u*TS + i]):
  // lane (bi, bj) computes real rows 8 bi .. (complex rows 4 bi ..) of
  // members 8 bj .., with sum_a (z_a - mu) W_a = sum_a z_a W_a - mu sum_a W_a
  {
    const int bi = lane >> 3, bj = lane & 7;
    double wsr[8], wsi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      wsr[q] = srr[8 * bj + q];
      wsi[q] = sri[8 * bj + q];
    }
    for (int d0 = 0; d0 < D; d0 += BR) {
      const int nb = min(BR, D - d0);
      load_rows(xi, spos, d0, nb, K, P, W, 2, Bl, smu, TS, KP, true);
      double acc[8][8];
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[p][q] = 0.0;
#pragma unroll 2
      for (int a = 0; a < KP; ++a) {
        float yv[8], wr[8], wi[8];
        load_vec(yv, Bl + a * TS + 8 * bi);
        load_vec(wr, Wr + a * TS + 8 * bj);
        load_vec(wi, Wi + a * TS + 8 * bj);
        double wrd[8], wid[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          wrd[q] = (double)wr[q];
          wid[q] = (double)wi[q];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double yr = (double)yv[2 * t], yi = (double)yv[2 * t + 1];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            acc[2 * t][q] = fma(yr, wrd[q], fma(-yi, wid[q], acc[2 * t][q]));
            acc[2 * t + 1][q] = fma(yr, wid[q], fma(yi, wrd[q], acc[2 * t + 1][q]));
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = 8 * bj + q;
        if (j >= K) continue;
        float* outp = xhat + ((size_t)g * K + j) * D + d0;
        float yv[8];
        load_vec(yv, Bl + j * TS + 8 * bi);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = 8 * bi + 2 * t;
          const double mur = (double)smu[i], mui = (double)smu[i + 1];
          const double rr = acc[2 * t][q] - (mur * wsr[q] - mui * wsi[q]);
          const double ri = acc[2 * t + 1][q] - (mur * wsi[q] + mui * wsr[q]);
          if (i < nb) {
            outp[i] = (float)((double)yv[2 * t] - rr);
            outp[i + 1] = (float)((double)yv[2 * t + 1] - ri);
          }
        }
      }
      __syncthreads();
    }
  }
}

// Iterative regularisation between inner WNNM iterations:
// y_new = x + delta (xbar - y_prev) elementwise (FP32), and per block the
// FP64 sum of (xbar - y_new)^2 in a fixed order (grid-stride per thread,
// then a fixed tree over the block).
constexpr int IB = 256, IG = 1024;     // threads per block, blocks (fixed: the sum's order)
__global__ void __launch_bounds__(IB)
k_inner_update(const float* __restrict__ xbar, const float* __restrict__ x,
               const float* yprev, float* ynew, size_t n, float delta,
               double* __restrict__ part) {
  __shared__ double red[IB];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * IB + threadIdx.x; i < n; i += (size_t)IG * IB) {
    const float xb = xbar[i];
    const float y = fmaf(delta, xb - yprev[i], x[i]);
    ynew[i] = y;
    const double d = (double)xb - (double)y;
    acc = fma(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = IB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// sigma_k = lambda sqrt(max(sigma^2 - S / n, 0)), S the sum of the partials
__global__ void __launch_bounds__(IG)
k_inner_sigma(const double* __restrict__ part, size_t n, float sigma, float lambda,
              float* __restrict__ sig_out) {
  __shared__ double red[IG];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int h = IG / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double s2 = (double)sigma * (double)sigma - red[0] / (double)n;
    sig_out[0] = (float)((double)lambda * sqrt(s2 > 0.0 ? s2 : 0.0));
  }
}

}  // namespace

void launch_inner_update(const float* xbar, const float* x, const float* yprev, float* ynew,
                         size_t n, float delta, float sigma, float lambda, double* part,
                         float* sig_out, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_update, dim3(IG), dim3(IB), 0, s, xbar, x, yprev, ynew, n, delta,
                     part);
  hipLaunchKernelGGL(k_inner_sigma, dim3(1), dim3(IG), 0, s, part, n, sigma, lambda, sig_out);
}

void launch_interleave(const glr_plan* pl, const float* xp, float* xi, hipStream_t s) {
  const size_t HW = (size_t)pl->H * pl->W, n = HW * pl->Cp;
  hipLaunchKernelGGL(k_interleave, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xp, pl->Cp,
                     HW, xi);
}

void launch_wnnm(const glr_plan* pl, const float* xi, const int32_t* idx, float sigma,
                 float* xhat, float* sv, DevStats* st, int32_t* zbuf, int zn, int bump,
                 float* gw, const float* sigp, hipStream_t s) {
  const int K = pl->K;
  if (pl->lowrank_complex) {
    auto kern = K <= 32 ? k_wnnm_cplx<32> : K <= 48 ? k_wnnm_cplx<48> : k_wnnm_cplx<64>;
    hipLaunchKernelGGL(kern, dim3(pl->N), dim3(64), 0, s, xi, pl->H, pl->W, pl->P, pl->D, idx, K,
                       sigma, sigp, pl->wnnm_c, pl->wnnm_eps, 30, xhat, sv, st, zbuf, zn, bump,
                       gw);
    return;
  }
  if (K <= 32)
    hipLaunchKernelGGL(k_wnnm<32>, dim3(pl->N), dim3(64), 0, s, xi, pl->H, pl->W, pl->P, pl->D,
                       idx, K, sigma, sigp, pl->wnnm_c, pl->wnnm_eps, 30, xhat, sv, st, zbuf, zn, bump,
                       gw);
  else if (K <= 48)
    hipLaunchKernelGGL(k_wnnm<48>, dim3(pl->N), dim3(64), 0, s, xi, pl->H, pl->W, pl->P, pl->D,
                       idx, K, sigma, sigp, pl->wnnm_c, pl->wnnm_eps, 30, xhat, sv, st, zbuf, zn, bump,
                       gw);
  else
    hipLaunchKernelGGL(k_wnnm<64>, dim3(pl->N), dim3(64), 0, s, xi, pl->H, pl->W, pl->P, pl->D,
                       idx, K, sigma, sigp, pl->wnnm_c, pl->wnnm_eps, 30, xhat, sv, st, zbuf, zn, bump,
                       gw);
}
