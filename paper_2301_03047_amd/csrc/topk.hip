// Top-K grouping (eq. 1 with KNN grouping, searched over the whole image).
//
// The matcher's d~ carries a rounding error bounded by
//     eps_j = coef * (||k|| + ||p_j||)^2,   coef = 2 (D + 8) 2^-24
// (dot product and norms in FP32, plus the epilogue roundings, with a safety
// factor of two).  With U_j = d~_j + eps_j and L_j = d~_j - eps_j, let T be
// the K-th smallest U_j of a key: every member of the exact top-K has
// L_j <= d_j <= T, so the margin set {j : L_j <= T} contains the exact
// answer.  Stage 1 finds, per (key, candidate range), the range's margin set
// against the range's own T (an upper bound of the key's T) in one streaming
// pass; stage 2 merges the ranges, applies the key's T, recomputes the
// distance of each margin member with compensated (double-float32)
// arithmetic and sorts by (distance, position), lowest position winning ties.
#include "common.h"
#include "internal.h"

namespace {

constexpr int CAP = GLR_SPLIT_CAP;        // entries per wave buffer
constexpr int UCAP = GLR_UNION_CAP;       // entries per key in stage 2

// K-th smallest of vals[0..n) (as ordered uint32) by bisection over the
// value range; one wave.  Requires n >= K >= 1.
__device__ float wave_kth_smallest(const float* vals, int n, int K) {
  uint32_t lo = 0u, hi = 0xffffffffu;
  const int l = lane_id();
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    int c = 0;
    for (int i = l; i < n; i += 64) c += (f2ord(vals[i]) <= mid) ? 1 : 0;
    c = wave_sum_i32(c);
    if (c >= K) hi = mid; else lo = mid + 1;
  }
  return ord2f(lo);
}

// keep entries with L <= T (ordered, in place); returns the new count
__device__ int wave_compact(int* bj, float* bu, float* bl, int n, float T) {
  int w = 0;
  const int l = lane_id();
  for (int base = 0; base < n; base += 64) {
    int i = base + l;
    bool in = i < n;
    int j = in ? bj[i] : 0;
    float u = in ? bu[i] : 0.f;
    float lo = in ? bl[i] : 0.f;
    bool keep = in && (lo <= T);
    uint64_t m = __ballot(keep);
    int pos = w + lanes_below(m);
    // all lanes have read their entry before any write (lockstep wave)
    if (keep) {
      bj[pos] = j;
      bu[pos] = u;
      bl[pos] = lo;
    }
    w += __popcll(m);
  }
  return w;
}

__global__ void __launch_bounds__(256)
k_topk_partial(const float* __restrict__ dist, size_t ldd, const float2* __restrict__ kmeta, int g0,
               const float* __restrict__ prt, int Ncand, int split_len, int S, int nk, int K,
               float coef, int32_t* __restrict__ lj, float* __restrict__ lu, float* __restrict__ ll,
               int32_t* __restrict__ lcnt) {
  __shared__ int sbj[4][CAP];
  __shared__ float sbu[4][CAP];
  __shared__ float sbl[4][CAP];
  const int wave = threadIdx.x >> 6;
  const int l = lane_id();
  const int item = blockIdx.x * 4 + wave;
  if (item >= nk * S) return;               // wave-uniform; no block barriers below
  int* bj = sbj[wave];
  float* bu = sbu[wave];
  float* bl = sbl[wave];
  const int g = item / S, sp = item - g * S;
  const int j0 = sp * split_len;
  const int j1 = min(Ncand, j0 + split_len);
  const float kr = kmeta[g0 + g].y;
  const float* drow = dist + (size_t)g * ldd;
  float T = __int_as_float(0x7f800000);     // +inf
  int cnt = 0;
  bool ovf = false;
  for (int base = j0; base < j1; base += 256) {
    const int j = base + 4 * l;
    float dv[4], pv[4];
    if (j + 3 < j1) {
      float4 a = *reinterpret_cast<const float4*>(drow + j);
      float4 b = *reinterpret_cast<const float4*>(prt + j);
      dv[0] = a.x; dv[1] = a.y; dv[2] = a.z; dv[3] = a.w;
      pv[0] = b.x; pv[1] = b.y; pv[2] = b.z; pv[3] = b.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bool ok = j + e < j1;
        dv[e] = ok ? drow[j + e] : 0.f;
        pv[e] = ok ? prt[j + e] : 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float s = kr + pv[e];
      const float eps = coef * (s * s);
      const float U = dv[e] + eps;
      const float L = dv[e] - eps;
      const bool adm = (j + e < j1) && (L <= T);
      uint64_t m = __ballot(adm);
      if (adm) {
        int pos = cnt + lanes_below(m);
        bj[pos] = j + e;
        bu[pos] = U;
        bl[pos] = L;
      }
      cnt += __popcll(m);
    }
    if (cnt > CAP - 256) {
      float Tn = wave_kth_smallest(bu, cnt, K);
      T = fminf(T, Tn);
      cnt = wave_compact(bj, bu, bl, cnt, T);
      if (cnt > CAP - 256) {
        ovf = true;
        break;
      }
    }
  }
  if (!ovf && cnt >= K) {
    float Tn = wave_kth_smallest(bu, cnt, K);
    T = fminf(T, Tn);
    cnt = wave_compact(bj, bu, bl, cnt, T);
  }
  const size_t o = (size_t)item * CAP;
  if (!ovf)
    for (int i = l; i < cnt; i += 64) {
      lj[o + i] = bj[i];
      lu[o + i] = bu[i];
      ll[o + i] = bl[i];
    }
  if (l == 0) lcnt[item] = ovf ? -1 : cnt;
}

// ---------------------------------------------------------------- stage 2
constexpr int ST = 256;

__device__ int block_sum_i(int v, int* sh) {
  v = wave_sum_i32(v);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < ST / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// exact (compensated) squared distance between key g's vector and patch j
__device__ __forceinline__ df32 exact_dist(const float* __restrict__ xp, int H, int W, int P, int Cp,
                                           const float* __restrict__ kvec, int j, int Wc) {
  const int r = j / Wc, c = j - r * Wc;
  df32 acc = {0.f, 0.f};
  int d = 0;
  for (int ch = 0; ch < Cp; ++ch)
    for (int dy = 0; dy < P; ++dy) {
      const float* row = xp + ((size_t)ch * H + r + dy) * W + c;
      for (int dx = 0; dx < P; ++dx, ++d) df_add_sqdiff(acc, kvec[d], row[dx]);
    }
  return acc;
}

// bitonic sort of n (power of two) entries by (hi, lo, j) ascending
__device__ void block_bitonic(float* h, float* lo, int* j, int n) {
  for (int k = 2; k <= n; k <<= 1)
    for (int s = k >> 1; s > 0; s >>= 1) {
      for (int i = threadIdx.x; i < n; i += ST) {
        int p = i ^ s;
        if (p > i) {
          bool up = (i & k) == 0;
          bool gt = df_less(h[p], lo[p], j[p], h[i], lo[i], j[i]);   // a[i] > a[p]
          if (gt == up) {
            float th = h[i], tl = lo[i];
            int tj = j[i];
            h[i] = h[p]; lo[i] = lo[p]; j[i] = j[p];
            h[p] = th; lo[p] = tl; j[p] = tj;
          }
        }
      }
      __syncthreads();
    }
}

__global__ void __launch_bounds__(ST)
k_select_rescore(const float* __restrict__ xp, int H, int W, int P, int Cp, int D,
                 const float* __restrict__ A, int g0, int S, int Ncand, int K,
                 const int32_t* __restrict__ lj, const float* __restrict__ lu,
                 const float* __restrict__ ll, const int32_t* __restrict__ lcnt,
                 int32_t* __restrict__ idx, float* __restrict__ dd, DevStats* st) {
  __shared__ float su[UCAP];
  __shared__ float sl[UCAP];
  __shared__ int sj[UCAP];
  __shared__ int soff[65];
  __shared__ int ssh[ST / 64 + 1];
  __shared__ int sflag;
  const int g = blockIdx.x;
  const int gg = g0 + g;
  const int tid = threadIdx.x;
  const int Wc = W - P + 1;
  const float* kvec = A + (size_t)gg * D;

  if (tid == 0) {
    int tot = 0, ovf = 0;
    for (int sp = 0; sp < S; ++sp) {
      int c = lcnt[g * S + sp];
      soff[sp] = tot;
      if (c < 0) ovf = 1; else tot += c;
    }
    soff[S] = tot;
    sflag = (ovf || tot > UCAP) ? 1 : 0;
  }
  __syncthreads();
  const bool overflow = sflag != 0;
  int m = 0;
  if (!overflow) {
    const int tot = soff[S];
    for (int sp = 0; sp < S; ++sp) {
      const int c = soff[sp + 1] - soff[sp];
      const size_t o = ((size_t)g * S + sp) * CAP;
      for (int i = tid; i < c; i += ST) {
        su[soff[sp] + i] = lu[o + i];
        sl[soff[sp] + i] = ll[o + i];
        sj[soff[sp] + i] = lj[o + i];
      }
    }
    __syncthreads();
    // key threshold T = K-th smallest U of the union
    uint32_t lo = 0u, hi = 0xffffffffu;
    while (lo < hi) {
      uint32_t mid = lo + ((hi - lo) >> 1);
      int c = 0;
      for (int i = tid; i < tot; i += ST) c += (f2ord(su[i]) <= mid) ? 1 : 0;
      c = block_sum_i(c, ssh);
      if (c >= K) hi = mid; else lo = mid + 1;
    }
    const float T = ord2f(lo);
    // margin set, ordered compaction into the front of the arrays
    for (int base = 0; base < tot; base += ST) {
      int i = base + tid;
      bool keep = i < tot && sl[i] <= T;
      int jj = keep ? sj[i] : 0;
      int tc;
      int pre = block_excl_scan(keep ? 1 : 0, ssh, &tc);
      if (keep) sj[m + pre] = jj;            // pre + m <= i: never ahead of unread entries
      m += tc;
    }
    __syncthreads();
    // compensated rescoring of the margin set
    for (int i = tid; i < m; i += ST) {
      df32 v = exact_dist(xp, H, W, P, Cp, kvec, sj[i], Wc);
      su[i] = v.hi;
      sl[i] = v.lo;
    }
    int n2 = 1;
    while (n2 < m) n2 <<= 1;
    for (int i = m + tid; i < n2; i += ST) {
      su[i] = __int_as_float(0x7f800000);
      sl[i] = 0.f;
      sj[i] = 0x7fffffff;
    }
    __syncthreads();
    block_bitonic(su, sl, sj, n2);
    for (int q = tid; q < K; q += ST) {
      idx[(size_t)gg * K + q] = sj[q];
      dd[(size_t)gg * K + q] = su[q];
    }
  } else {
    // exact scan of the whole row: keep a running best list
    const int BEST = UCAP;
    int cur = 0;
    float th = __int_as_float(0x7f800000), tl = 0.f;
    int tj = 0x7fffffff;
    for (int base = 0; base < Ncand; base += ST) {
      int j = base + tid;
      df32 v = {0.f, 0.f};
      bool adm = false;
      if (j < Ncand) {
        v = exact_dist(xp, H, W, P, Cp, kvec, j, Wc);
        adm = df_less(v.hi, v.lo, j, th, tl, tj) || cur < K;
      }
      int tc;
      int pre = block_excl_scan(adm ? 1 : 0, ssh, &tc);
      if (adm) {
        su[cur + pre] = v.hi;
        sl[cur + pre] = v.lo;
        sj[cur + pre] = j;
      }
      cur += tc;
      __syncthreads();
      if (cur > BEST - ST || base + ST >= Ncand) {
        int n2 = 1;
        while (n2 < cur) n2 <<= 1;
        for (int i = cur + tid; i < n2; i += ST) {
          su[i] = __int_as_float(0x7f800000);
          sl[i] = 0.f;
          sj[i] = 0x7fffffff;
        }
        __syncthreads();
        block_bitonic(su, sl, sj, n2);
        cur = cur < K ? cur : K;
        if (cur >= K) {
          th = su[K - 1];
          tl = sl[K - 1];
          tj = sj[K - 1];
        }
        __syncthreads();
      }
    }
    for (int q = tid; q < K; q += ST) {
      idx[(size_t)gg * K + q] = sj[q];
      dd[(size_t)gg * K + q] = su[q];
    }
    m = -1;
  }
  if (tid == 0 && st) {
    if (m >= 0) {
      atomicAdd(&st->margin_sum, (unsigned long long)m);
      atomicMax(&st->margin_max, m);
    } else {
      atomicAdd(&st->overflow, 1);
    }
  }
}

}  // namespace

void launch_topk_partial(const glr_plan* pl, const float* dist, const float* kmeta,
                         const float* prt, int g0, int nk, int32_t* lj, float* lu, float* ll,
                         int32_t* lcnt, hipStream_t s) {
  const float coef = 2.0f * (float)(pl->D + 8) * 5.9604644775390625e-08f;   // 2^-24
  const int items = nk * pl->n_split;
  hipLaunchKernelGGL(k_topk_partial, dim3((items + 3) / 4), dim3(256), 0, s, dist, (size_t)pl->ldd,
                     (const float2*)kmeta, g0, prt, pl->Ncand, pl->split_len, pl->n_split, nk,
                     pl->K, coef, lj, lu, ll, lcnt);
}

void launch_select_rescore(const glr_plan* pl, const float* xp, const float* A, int g0, int nk,
                           const int32_t* lj, const float* lu, const float* ll,
                           const int32_t* lcnt, int32_t* idx, float* dd, DevStats* st,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_select_rescore, dim3(nk), dim3(ST), 0, s, xp, pl->H, pl->W, pl->P, pl->Cp,
                     pl->D, A, g0, pl->n_split, pl->Ncand, pl->K, lj, lu, ll,
                     lcnt, idx, dd, st);
}
