// Top-K grouping (eq. 1 with KNN grouping, searched over the whole image).
//
// The matcher's d~ carries a rounding error bounded by eps_j:
//  FP32 form:  eps_j = 2 (D + 8) u (||k|| + ||p_j||)^2
//    (dot product and norms in FP32, plus the epilogue roundings);
//  BF16 form:  eps_j = 4 (2 b + b^2) ||a|| ||pbar_j|| + (3 D + 26) u R_j^2,
//              R_j = ||a|| + ||pbar_j|| + sqrt(D) |mu_k - mu_j|
//    (a, pbar_j the centred key and candidate, b = 2^-9 the BF16 operand
//    rounding, FP32 accumulation and epilogue in the second term),
// u = 2^-24, each with a safety factor of two.  With U_j = d~_j + eps_j and L_j = d~_j - eps_j, let T be
// the K-th smallest U_j of a key: every member of the exact top-K has
// L_j <= d_j <= T, so the margin set {j : L_j <= T} contains the exact
// answer.  Stage 1 finds, per (key, candidate range), the range's margin set
// against the range's own T (an upper bound of the key's T) in one streaming
// pass; stage 2 merges the ranges, applies the key's T, recomputes the
// distance of each margin member with compensated (double-float32)
// arithmetic and sorts by (distance, position), lowest position winning ties.
#include <cmath>

#include "common.h"
#include "internal.h"

namespace {

constexpr int CAP = GLR_SPLIT_CAP;        // entries per wave buffer
constexpr int UCAP = GLR_UNION_CAP;       // entries per key in stage 2

// One digit of a radix selection: hist[256] holds the counts of the keys
// that match the prefix so far, by digit; find the digit of the
// remaining-th smallest of them and fold it into prefix / remaining.
// Lane l owns bins 4l..4l+3.
__device__ __forceinline__ void wave_radix_digit(const int* hist, int shift, uint32_t& prefix,
                                                 int& remaining) {
  const int l = lane_id();
  const int c0 = hist[4 * l], c1 = hist[4 * l + 1], c2 = hist[4 * l + 2], c3 = hist[4 * l + 3];
  const int tot = c0 + c1 + c2 + c3;
  const int incl = wave_incl_scan(tot);
  const int excl = incl - tot;
  const bool mine = excl < remaining && remaining <= incl;
  int digit = 0, below = 0;
  if (mine) {
    int r = remaining - excl;
    if (r <= c0) { digit = 4 * l; below = excl; }
    else if (r <= c0 + c1) { digit = 4 * l + 1; below = excl + c0; }
    else if (r <= c0 + c1 + c2) { digit = 4 * l + 2; below = excl + c0 + c1; }
    else { digit = 4 * l + 3; below = excl + c0 + c1 + c2; }
  }
  const uint64_t who = __ballot(mine);
  const int src = who ? (int)__builtin_ctzll(who) : 0;
  digit = __shfl(digit, src, 64);
  below = __shfl(below, src, 64);
  prefix |= (uint32_t)digit << shift;
  remaining -= below;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// K-th smallest of vals[0..n) by radix selection on the ordered uint32 keys:
// four passes of an 8-bit digit histogram in LDS (integer adds), most
// significant digit first.  One wave; requires n >= K >= 1.
__device__ float wave_kth_smallest(const float* vals, int n, int K, int* hist) {
  const int l = lane_id();
  uint32_t prefix = 0u;
  int remaining = K;
  for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[4 * l + b] = 0;
    wave_sync_lds();
    const uint32_t hmask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
    for (int i = l; i < n; i += 64) {
      const uint32_t key = f2ord(vals[i]);
      if ((key & hmask) == (prefix & hmask)) atomicAdd(&hist[(key >> shift) & 255u], 1);
    }
    wave_sync_lds();
    wave_radix_digit(hist, shift, prefix, remaining);
  }
  return ord2f(prefix);
}

// Same selection over S lists in global memory: list sp holds
// __shfl(c, sp) values at lists + sp * CAP (c: lane sp's count).  Requires
// the total count >= K >= 1.
__device__ float wave_kth_lists(const float* __restrict__ lists, int c, int S, int K, int* hist) {
  const int l = lane_id();
  uint32_t prefix = 0u;
  int remaining = K;
  for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[4 * l + b] = 0;
    wave_sync_lds();
    const uint32_t hmask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
    for (int sp = 0; sp < S; ++sp) {
      const int csp = __shfl(c, sp, 64);
      const float* src = lists + (size_t)sp * CAP;
      for (int i = l; i < csp; i += 64) {
        const uint32_t key = f2ord(src[i]);
        if ((key & hmask) == (prefix & hmask)) atomicAdd(&hist[(key >> shift) & 255u], 1);
      }
    }
    wave_sync_lds();
    wave_radix_digit(hist, shift, prefix, remaining);
  }
  return ord2f(prefix);
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

// BF = false: km = (||k||^2, ||k||) per key, cm = ||p_j|| per candidate.
// BF = true:  km = (||a||^2, mu_k, sum a, ||a||) per key, cm = (mu_j, ||pbar_j||)
//             per candidate.
template <bool BF>
__global__ void __launch_bounds__(256)
k_topk_partial(const float* __restrict__ dist, size_t ldd, const float* __restrict__ km, int g0,
               const float* __restrict__ cm, int Ncand, int split_len, int S, int nk, int K,
               float coef, float coef2, float sqrtD, int32_t* __restrict__ lj,
               float* __restrict__ lu, float* __restrict__ ll, int32_t* __restrict__ lcnt) {
  __shared__ int sbj[4][CAP];
  __shared__ float sbu[4][CAP];
  __shared__ float sbl[4][CAP];
  __shared__ int shist[4][256];
  const int wave = threadIdx.x >> 6;
  const int l = lane_id();
  const int item = blockIdx.x * 4 + wave;
  if (item >= nk * S) return;               // wave-uniform; no block barriers below
  int* bj = sbj[wave];
  float* bu = sbu[wave];
  float* bl = sbl[wave];
  int* hist = shist[wave];
  const int g = item / S, sp = item - g * S;
  const int j0 = sp * split_len;
  const int j1 = min(Ncand, j0 + split_len);
  const float kr = BF ? km[4 * (size_t)(g0 + g) + 3] : km[2 * (size_t)(g0 + g) + 1];
  const float kmu = BF ? km[4 * (size_t)(g0 + g) + 1] : 0.f;
  const float* drow = dist + (size_t)g * ldd;
  float T = __int_as_float(0x7f800000);     // +inf
  int cnt = 0;
  bool ovf = false;
  // 1024 candidates per chunk (four float4 loads of d~ and of ||p|| per
  // lane); the next chunk's loads are issued before the current chunk is
  // processed.  One ballot rejects a chunk in the common case where no
  // element can enter the margin set.
  constexpr int U4 = 4;
  constexpr int CH = 256 * U4;
  // pv: ||p_j|| (FP32 form) or ||pbar_j|| (BF16 form); mv: mu_j (BF16 form)
  float dv[U4][4], pv[U4][4], mv[U4][4], dn[U4][4], pn[U4][4], mn[U4][4];
  auto load = [&](int base, float (&d)[U4][4], float (&p)[U4][4], float (&m)[U4][4]) {
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int j = base + u * 256 + 4 * l;
      if (j + 3 < j1) {
        const float4 a = *reinterpret_cast<const float4*>(drow + j);
        d[u][0] = a.x; d[u][1] = a.y; d[u][2] = a.z; d[u][3] = a.w;
        if constexpr (BF) {
          const float4 b0 = *reinterpret_cast<const float4*>(cm + 2 * (size_t)j);
          const float4 b1 = *reinterpret_cast<const float4*>(cm + 2 * (size_t)j + 4);
          m[u][0] = b0.x; p[u][0] = b0.y; m[u][1] = b0.z; p[u][1] = b0.w;
          m[u][2] = b1.x; p[u][2] = b1.y; m[u][3] = b1.z; p[u][3] = b1.w;
        } else {
          const float4 b = *reinterpret_cast<const float4*>(cm + j);
          p[u][0] = b.x; p[u][1] = b.y; p[u][2] = b.z; p[u][3] = b.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = j + e < j1;
          d[u][e] = ok ? drow[j + e] : 0.f;
          if constexpr (BF) {
            m[u][e] = ok ? cm[2 * (size_t)(j + e)] : 0.f;
            p[u][e] = ok ? cm[2 * (size_t)(j + e) + 1] : 0.f;
          } else {
            p[u][e] = ok ? cm[j + e] : 0.f;
          }
        }
      }
    }
  };
  load(j0, dv, pv, mv);
  for (int base = j0; base < j1; base += CH) {
    if (base + CH < j1) load(base + CH, dn, pn, mn);
    // positions past the end of the range are never admitted (explicit
    // validity: an infinite L would still pass L <= T while T is +inf)
    float Lv[U4][4], Uv[U4][4];
    bool ok[U4][4];
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = base + u * 256 + 4 * l + e;
        float eps;
        if constexpr (BF) {
          const float R = (kr + pv[u][e]) + sqrtD * fabsf(kmu - mv[u][e]);
          eps = coef * (kr * pv[u][e]) + coef2 * (R * R);
        } else {
          const float sm = kr + pv[u][e];
          eps = coef * (sm * sm);
        }
        ok[u][e] = j < j1;
        Uv[u][e] = dv[u][e] + eps;
        Lv[u][e] = dv[u][e] - eps;
      }
    if (base == j0) {
      // seed T with the K-th smallest U of the first chunk (an upper bound of
      // the range's K-th smallest U)
#pragma unroll
      for (int u = 0; u < U4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          bu[(u * 64 + l) * 4 + e] = ok[u][e] ? Uv[u][e] : __int_as_float(0x7f800000);
      T = wave_kth_smallest(bu, CH, K, hist);
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) any = any || (ok[u][e] && Lv[u][e] <= T);
    if (__ballot(any) != 0) {
#pragma unroll
      for (int u = 0; u < U4; ++u) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool adm = ok[u][e] && Lv[u][e] <= T;
          const uint64_t m = __ballot(adm);
          if (adm) {
            const int pos = cnt + lanes_below(m);
            bj[pos] = base + u * 256 + 4 * l + e;
            bu[pos] = Uv[u][e];
            bl[pos] = Lv[u][e];
          }
          cnt += __popcll(m);
        }
        // room for the next 256 entries, else tighten T and compact
        if (cnt > CAP - 256) {
          const float Tn = wave_kth_smallest(bu, cnt, K, hist);
          T = fminf(T, Tn);
          cnt = wave_compact(bj, bu, bl, cnt, T);
          if (cnt > CAP - 256) {
            ovf = true;
            break;
          }
        }
      }
    }
    if (ovf) break;
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        dv[u][e] = dn[u][e];
        pv[u][e] = pn[u][e];
        if constexpr (BF) mv[u][e] = mn[u][e];
      }
  }
  if (!ovf && cnt >= K) {
    const float Tn = wave_kth_smallest(bu, cnt, K, hist);
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

// Wave-level bitonic sort of n (power of two, <= UW) entries by (hi, lo, j).
__device__ void wave_bitonic(float* h, float* lo, int* j, int n) {
  const int l = lane_id();
  for (int k = 2; k <= n; k <<= 1)
    for (int s = k >> 1; s > 0; s >>= 1) {
      for (int i = l; i < n; i += 64) {
        const int p = i ^ s;
        if (p > i) {
          const bool up = (i & k) == 0;
          const bool gt = df_less(h[p], lo[p], j[p], h[i], lo[i], j[i]);   // a[i] > a[p]
          if (gt == up) {
            const float th = h[i], tl = lo[i];
            const int tj = j[i];
            h[i] = h[p]; lo[i] = lo[p]; j[i] = j[p];
            h[p] = th; lo[p] = tl; j[p] = tj;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

constexpr int UW = 1024;          // margin-set capacity per key (wave path)

// One wave per key: the key's threshold T (K-th smallest U over all range
// lists) by a radix selection streamed over the lists, the margin set
// {L <= T} gathered in list order, rescored with compensated arithmetic,
// sorted by (distance, position); the first K are kept.  Only the margin set
// is held in LDS, so the lists' union may be far larger than UW.  Keys
// whose margin set exceeds UW, or whose range lists overflowed, are flagged
// for the kernel below.
__global__ void __launch_bounds__(256)
k_select_rescore(const float* __restrict__ xp, int H, int W, int P, int Cp, int D,
                 const float* __restrict__ A, int g0, int nk, int S, int Ncand, int K,
                 const int32_t* __restrict__ lj, const float* __restrict__ lu,
                 const float* __restrict__ ll, const int32_t* __restrict__ lcnt,
                 int32_t* __restrict__ idx, float* __restrict__ dd, int32_t* __restrict__ oflag,
                 DevStats* st) {
  __shared__ float su[4][UW];
  __shared__ float sl[4][UW];
  __shared__ int sj[4][UW];
  __shared__ int shist[4][256];
  const int wave = threadIdx.x >> 6;
  const int l = lane_id();
  const int g = blockIdx.x * 4 + wave;
  if (g >= nk) return;                      // wave-uniform
  float* u = su[wave];
  float* lo = sl[wave];
  int* jj = sj[wave];
  const int gg = g0 + g;
  const int Wc = W - P + 1;
  // split counts (S <= 64: one lane per split)
  const int c = l < S ? lcnt[g * S + l] : 0;
  const bool bad = __ballot(c < 0) != 0;
  const int tot = wave_sum_i32(c < 0 ? 0 : c);
  if (bad || tot < K) {
    if (l == 0) oflag[g] = 2;               // exact full-row path
    return;
  }
  const size_t o0 = (size_t)g * S * CAP;
  const float T = wave_kth_lists(lu + o0, c, S, K, shist[wave]);
  // margin set: ordered compaction of the entries with L <= T
  int m = 0;
  for (int sp = 0; sp < S; ++sp) {
    const int csp = __shfl(c, sp, 64);
    const size_t o = o0 + (size_t)sp * CAP;
    for (int base = 0; base < csp; base += 64) {
      const int i = base + l;
      const int jv = i < csp ? lj[o + i] : -1;
      const bool keep = i < csp && ll[o + i] <= T && jv >= 0 && jv < Ncand;
      const uint64_t msk = __ballot(keep);
      const int pos = m + lanes_below(msk);
      if (keep && pos < UW) jj[pos] = jv;
      m += __popcll(msk);
    }
  }
  if (m > UW || m < K) {                     // m < K cannot happen with valid lists
    if (l == 0) oflag[g] = m > UW ? 1 : 2;
    return;
  }
  if (l == 0) oflag[g] = 0;
  wave_sync_lds();
  // compensated rescoring, one entry per lane
  const float* kvec = A + (size_t)gg * D;
  for (int i = l; i < m; i += 64) {
    const df32 v = exact_dist(xp, H, W, P, Cp, kvec, jj[i], Wc);
    u[i] = v.hi;
    lo[i] = v.lo;
  }
  int n2 = 1;
  while (n2 < m) n2 <<= 1;
  for (int i = m + l; i < n2; i += 64) {
    u[i] = __int_as_float(0x7f800000);
    lo[i] = 0.f;
    jj[i] = 0x7fffffff;
  }
  wave_sync_lds();
  wave_bitonic(u, lo, jj, n2);
  for (int q = l; q < K; q += 64) {
    idx[(size_t)gg * K + q] = jj[q];
    dd[(size_t)gg * K + q] = u[q];
  }
  if (l == 0 && st) {
    atomicAdd(&st->margin_sum, (unsigned long long)m);
    atomicMax(&st->margin_max, m);
  }
}

// Flagged keys, one block per key (unflagged keys exit at once):
//  flag 1: the margin set exceeds the wave buffer; same threshold / rescore /
//          sort as the wave path with up to UCAP margin entries in LDS;
//  flag 2 (a range list overflowed) or a margin set above UCAP: exact
//          full-row path, every candidate rescored with compensated
//          arithmetic and a running best list kept in LDS (flat images, where
//          most distances lie within the error bound of each other).
__global__ void __launch_bounds__(ST)
k_rescore_overflow(const float* __restrict__ xp, int H, int W, int P, int Cp, int D,
                   const float* __restrict__ A, int g0, int S, int Ncand, int K,
                   const int32_t* __restrict__ lj, const float* __restrict__ lu,
                   const float* __restrict__ ll, const int32_t* __restrict__ lcnt,
                   const int32_t* __restrict__ oflag, int32_t* __restrict__ idx,
                   float* __restrict__ dd, DevStats* st) {
  __shared__ float su[UCAP];
  __shared__ float sl[UCAP];
  __shared__ int sj[UCAP];
  __shared__ int ssh[ST / 64 + 1];
  __shared__ int scnt[64];
  const int g = blockIdx.x;
  const int flag = oflag[g];
  if (flag == 0) return;                     // block-uniform
  const int gg = g0 + g;
  const int tid = threadIdx.x;
  const int Wc = W - P + 1;
  const float* kvec = A + (size_t)gg * D;
  if (tid < S) scnt[tid] = lcnt[g * S + tid];
  __syncthreads();
  if (flag == 1) {
    const size_t o0 = (size_t)g * S * CAP;
    // T: smallest U value (as ordered bits) with at least K list values <= it
    uint32_t lo = 0u, hi = 0xffffffffu;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      int c = 0;
      for (int sp = 0; sp < S; ++sp) {
        const int csp = scnt[sp];
        for (int i = tid; i < csp; i += ST) c += (f2ord(lu[o0 + (size_t)sp * CAP + i]) <= mid) ? 1 : 0;
      }
      c = block_sum_i(c, ssh);
      if (c >= K) hi = mid; else lo = mid + 1;
    }
    const float T = ord2f(lo);
    int m = 0;
    for (int sp = 0; sp < S; ++sp) {
      const int csp = scnt[sp];
      const size_t o = o0 + (size_t)sp * CAP;
      for (int base = 0; base < csp; base += ST) {
        const int i = base + tid;
        const int jv = i < csp ? lj[o + i] : -1;
        const bool keep = i < csp && ll[o + i] <= T && jv >= 0 && jv < Ncand;
        int tc;
        const int pre = block_excl_scan(keep ? 1 : 0, ssh, &tc);
        if (keep && m + pre < UCAP) sj[m + pre] = jv;
        m += tc;
      }
    }
    __syncthreads();
    if (m > UCAP) goto full_row;
    if (m < K) goto full_row;                 // cannot happen with valid lists; stay safe
    for (int i = tid; i < m; i += ST) {
      const df32 v = exact_dist(xp, H, W, P, Cp, kvec, sj[i], Wc);
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
    if (tid == 0 && st) {
      atomicAdd(&st->margin_sum, (unsigned long long)m);
      atomicMax(&st->margin_max, m);
    }
    return;
  }
full_row:
  const int BEST = UCAP;
  int cur = 0;
  float th = __int_as_float(0x7f800000), tl = 0.f;
  int tj = 0x7fffffff;
  for (int base = 0; base < Ncand; base += ST) {
    const int j = base + tid;
    df32 v = {0.f, 0.f};
    bool adm = false;
    if (j < Ncand) {
      v = exact_dist(xp, H, W, P, Cp, kvec, j, Wc);
      adm = cur < K || df_less(v.hi, v.lo, j, th, tl, tj);
    }
    int tc;
    const int pre = block_excl_scan(adm ? 1 : 0, ssh, &tc);
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
  if (tid == 0 && st) atomicAdd(&st->overflow, 1);
}

}  // namespace

void launch_topk_partial(const glr_plan* pl, const float* dist, const float* km,
                         const float* cm, int g0, int nk, int32_t* lj, float* lu, float* ll,
                         int32_t* lcnt, hipStream_t s) {
  const double u = 5.9604644775390625e-08;      // 2^-24
  const double b = 0.001953125;                 // 2^-9
  const int items = nk * pl->n_split;
  const dim3 grid((items + 3) / 4);
  if (pl->precision == GLR_PREC_BF16_RESCORE) {
    // coefficients rounded up so that the float values are not below the bound
    const float coef = std::nextafter((float)(4.0 * (2.0 * b + b * b)), 1.f);
    const float coef2 = std::nextafter((float)((3.0 * pl->D + 26.0) * u), 1.f);
    const float sqrtD = std::nextafter((float)std::sqrt((double)pl->D), 1e9f);
    hipLaunchKernelGGL(k_topk_partial<true>, grid, dim3(256), 0, s, dist, (size_t)pl->ldd, km, g0,
                       cm, pl->Ncand, pl->split_len, pl->n_split, nk, pl->K, coef, coef2, sqrtD,
                       lj, lu, ll, lcnt);
  } else {
    const float coef = std::nextafter((float)(2.0 * (pl->D + 8) * u), 1.f);
    hipLaunchKernelGGL(k_topk_partial<false>, grid, dim3(256), 0, s, dist, (size_t)pl->ldd, km, g0,
                       cm, pl->Ncand, pl->split_len, pl->n_split, nk, pl->K, coef, 0.f, 0.f, lj,
                       lu, ll, lcnt);
  }
}

void launch_select_rescore(const glr_plan* pl, const float* xp, const float* A, int g0, int nk,
                           const int32_t* lj, const float* lu, const float* ll,
                           const int32_t* lcnt, int32_t* idx, float* dd, int32_t* oflag,
                           DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_select_rescore, dim3((nk + 3) / 4), dim3(256), 0, s, xp, pl->H, pl->W, pl->P,
                     pl->Cp, pl->D, A, g0, nk, pl->n_split, pl->Ncand, pl->K, lj, lu, ll, lcnt, idx,
                     dd, oflag, st);
  hipLaunchKernelGGL(k_rescore_overflow, dim3(nk), dim3(ST), 0, s, xp, pl->H, pl->W, pl->P, pl->Cp,
                     pl->D, A, g0, pl->n_split, pl->Ncand, pl->K, lj, lu, ll, lcnt, oflag, idx, dd,
                     st);
}
