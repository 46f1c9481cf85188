// Top-K grouping (eq. 1 with KNN grouping, searched over the whole image).
//
// The matcher's d~ (BF16 form: one mean per patch) carries a rounding error
// bounded by
//     eps_j = c2 R_j^2 + c1 (||a|| ||e_j|| + ||e_a|| (||pbar_j|| + ||e_j||)),
//     R_j = ||a|| + ||pbar_j|| + sqrt(D) |mu_k - mu_j|,
// with a, pbar_j the centred key and candidate (FP32), e_a = a - bf16(a) and
// e_j = pbar_j - bf16(pbar_j) the exact residuals of the BF16 operands (their
// norms computed by the metadata kernels), u = 2^-24 (FP32 unit round-off)
// and
//     c2 = (3 D + 26) u       (FP32 dot-product sums, centring, epilogue;
//                              a safety factor of two),
//     c1 = 2 (1 + 2^-8)       (the BF16 operands: <a, pbar> - <bf16(a),
//                              bf16(pbar)> = <a, e_j> + <e_a, bf16(pbar)>
//                              exactly, at most ||a|| ||e_j|| + ||e_a||
//                              (||pbar|| + ||e_j||) by Cauchy-Schwarz, twice
//                              on -2 S; the factor 1 + 2^-8 covers the FP32
//                              roundings of the norms and products).
// The FP32 form's bound (channel-centred) is described at k_topk_partial.
// With U_j = d~_j + eps_j and
// L_j = d~_j - eps_j, let T be the K-th smallest U_j of a key: every member
// of the exact top-K has L_j <= d_j <= T, so the margin set {j : L_j <= T}
// contains the exact answer.  Stage 1 finds, per (key, candidate range), the
// range's margin set against an upper bound of T (the range's own K-th
// smallest U, tightened by the best bound any range of the key has
// published so far) in one streaming pass; stage 2 selects the key's T over
// the range lists, recomputes the distance of each margin member in FP64
// (exact differences, FP64 sums) and sorts by (distance, position), lowest
// position winning ties.
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

// Error bound eps of one candidate's d~ (see k_topk_partial for the two
// forms); d: d~, p: the candidate's centred norm, m: its mean (BF16 form) or
// channel-mean term h_j (FP32 form), ep: its BF16 residual norm (BF16 form);
// kr, kmu, ek: the key's.
__device__ __forceinline__ float margin_eps(float d, float p, float m, float ep, float kr,
                                            float kmu, float ek, int pc, float coef,
                                            float coef2, float cz) {
  if (pc) {
    const float w = cz * (kmu + m);
    // hardware square root (within 1 ulp; the bound's slack covers it)
    // of max(d~, smallest normal), which is never below sqrt(max(d~, 0))
    const float y = ((kr + p) + __builtin_amdgcn_sqrtf(fmaxf(d, 0x1p-126f))) + w;
    return fmaf(y, fmaf(coef2, y, w), w * w);
  }
  // (fused: nine instructions per candidate instead of twelve; every
  // rounding is still covered by the coefficients' slack)
  const float R = fmaf(cz, fabsf(kmu - m), kr + p);
  return fmaf(coef2 * R, R, coef * fmaf(ek, p + ep, kr * ep));
}

// Error bound of d~ per candidate (key row kmap[g0+g] or g0+g):
//  pc == 0 (BF16 form, one mean per patch): km = (||a||^2, mu_k, sum a, ||a||),
//    ke = ||e_a||, cm = (mu_j, ||pbar_j||), ce = ||e_j||; eps = coef (||a||
//    ||e_j|| + ||e_a|| (||pbar_j|| + ||e_j||)) + coef2 R^2 with
//    R = ||a|| + ||pbar|| + cz |mu_k - mu_j|, cz = sqrt(D);
//  pc == 1 (channel-centred FP32 form): km = (||a~||^2, h_k, 0, ||a~||),
//    cm = (h_j, ||p~_j||); with w = cz (h_k + h_j) (the centring residues)
//    and y = ||a~|| + ||p~|| + sqrt(max(d~, 0)) + w, eps = y (coef2 y + w) + w^2:
//    the channel-mean part of the bound is itself bounded through the
//    distance.
// tsh[g]: the key's shared bound of T (ordered bits, +inf at launch), lowered
// with atomicMin by every range.
template <int U4, int WCAP, int MINW, bool PF, int pc>
__global__ void __launch_bounds__(256, MINW)
k_topk_partial(const float* __restrict__ dist, size_t ldd, const float4* __restrict__ km,
               const float* __restrict__ ke, const int32_t* __restrict__ kmap, int g0,
               const float* __restrict__ cm, const float* __restrict__ ce, int Ncand,
               int split_len, int S, int nk, int K, float coef, float coef2, float cz,
               uint32_t* __restrict__ tsh, int32_t* __restrict__ lj, float* __restrict__ lu,
               float* __restrict__ ll, int32_t* __restrict__ lcnt) {
  static_assert(WCAP >= 512 && WCAP <= CAP, "wave buffer size");
  __shared__ int sbj[4][WCAP];
  __shared__ float sbu[4][WCAP];
  __shared__ float sbl[4][WCAP];
  __shared__ int shist[4][256];
  const int wave = threadIdx.x >> 6;
  const int l = lane_id();
  // the four waves of a block take four keys over the same candidate range,
  // so they read the same candidate bound terms (mostly from L1)
  const int sp = blockIdx.x % S;
  const int g = (blockIdx.x / S) * 4 + wave;
  if (g >= nk) return;                      // wave-uniform; no block barriers below
  const int item = g * S + sp;
  int* bj = sbj[wave];
  float* bu = sbu[wave];
  float* bl = sbl[wave];
  int* hist = shist[wave];
  const int j0 = sp * split_len;
  const int j1 = min(Ncand, j0 + split_len);
  const int gk = kmap ? kmap[g0 + g] : g0 + g;
  const float4 kmv = km[gk];
  const float kr = kmv.w, kmu = kmv.y;
  const float ek = pc ? 0.f : ke[gk];
  // publish T to the key's shared bound and take the bound back
  auto share = [&](float Tl) {
    uint32_t old = 0u;
    if (l == 0) old = atomicMin(&tsh[g], f2ord(Tl));
    old = __shfl(old, 0, 64);
    return fminf(Tl, ord2f(old));
  };
  const float* drow = dist + (size_t)g * ldd;
  float T = __int_as_float(0x7f800000);     // +inf
  int cnt = 0;
  bool ovf = false;
  // 256 U4 candidates per chunk (U4 float4 loads of d~ and 2 U4 of the
  // candidate bound terms per lane); the next chunk's loads are issued before
  // the current chunk is processed.  One ballot rejects a chunk in the common
  // case where no element can enter the margin set.  WCAP entries of wave
  // buffer: the first chunk's first WCAP candidates seed T.
  constexpr int CH = 256 * U4;
  constexpr int SU = WCAP / 256 < U4 ? WCAP / 256 : U4;   // chunk blocks that seed T
  // pv: ||pbar_j||; mv: mu_j; ev: ||e_j|| (BF16 form)
  // ev: the BF16 form's residual norms, loaded with the next chunk (PF) or
  // at the start of each chunk (fewer registers; the other waves of the
  // SIMD cover the latency)
  float dv[U4][4], pv[U4][4], mv[U4][4], dn[U4][4], pn[U4][4], mn[U4][4];
  float ev[U4][4], en[U4][4];
  // Every load is one unconditional 16-byte read, and the next chunk is
  // always prefetched: a chunk starts at most one chunk past the range (j0
  // and the chunk size are multiples of 4, so j is too) and the streamed
  // arrays carry SPAD entries of padding, so reads past j1 stay in bounds;
  // their values are never admitted (ok below).  No branch around a load,
  // so the next chunk's loads stay in flight while this one is processed.
  auto load_ev = [&](int base, float (&ee)[U4][4]) {
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int j = base + u * 256 + 4 * l;
      float4 c4 = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (!pc) c4 = *reinterpret_cast<const float4*>(ce + j);   // pc: no residual norms
      ee[u][0] = c4.x; ee[u][1] = c4.y; ee[u][2] = c4.z; ee[u][3] = c4.w;
    }
  };
  auto load = [&](int base, float (&d)[U4][4], float (&p)[U4][4], float (&m)[U4][4]) {
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int j = base + u * 256 + 4 * l;
      const float4 a = *reinterpret_cast<const float4*>(drow + j);
      d[u][0] = a.x; d[u][1] = a.y; d[u][2] = a.z; d[u][3] = a.w;
      const float4 b0 = *reinterpret_cast<const float4*>(cm + 2 * (size_t)j);
      const float4 b1 = *reinterpret_cast<const float4*>(cm + 2 * (size_t)j + 4);
      m[u][0] = b0.x; p[u][0] = b0.y; m[u][1] = b0.z; p[u][1] = b0.w;
      m[u][2] = b1.x; p[u][2] = b1.y; m[u][3] = b1.z; p[u][3] = b1.w;
    }
  };
  load(j0, dv, pv, mv);
  if constexpr (PF) load_ev(j0, ev);
  for (int base = j0; base < j1; base += CH) {
    load(base + CH, dn, pn, mn);
    if constexpr (PF) load_ev(base + CH, en);
    if constexpr (!PF) load_ev(base, ev);
    // positions past the end of the range are never admitted (explicit
    // validity: an infinite L would still pass L <= T while T is +inf)
    float Lv[U4][4], Uv[U4][4];
    bool ok[U4][4];
#pragma unroll
    for (int u = 0; u < U4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = base + u * 256 + 4 * l + e;
        const float eps = margin_eps(dv[u][e], pv[u][e], mv[u][e], ev[u][e], kr, kmu, ek, pc,
                                     coef, coef2, cz);
        ok[u][e] = j < j1;
        Uv[u][e] = dv[u][e] + eps;
        Lv[u][e] = dv[u][e] - eps;
      }
    if (base == j0) {
      // seed T with the K-th smallest U of the first chunk (an upper bound of
      // the range's K-th smallest U)
#pragma unroll
      for (int u = 0; u < SU; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          bu[(u * 64 + l) * 4 + e] = ok[u][e] ? Uv[u][e] : __int_as_float(0x7f800000);
      T = share(wave_kth_smallest(bu, SU * 256, K, hist));
    } else if ((((base - j0) / CH) & 7) == 0) {
      T = share(T);                         // take up other ranges' progress
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
        if (cnt > WCAP - 256) {
          const float Tn = wave_kth_smallest(bu, cnt, K, hist);
          T = share(fminf(T, Tn));
          cnt = wave_compact(bj, bu, bl, cnt, T);
          if (cnt > WCAP - 256) {
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
        mv[u][e] = mn[u][e];
        if constexpr (PF) ev[u][e] = en[u][e];
      }
  }
  if (!ovf) {
    if (cnt >= K) T = fminf(T, wave_kth_smallest(bu, cnt, K, hist));
    T = share(T);
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

// ---------------------------------------------------------------- exact rescoring
// The FP64 distance of one candidate is computed by L lanes together
// (L = 8..64, a power of two fixed by D): lane s of the group owns the patch
// elements t = s + e L in the channel-interleaved order t = (dy P + dx) Cp +
// c, holds the key's values and the elements' offsets in registers,
// accumulates its squared differences in FP64, and the group combines its
// partial sums with a butterfly of FP64 additions.  Candidates
// are read from the channel-interleaved copy of the image, xi[(r W + c) Cp +
// ch]: a patch row over all channels is one contiguous run of P Cp floats,
// so consecutive lanes read consecutive addresses and a patch spans P runs
// (P Cp / 32 cache lines each) instead of Cp P segments of P floats.
template <int EM>
struct KeySlice {
  double kv[EM];     // the key's values (FP32 data held in FP64 for the sums)
  int off[EM];       // offset of element t in xi relative to the patch's top-left
};

// Elements past D get offset 0 and are masked to a zero difference, so every
// load is unconditional (all of a lane's loads can be in flight at once).
template <int EM>
__device__ __forceinline__ void key_slice_load(KeySlice<EM>& ks, const float* __restrict__ kvec,
                                               int D, int P, int H, int W, int L, int s) {
  const int Cp = D / (P * P);
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    const int t = s + e * L;
    if (t < D) {
      const int pix = t / Cp, c = t - pix * Cp;
      const int dy = pix / P, dx = pix - dy * P;
      ks.kv[e] = (double)kvec[(c * P + dy) * P + dx];   // the key vector is in (c, dy, dx) order
      ks.off[e] = (dy * W + dx) * Cp + c;
    } else {
      ks.kv[e] = 0.0;
      ks.off[e] = -1;
    }
  }
}

// Exact-order distances of two candidates (xi offsets b0, b1 of their
// top-left pixels; both valid positions) by the L-lane group, in FP64: the
// difference of two FP32 values is exact in FP64 (their exponents are close
// for patch values; otherwise rounded at 2^-53), so the only roundings are
// those of the FP64 squares and sums, a relative error of about D 2^-53 —
// the oracle's own.  FP64 VALU instructions issue at the FP32 rate on gfx950,
// and the three per element here replace the ~25 of a double-float32 sum.
// The result is returned as (hi, lo) = (fl32(s), fl32(s - hi)), whose
// lexicographic order is the order of s up to 2^-48 relative.  Every lane of
// the group returns the group's sums; the lanes are combined by a fixed
// butterfly, and only the group's lane 0 result is stored by the callers.
template <int EM>
__device__ __forceinline__ void coop_dist2(const KeySlice<EM>& ks, const float* __restrict__ xi,
                                           size_t b0, size_t b1, int L, df32& r0, df32& r1) {
  float p0[EM], p1[EM];
  const float* x0 = xi + b0;
  const float* x1 = xi + b1;
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    const int o = ks.off[e] < 0 ? 0 : ks.off[e];
    p0[e] = x0[o];
    p1[e] = x1[o];
  }
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int e = 0; e < EM; ++e) {
    const bool ok = ks.off[e] >= 0;             // elements past D: zero difference
    const double d0 = ok ? ks.kv[e] - (double)p0[e] : 0.0;
    const double d1 = ok ? ks.kv[e] - (double)p1[e] : 0.0;
    a0 = fma(d0, d0, a0);
    a1 = fma(d1, d1, a1);
  }
  for (int o = L >> 1; o > 0; o >>= 1) {
    a0 += __shfl_xor(a0, o, 64);
    a1 += __shfl_xor(a1, o, 64);
  }
  r0.hi = (float)a0;
  r0.lo = (float)(a0 - (double)r0.hi);
  r1.hi = (float)a1;
  r1.lo = (float)(a1 - (double)r1.hi);
}

// Rescore entries i in [0, m) of a candidate list (pos(i) = image grid
// position) into (hh[i], ll[i]).  Each step a wave takes 2 * (64 / L)
// consecutive entries starting at i0 = first, first + stride, ...; the lane
// groups take two entries each.  Invalid slots read position 0 and are not
// written.
template <int EM, typename PosF>
__device__ __forceinline__ void coop_rescore(const KeySlice<EM>& ks, const float* __restrict__ xi,
                                             PosF pos, int first, int m, int stride, int Wc,
                                             int W, int Cp, int L, float* hh, float* ll) {
  const int l = lane_id();
  const int s = l & (L - 1), grp = l / L, cpi = 64 / L;
  for (int i0 = first; i0 < m; i0 += stride) {
    const int ia = i0 + grp, ib = i0 + cpi + grp;
    const bool va = ia < m, vb = ib < m;
    const int ja = va ? pos(ia) : 0, jb = vb ? pos(ib) : 0;
    const int ra = ja / Wc, rb = jb / Wc;
    df32 da, db;
    coop_dist2(ks, xi, (size_t)(ra * W + (ja - ra * Wc)) * Cp,
               (size_t)(rb * W + (jb - rb * Wc)) * Cp, L, da, db);
    if (s == 0) {
      if (va) { hh[ia] = da.hi; ll[ia] = da.lo; }
      if (vb) { hh[ib] = db.hi; ll[ib] = db.lo; }
    }
  }
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

constexpr int UW = 1024;          // list entries staged per key (wave path)
// Margin sets above MW go to the block path (four waves per key): the wave
// path rescores two candidates at a time, so a launch would otherwise wait
// on its keys with the largest sets.
constexpr int MW = 256;

// One wave per key: the key's threshold T (K-th smallest U over all range
// lists) by a radix selection streamed over the lists, the margin set
// {L <= T} gathered in list order, rescored in FP64,
// sorted by (distance, position); the first K are kept.  Only the margin set
// is held in LDS, so the lists' union may be far larger than UW.  Keys
// whose margin set exceeds MW, or whose range lists overflowed, are flagged
// for the kernel below.
template <int EM>
__global__ void __launch_bounds__(256)
k_select_rescore(const float* __restrict__ xi, int H, int W, int P, int Cp, int D, int L,
                 const float* __restrict__ A, const int32_t* __restrict__ kmap, int g0, int nk,
                 int S, int Ncand, int K,
                 const int32_t* __restrict__ lj, const float* __restrict__ lu,
                 const float* __restrict__ ll, const int32_t* __restrict__ lcnt,
                 int32_t* __restrict__ idx, float* __restrict__ dd, int32_t* __restrict__ oflag,
                 uint32_t* __restrict__ tsh, float* __restrict__ tkey, DevStats* st) {
  __shared__ float su[4][UW];
  __shared__ float sl[4][UW];
  __shared__ int sj[4][UW];
  __shared__ int shist[4][256];
  const int wave = threadIdx.x >> 6;
  const int l = lane_id();
  const int g = blockIdx.x * 4 + wave;
  if (g >= nk) return;                      // wave-uniform
  // the scan that used the key's shared bound has finished: keep its value
  // (an upper bound of the key's T, for the large-margin path) and restore
  // it to +inf for the next chunk or call
  if (l == 0) tkey[g] = ord2f(atomicExch(&tsh[g], 0xffffffffu));
  float* u = su[wave];
  float* lo = sl[wave];
  int* jj = sj[wave];
  const int gg = kmap ? kmap[g0 + g] : g0 + g;
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
  int m = 0;
  float T;                                   // the key's K-th smallest U over its lists
  if (tot <= UW) {
    // every list entry into LDS in list order (entry e of the concatenation
    // is in the last list whose offset is <= e), up to four loads per lane in
    // flight; an invalid position gets L = NaN, so it is never kept
    const int excl = wave_incl_scan(c) - c;  // lanes >= S hold c = 0
    for (int e0 = 0; e0 < tot; e0 += 256) {
      int sp[4] = {0, 0, 0, 0}, ex[4] = {0, 0, 0, 0};
      for (int q = 1; q < S; ++q) {
        const int eq = __builtin_amdgcn_readlane(excl, q);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (e0 + 64 * k + l >= eq) {
            sp[k] = q;
            ex[k] = eq;
          }
      }
      int jv[4];
      float uv[4], lv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = e0 + 64 * k + l;
        const size_t o = o0 + (size_t)sp[k] * CAP + (e - ex[k]);
        jv[k] = e < tot ? lj[o] : -1;
        uv[k] = e < tot ? lu[o] : 0.f;
        lv[k] = e < tot ? ll[o] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = e0 + 64 * k + l;
        if (e < tot) {
          jj[e] = jv[k];
          u[e] = uv[k];
          lo[e] = (jv[k] >= 0 && jv[k] < Ncand) ? lv[k] : __int_as_float(0x7fc00000);
        }
      }
    }
    wave_sync_lds();
    T = wave_kth_smallest(u, tot, K, shist[wave]);
    // margin set: ordered compaction of the entries with L <= T
    m = wave_compact(jj, u, lo, tot, T);
  } else {
    T = wave_kth_lists(lu + o0, c, S, K, shist[wave]);
    // margin set: ordered compaction of the entries with L <= T
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
  }
  if (m > MW || m < K) {                     // m < K cannot happen with valid lists
    if (l == 0) {
      oflag[g] = m > MW ? 1 : 2;
      if (m > MW) tkey[g] = T;               // the block path reuses the key's T
    }
    return;
  }
  if (l == 0) oflag[g] = 0;
  wave_sync_lds();
  // FP64 rescoring, L lanes per candidate, two candidates per group
  {
    KeySlice<EM> ks;
    key_slice_load(ks, A + (size_t)gg * D, D, P, H, W, L, l & (L - 1));
    coop_rescore(ks, xi, [&](int i) { return jj[i]; }, 0, m, 2 * (64 / L), Wc, W, Cp, L, u, lo);
  }
  wave_sync_lds();
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

// Rescore the margin set held in global scratch (positions gp[0..m)) and
// write the key's K smallest by (hi, lo, position), sorted, to idx/dd row gg:
// FP64 distances (as hi/lo pairs) into gh/gl, a radix selection of the K-th smallest
// 96-bit key (ord(hi), ord(lo + 0), position), the K entries at or below it
// gathered and sorted in LDS.  Every thread of the block calls it.
template <int EM>
__device__ void rescore_select_set(const KeySlice<EM>& ks, const float* __restrict__ xi,
                                   const int32_t* gp, float* gh, float* gl, int m, int K, int Wc,
                                   int W, int Cp, int L, int gg, int32_t* __restrict__ idx,
                                   float* __restrict__ dd, float* su, float* sl, int* sj,
                                   int* ssh, int* hist, uint32_t* sdig) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int cpi = 64 / L;
  coop_rescore(ks, xi, [&](int i) { return gp[i]; }, wave * 2 * cpi, m, 8 * cpi, Wc, W, Cp, L, gh,
               gl);
  __syncthreads();
  uint32_t pre[3] = {0u, 0u, 0u};
  int remaining = K;
  for (int p = 0; p < 12; ++p) {
    const int w = p >> 2, shift = 24 - 8 * (p & 3);
    const uint32_t hm = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
    hist[tid] = 0;
    __syncthreads();
    for (int i = tid; i < m; i += ST) {
      const uint32_t k0 = f2ord(gh[i]), k1 = f2ord(gl[i] + 0.f);
      const uint32_t k2 = (uint32_t)gp[i];
      bool match = true;
      if (w > 0) match = k0 == pre[0];
      if (w > 1) match = match && k1 == pre[1];
      const uint32_t kw = w == 0 ? k0 : (w == 1 ? k1 : k2);
      if (match && (kw & hm) == (pre[w] & hm)) atomicAdd(&hist[(kw >> shift) & 255u], 1);
    }
    __syncthreads();
    if (wave == 0) {
      uint32_t pfx = 0u;
      int rem = remaining;
      wave_radix_digit(hist, shift, pfx, rem);
      if (tid == 0) {
        sdig[0] = pfx;
        sdig[1] = (uint32_t)(remaining - rem);
      }
    }
    __syncthreads();
    pre[w] |= sdig[0];
    remaining -= (int)sdig[1];
    // entries that match the key so far and fall in the chosen bin
    const int inbin = hist[(sdig[0] >> shift) & 255u];
    __syncthreads();
    // a word of the key complete and every entry that matches it needed (the
    // common case: the K-th distance is not tied): the K entries are those
    // with a key up to this word, whatever the remaining words hold
    if ((p & 3) == 3 && w < 2 && inbin == remaining) {
      for (int v = w + 1; v < 3; ++v) pre[v] = 0xffffffffu;
      break;
    }
  }
  // the K entries with key <= the K-th key, in list order, then sorted
  int n = 0;
  for (int base = 0; base < m; base += ST) {
    const int i = base + tid;
    bool keep = false;
    float h = 0.f, lw = 0.f;
    int jv = 0;
    if (i < m) {
      h = gh[i];
      lw = gl[i] + 0.f;
      jv = gp[i];
      const uint32_t k0 = f2ord(h), k1 = f2ord(lw), k2 = (uint32_t)jv;
      keep = k0 < pre[0] || (k0 == pre[0] && (k1 < pre[1] || (k1 == pre[1] && k2 <= pre[2])));
    }
    int tc;
    const int q = block_excl_scan(keep ? 1 : 0, ssh, &tc);
    if (keep && n + q < 64) {
      su[n + q] = h;
      sl[n + q] = lw;
      sj[n + q] = jv;
    }
    n += tc;
  }
  __syncthreads();
  n = min(n, 64);                            // exactly K (positions are unique)
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = n + tid; i < n2; i += ST) {
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
}

// Smallest value v (as ordered bits) of vals[0..m) with at least K values
// <= v: the K-th smallest (requires m >= K).  Every thread calls it.
__device__ float block_kth_by_bisection(const float* vals, int m, int K, int* ssh) {
  uint32_t lo = 0u, hi = 0xffffffffu;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    int c = 0;
    for (int i = threadIdx.x; i < m; i += ST) c += (f2ord(vals[i]) <= mid) ? 1 : 0;
    c = block_sum_i(c, ssh);
    if (c >= K) hi = mid; else lo = mid + 1;
  }
  return ord2f(lo);
}

// Flagged keys, one block per key (unflagged keys exit at once):
//  flag 1: the margin set exceeds the wave path's share.  With the key's T
//          (the wave path leaves it in rb.tkey) it is gathered from the
//          range lists into global scratch (up to mcap entries) and handed
//          to rescore_select_set;
//  flag 2: a range list overflowed, so the lists do not hold the margin set.
//          With the key's distance row still in the chunk (rb.dist), it is
//          re-derived from the row: every candidate with L_j <= T', T' the
//          bound the key's scan published (T' >= T, so the candidates with
//          U_j <= T, hence the K smallest U, are all among them), is gathered
//          with (U, L); T is their K-th smallest U and the margin set
//          {L_j <= T} is compacted in place and handed to rescore_select_set;
//  either set above mcap: exact full-row path, every candidate rescored with
//          FP64 arithmetic and a running best list kept in LDS (flat
//          images, where most distances lie within the error bound of each
//          other).
// With defer != 0, flag-2 keys, and flag-1 keys whose set exceeds mcap, are
// left flagged for a later pass; keys completed here get their flag cleared.
template <int EM>
__global__ void __launch_bounds__(ST)
k_rescore_overflow(const float* __restrict__ xi, int H, int W, int P, int Cp, int D, int L,
                   const float* __restrict__ A, const int32_t* __restrict__ kmap, int g0, int S,
                   int Ncand, int K, int defer,
                   const int32_t* __restrict__ lj, const float* __restrict__ lu,
                   const float* __restrict__ ll, const int32_t* __restrict__ lcnt,
                   int32_t* __restrict__ oflag, int32_t* __restrict__ gpos,
                   float* __restrict__ ghi, float* __restrict__ glo, int mcap,
                   int32_t* __restrict__ idx, float* __restrict__ dd, RowBound rb,
                   DevStats* st) {
  __shared__ float su[UCAP];
  __shared__ float sl[UCAP];
  __shared__ int sj[UCAP];
  __shared__ int ssh[ST / 64 + 1];
  __shared__ int scnt[64];
  __shared__ float fh[ST], fl[ST];           // full-row path: staged distances
  __shared__ int hist[256];
  __shared__ uint32_t sdig[2];
  __shared__ int sgat;
  const int g = blockIdx.x;
  const int flag = oflag[g];
  if (flag == 0 || (flag == 2 && defer)) return;   // block-uniform
  const int gg = kmap ? kmap[g0 + g] : g0 + g;
  const int tid = threadIdx.x;
  const int Wc = W - P + 1;
  const int wave = tid >> 6;
  const int cpi = 64 / L;
  const size_t go = (size_t)g * mcap;
  KeySlice<EM> ks;
  key_slice_load(ks, A + (size_t)gg * D, D, P, H, W, L, (tid & 63) & (L - 1));
  if (tid < S) scnt[tid] = lcnt[g * S + tid];
  if (tid == 0) sgat = 0;
  __syncthreads();
  if (flag == 1) {
    const size_t o0 = (size_t)g * S * CAP;
    // T (the K-th smallest U over the key's lists) as the wave path found it
    const float T = rb.tkey[g];
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
        if (keep && m + pre < mcap) gpos[go + m + pre] = jv;
        m += tc;
      }
    }
    __syncthreads();
    if (m > mcap || m < K) {                 // m < K cannot happen with valid lists
      if (defer) return;
      goto full_row;
    }
    rescore_select_set(ks, xi, gpos + go, ghi + go, glo + go, m, K, Wc, W, Cp, L, gg, idx, dd, su,
                       sl, sj, ssh, hist, sdig);
    if (tid == 0) {
      oflag[g] = 0;
      if (st) {
        atomicAdd(&st->margin_sum, (unsigned long long)m);
        atomicMax(&st->margin_max, m);
      }
    }
    return;
  }
  if (rb.dist) {
    // flag 2: the margin set re-derived from the key's distance row
    const float Tp = rb.tkey[g];
    const float* drow = rb.dist + (size_t)g * rb.ldd;
    const float4 kmv = reinterpret_cast<const float4*>(rb.km)[gg];
    const float kr = kmv.w, kmu = kmv.y;
    const float ek = rb.pc ? 0.f : rb.kre[gg];
    const int l = tid & 63;
    for (int base = 0; base < Ncand; base += 4 * ST) {
      const int j = base + 4 * tid;
      float dv[4], pv[4], mv[4], ev[4];
      if (j + 3 < Ncand) {
        const float4 a = *reinterpret_cast<const float4*>(drow + j);
        const float4 b0 = *reinterpret_cast<const float4*>(rb.cm + 2 * (size_t)j);
        const float4 b1 = *reinterpret_cast<const float4*>(rb.cm + 2 * (size_t)j + 4);
        dv[0] = a.x; dv[1] = a.y; dv[2] = a.z; dv[3] = a.w;
        mv[0] = b0.x; pv[0] = b0.y; mv[1] = b0.z; pv[1] = b0.w;
        mv[2] = b1.x; pv[2] = b1.y; mv[3] = b1.z; pv[3] = b1.w;
        if (!rb.pc) {
          const float4 c4 = *reinterpret_cast<const float4*>(rb.cre + j);
          ev[0] = c4.x; ev[1] = c4.y; ev[2] = c4.z; ev[3] = c4.w;
        } else {
          ev[0] = ev[1] = ev[2] = ev[3] = 0.f;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = j + e < Ncand;
          dv[e] = ok ? drow[j + e] : 0.f;
          mv[e] = ok ? rb.cm[2 * (size_t)(j + e)] : 0.f;
          pv[e] = ok ? rb.cm[2 * (size_t)(j + e) + 1] : 0.f;
          ev[e] = (ok && !rb.pc) ? rb.cre[j + e] : 0.f;
        }
      }
      float Uv[4], Lv[4];
      bool keep[4];
      int nkeep = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float eps = margin_eps(dv[e], pv[e], mv[e], ev[e], kr, kmu, ek, rb.pc, rb.coef,
                                     rb.coef2, rb.cz);
        Uv[e] = dv[e] + eps;
        Lv[e] = dv[e] - eps;
        keep[e] = j + e < Ncand && Lv[e] <= Tp;
        nkeep += keep[e] ? 1 : 0;
      }
      // a wave reserves room for its entries with one LDS atomic
      const int incl = wave_incl_scan(nkeep);
      const int wtot = __shfl(incl, 63, 64);
      if (wtot == 0) continue;               // wave-uniform
      int wbase = 0;
      if (l == 63) wbase = atomicAdd(&sgat, wtot);
      int p = __shfl(wbase, 63, 64) + incl - nkeep;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (keep[e]) {
          if (p < mcap) {
            gpos[go + p] = j + e;
            ghi[go + p] = Uv[e];
            glo[go + p] = Lv[e];
          }
          ++p;
        }
    }
    __syncthreads();
    int m = sgat;
    if (m <= mcap && m >= K) {               // block-uniform
      // T = K-th smallest U of the gathered entries (they hold the row's K
      // smallest U); keep {L <= T} in place, in gathered order
      const float T = block_kth_by_bisection(ghi + go, m, K, ssh);
      int n = 0;
      for (int b0 = 0; b0 < m; b0 += ST) {
        const int i = b0 + tid;
        bool kp = false;
        int jv = 0;
        if (i < m) {
          jv = gpos[go + i];
          kp = glo[go + i] <= T;
        }
        int tc;
        const int pre = block_excl_scan(kp ? 1 : 0, ssh, &tc);
        if (kp) gpos[go + n + pre] = jv;
        n += tc;
      }
      __syncthreads();
      m = n;
      rescore_select_set(ks, xi, gpos + go, ghi + go, glo + go, m, K, Wc, W, Cp, L, gg, idx, dd, su,
                         sl, sj, ssh, hist, sdig);
      if (tid == 0) {
        oflag[g] = 0;
        if (st) {
          atomicAdd(&st->margin_sum, (unsigned long long)m);
          atomicMax(&st->margin_max, m);
          atomicAdd(&st->regather, 1);
        }
      }
      return;
    }
  }
full_row:
  const int BEST = UCAP;
  int cur = 0;
  float th = __int_as_float(0x7f800000), tl = 0.f;
  int tj = 0x7fffffff;
  for (int base = 0; base < Ncand; base += ST) {
    coop_rescore(ks, xi, [&](int i) { return base + i; }, wave * 2 * cpi, min(ST, Ncand - base),
                 8 * cpi, Wc, W, Cp, L, fh, fl);
    __syncthreads();
    const int j = base + tid;
    df32 v = {0.f, 0.f};
    bool adm = false;
    if (j < Ncand) {
      v.hi = fh[tid];
      v.lo = fl[tid];
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
  if (tid == 0) {
    oflag[g] = 0;
    if (st) atomicAdd(&st->overflow, 1);
  }
}

// Block matching in a local window (eq. 1 with KNN grouping, the vanilla
// BM the paper compares global matching against): one block per key; the
// candidates are the grid positions within `win` rows and columns of the
// key (clipped to the grid), every one rescored with the FP64
// arithmetic of the margin sets, and a running best list kept in LDS gives
// the first K by (distance, position).  No contraction form and no margin:
// the window is small enough to score directly.
template <int EM>
__global__ void __launch_bounds__(ST)
k_window_topk(const float* __restrict__ xi, int H, int W, int P, int D, int L,
              const float* __restrict__ A, const int32_t* __restrict__ keys, int N, int K,
              int win, int32_t* __restrict__ idx, float* __restrict__ dd) {
  __shared__ float su[UCAP];
  __shared__ float sl[UCAP];
  __shared__ int sj[UCAP];
  __shared__ int ssh[ST / 64 + 1];
  __shared__ float fh[ST], fl[ST];
  const int g = blockIdx.x;
  if (g >= N) return;                        // block-uniform
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int cpi = 64 / L;
  const int Hc = H - P + 1, Wc = W - P + 1;
  const int t = keys[g];
  const int gr = t / Wc, gc = t - gr * Wc;
  const int r0 = max(gr - win, 0), r1 = min(gr + win, Hc - 1);
  const int c0 = max(gc - win, 0), c1 = min(gc + win, Wc - 1);
  const int ww = c1 - c0 + 1;
  const int n = (r1 - r0 + 1) * ww;
  KeySlice<EM> ks;
  key_slice_load(ks, A + (size_t)g * D, D, P, H, W, L, (tid & 63) & (L - 1));
  auto pos = [&](int i) {
    const int a = i / ww;
    return (r0 + a) * Wc + c0 + (i - a * ww);
  };
  const int BEST = UCAP;
  int cur = 0;
  float th = __int_as_float(0x7f800000), tl = 0.f;
  int tj = 0x7fffffff;
  for (int base = 0; base < n; base += ST) {
    coop_rescore(ks, xi, [&](int i) { return pos(base + i); }, wave * 2 * cpi, min(ST, n - base),
                 8 * cpi, Wc, W, D / (P * P), L, fh, fl);
    __syncthreads();
    const int i = base + tid;
    df32 v = {0.f, 0.f};
    bool adm = false;
    int j = 0;
    if (i < n) {
      j = pos(i);
      v.hi = fh[tid];
      v.lo = fl[tid];
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
    if (cur > BEST - ST || base + ST >= n) {
      int n2 = 1;
      while (n2 < cur) n2 <<= 1;
      for (int q = cur + tid; q < n2; q += ST) {
        su[q] = __int_as_float(0x7f800000);
        sl[q] = 0.f;
        sj[q] = 0x7fffffff;
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
    idx[(size_t)g * K + q] = sj[q];
    dd[(size_t)g * K + q] = su[q];
  }
}

// Groups by the edge heat map (eq. 8; larger = more similar): the matcher
// wrote d = -2 H for the chunk's keys, H an exact integer in [0, hmax].
// One block per key: a histogram of H over the row (LDS), the threshold
// value H* with at least K candidates at or above it, then every wave scans
// its quarter of the row in order and keeps the candidates above H* and the
// ties at H* whose rank in position order (the ties of the lower quarters
// first) is below the number still needed; the K kept entries are sorted by
// (H desc, position asc).  Integer values: no margin, no rescoring.
constexpr int HEAT_BINS = 8193;
__global__ void __launch_bounds__(ST)
k_topk_heat(const float* __restrict__ dist, size_t ldd, int Ncand, int nk, int K, int hmax,
            const int32_t* __restrict__ kmap, int g0, int32_t* __restrict__ idx,
            float* __restrict__ dd) {
  __shared__ int hist[HEAT_BINS];
  __shared__ int seg[ST];
  __shared__ int wties[ST / 64];
  __shared__ int sth[2];
  __shared__ int sh_h[64], sh_j[64];
  __shared__ int scount;
  const int g = blockIdx.x;
  if (g >= nk) return;                       // block-uniform
  const int tid = threadIdx.x, l = lane_id(), wave = tid >> 6;
  const float* drow = dist + (size_t)g * ldd;
  auto heat = [&](int j) { return min(max((int)(-0.5f * drow[j]), 0), hmax); };
  for (int i = tid; i <= hmax; i += ST) hist[i] = 0;
  if (tid == 0) scount = 0;
  __syncthreads();
  for (int j = tid; j < Ncand; j += ST) atomicAdd(&hist[heat(j)], 1);
  __syncthreads();
  const int B = (hmax + 1 + ST - 1) / ST;
  {
    int sum = 0;
    for (int v = tid * B; v < min((tid + 1) * B, hmax + 1); ++v) sum += hist[v];
    seg[tid] = sum;
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0, t = ST - 1;
    for (; t > 0 && run + seg[t] < K; --t) run += seg[t];
    int v = min((t + 1) * B, hmax + 1) - 1;
    for (; v > t * B && run + hist[v] < K; --v) run += hist[v];
    sth[0] = v;                              // H*
    sth[1] = K - run;                        // ties at H* still needed
  }
  __syncthreads();
  const int hs = sth[0], need = sth[1];
  // each wave: a contiguous quarter of the row, in position order
  const int q4 = ((Ncand + 4 * 64 - 1) / (4 * 64)) * 64;
  const int ja = wave * q4, jb = min(Ncand, ja + q4);
  int nt = 0;
  for (int b = ja; b < jb; b += 64) {
    const int j = b + l;
    nt += __popcll(__ballot(j < jb && heat(j) == hs));
  }
  if (l == 0) wties[wave] = nt;
  __syncthreads();
  int seen = 0;
  for (int w = 0; w < wave; ++w) seen += wties[w];
  for (int b = ja; b < jb; b += 64) {
    const int j = b + l;
    const int h = j < jb ? heat(j) : -1;
    const uint64_t tie = __ballot(h == hs);
    const bool take = h > hs || (h == hs && seen + lanes_below(tie) < need);
    seen += __popcll(tie);
    if (take) {
      const int p = atomicAdd(&scount, 1);
      if (p < 64) {
        sh_h[p] = h;
        sh_j[p] = j;
      }
    }
  }
  __syncthreads();
  // K entries (the positions are distinct): sort by (H desc, j asc)
  if (wave == 0) {
    const int n = min(scount, 64);
    int hh = l < n ? sh_h[l] : -1, jj = l < n ? sh_j[l] : 0x7fffffff;
    for (int k = 2; k <= 64; k <<= 1)
      for (int s2 = k >> 1; s2 > 0; s2 >>= 1) {
        const int ho = __shfl_xor(hh, s2, 64), jo = __shfl_xor(jj, s2, 64);
        const bool before = hh > ho || (hh == ho && jj < jo);   // this entry first
        const bool up = (l & k) == 0, lower = (l & s2) == 0;
        const bool keep = (lower == up) ? before : !before;
        if (!keep) {
          hh = ho;
          jj = jo;
        }
      }
    const int gg = kmap ? kmap[g0 + g] : g0 + g;
    if (l < K) {
      idx[(size_t)gg * K + l] = jj;
      dd[(size_t)gg * K + l] = (float)hh;
    }
  }
}

}  // namespace

// The bound coefficients of margin_eps for the plan's two forms, rounded up
// so that the float values are not below the bound.
static void margin_coefs(const glr_plan* pl, int bf16, float* coef, float* coef2, float* cz) {
  const double u = 5.9604644775390625e-08;      // 2^-24
  const double b = 0.00390625;                  // 2^-8: slack of the BF16 residual term
  *coef = 0.f;
  if (bf16) {
    *coef = std::nextafter((float)(2.0 * (1.0 + b)), 1e9f);
    *coef2 = std::nextafter((float)((3.0 * pl->D + 26.0) * u), 1.f);
    *cz = std::nextafter((float)std::sqrt((double)pl->D), 1e9f);
  } else {
    *coef2 = std::nextafter((float)(2.02 * (pl->D + pl->Cp + 4.0) * u), 1.f);
    *cz = std::nextafter((float)(8.02 * pl->P * u), 1.f);
  }
}

void launch_topk_partial(const glr_plan* pl, const float* dist, const float* kmb,
                         const float* kre, const int32_t* kmap, int g0, const float* cm2,
                         const float* cre, int nk, int bf16, uint32_t* tsh, int32_t* lj,
                         float* lu, float* ll, int32_t* lcnt, hipStream_t s) {
  float coef, coef2, cz;
  margin_coefs(pl, bf16, &coef, &coef2, &cz);
  // tsh[0..nk) holds +inf here: set by the key gather at the start of every
  // match call and restored by the rescoring kernel after every scan
  // the FP32 form's margin sets stay far below the BF16 form's: a smaller
  // wave buffer (28 KB of LDS per block), no residual norms to prefetch and
  // 512-candidate steps (110 VGPRs) fit four waves per SIMD (12 % faster
  // than three with 768-candidate steps on the MRI 256^2 workload); the
  // BF16 form's 1024-entry buffers (53 KB) fit three blocks per CU, and its
  // 512-candidate steps (16 bytes per candidate, always prefetched one step
  // ahead) keep the registers within three waves per SIMD.  (768-candidate steps at two waves
  // per SIMD: 8 % slower on the 1024^2 x 24 workload; 768-entry buffers for
  // four waves overflow the range lists of the hardest keys.)
  const dim3 grid((nk + 3) / 4 * pl->n_split);
  if (bf16)
    hipLaunchKernelGGL((k_topk_partial<2, CAP, 3, true, 0>), grid, dim3(256), 0, s, dist,
                       (size_t)pl->ldd, (const float4*)kmb, kre, kmap, g0, cm2, cre, pl->Ncand,
                       pl->split_len, pl->n_split, nk, pl->K, coef, coef2, cz, tsh, lj, lu, ll,
                       lcnt);
  else
    hipLaunchKernelGGL((k_topk_partial<2, 512, 4, false, 1>), grid,
                       dim3(256), 0, s, dist, (size_t)pl->ldd, (const float4*)kmb, kre, kmap, g0,
                       cm2, cre, pl->Ncand, pl->split_len, pl->n_split, nk, pl->K, coef, coef2,
                       cz, tsh, lj, lu, ll, lcnt);
}

// Lanes per candidate of the exact rescoring: the fewest (>= 8) that keep
// every lane at <= 32 patch elements; D <= 4096 needs at most 64 per lane.
static int rescore_lanes(int D) {
  int L = 64;
  while (L > 8 && (D + L / 2 - 1) / (L / 2) <= 32) L >>= 1;
  return L;
}

template <int EM>
static void launch_select_t(const glr_plan* pl, const float* xi, const float* A,
                            const int32_t* kmap, int g0, int nk, const int32_t* lj,
                            const float* lu, const float* ll, const int32_t* lcnt, int32_t* idx,
                            float* dd, int32_t* oflag, uint32_t* tsh, int defer,
                            const BigMargin& bm, const RowBound& rb, DevStats* st, int L,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_select_rescore<EM>, dim3((nk + 3) / 4), dim3(256), 0, s, xi, pl->H, pl->W,
                     pl->P, pl->Cp, pl->D, L, A, kmap, g0, nk, pl->n_split, pl->Ncand, pl->K, lj,
                     lu, ll, lcnt, idx, dd, oflag, tsh, rb.tkey, st);
  hipLaunchKernelGGL(k_rescore_overflow<EM>, dim3(nk), dim3(ST), 0, s, xi, pl->H, pl->W, pl->P,
                     pl->Cp, pl->D, L, A, kmap, g0, pl->n_split, pl->Ncand, pl->K, defer, lj, lu,
                     ll, lcnt, oflag, bm.pos, bm.hi, bm.lo, bm.cap, idx, dd, rb, st);
}

void launch_select_rescore(const glr_plan* pl, const float* xi, const float* A,
                           const int32_t* kmap, int g0, int nk, const int32_t* lj,
                           const float* lu, const float* ll, const int32_t* lcnt, int32_t* idx,
                           float* dd, int32_t* oflag, uint32_t* tsh, int defer,
                           const BigMargin& bm, const float* dist, const float* kmb,
                           const float* kre, const float* cm2, const float* cre, int bf16,
                           float* tkey, DevStats* st, hipStream_t s) {
  RowBound rb;
  rb.dist = dist;
  rb.ldd = (size_t)pl->ldd;
  rb.km = kmb;
  rb.kre = kre;
  rb.cm = cm2;
  rb.cre = cre;
  rb.pc = bf16 ? 0 : 1;
  margin_coefs(pl, bf16, &rb.coef, &rb.coef2, &rb.cz);
  rb.tkey = tkey;
  // the slice held per lane: the smallest instance that fits (registers,
  // hence waves per SIMD, follow it)
  const int L = rescore_lanes(pl->D);
  const int em = (pl->D + L - 1) / L;
  if (em <= 16)
    launch_select_t<16>(pl, xi, A, kmap, g0, nk, lj, lu, ll, lcnt, idx, dd, oflag, tsh, defer, bm,
                        rb, st, L, s);
  else if (em <= 24)
    launch_select_t<24>(pl, xi, A, kmap, g0, nk, lj, lu, ll, lcnt, idx, dd, oflag, tsh, defer, bm,
                        rb, st, L, s);
  else if (em <= 32)
    launch_select_t<32>(pl, xi, A, kmap, g0, nk, lj, lu, ll, lcnt, idx, dd, oflag, tsh, defer, bm,
                        rb, st, L, s);
  else
    launch_select_t<64>(pl, xi, A, kmap, g0, nk, lj, lu, ll, lcnt, idx, dd, oflag, tsh, defer, bm,
                        rb, st, L, s);
}

// Append the chunk keys g0 + g with oflag[g] != 0 to klist at *kcount, in
// key order (one block).
__global__ void __launch_bounds__(1024)
k_collect_flags(const int32_t* __restrict__ oflag, int g0, int nk, int32_t* __restrict__ klist,
                int32_t* __restrict__ kcount, DevStats* st) {
  __shared__ int sh[1024 / 64 + 1];
  int base = kcount[0];
  const int start = base;
  for (int i0 = 0; i0 < nk; i0 += 1024) {
    const int i = i0 + threadIdx.x;
    const bool f = i < nk && oflag[i] != 0;
    int tot;
    const int pre = block_excl_scan(f ? 1 : 0, sh, &tot);
    if (f) klist[base + pre] = g0 + i;
    base += tot;
  }
  if (threadIdx.x == 0) {
    kcount[0] = base;
    if (st) atomicAdd(&st->rematch, base - start);
  }
}

void launch_collect_flags(const int32_t* oflag, int g0, int nk, int32_t* klist, int32_t* kcount,
                          DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_collect_flags, dim3(1), dim3(1024), 0, s, oflag, g0, nk, klist, kcount, st);
}

void launch_window_topk(const glr_plan* pl, const float* xi, const float* A, const int32_t* keys,
                        int32_t* idx, float* dd, hipStream_t s) {
  const int L = rescore_lanes(pl->D);
  const int em = (pl->D + L - 1) / L;
  if (em <= 16)
    hipLaunchKernelGGL(k_window_topk<16>, dim3(pl->N), dim3(ST), 0, s, xi, pl->H, pl->W, pl->P,
                       pl->D, L, A, keys, pl->N, pl->K, pl->window, idx, dd);
  else if (em <= 24)
    hipLaunchKernelGGL(k_window_topk<24>, dim3(pl->N), dim3(ST), 0, s, xi, pl->H, pl->W, pl->P,
                       pl->D, L, A, keys, pl->N, pl->K, pl->window, idx, dd);
  else if (em <= 32)
    hipLaunchKernelGGL(k_window_topk<32>, dim3(pl->N), dim3(ST), 0, s, xi, pl->H, pl->W, pl->P,
                       pl->D, L, A, keys, pl->N, pl->K, pl->window, idx, dd);
  else
    hipLaunchKernelGGL(k_window_topk<64>, dim3(pl->N), dim3(ST), 0, s, xi, pl->H, pl->W, pl->P,
                       pl->D, L, A, keys, pl->N, pl->K, pl->window, idx, dd);
}

void launch_topk_heat(const glr_plan* pl, const float* dist, int g0, int nk, int hmax,
                      int32_t* idx, float* dd, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_heat, dim3(nk), dim3(ST), 0, s, dist, (size_t)pl->ldd, pl->Ncand, nk,
                     pl->K, hmax, nullptr, g0, idx, dd);
}
