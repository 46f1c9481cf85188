// Aggregation of the group estimates back into the image (the grouping
// operator's adjoint for the low-rank objective of the Method section).
// Reading: every member estimate weighs 1; a pixel is the mean of all
// estimates covering it; uncovered pixels keep the pre-prior value.
//
// Deterministic: entries e = g*K + q are bucketed by position with a
// counting sort (integer counts, an exclusive scan for the CSR offsets, a
// scatter, then each bucket sorted by e), and each pixel gathers its
// covering estimates in a fixed order (slice, then dy, dx, e ascending,
// with the row segments' entry streams cut into equal slices for load
// balance); no floating-point atomics.
#include "common.h"
#include "internal.h"

namespace {

__global__ void k_count(const int32_t* __restrict__ idx, int M, int32_t* __restrict__ cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < M) atomicAdd(&cnt[idx[e]], 1);
}

constexpr int SB = 1024;          // threads of the scan blocks
constexpr int SPT = 4;            // elements per thread
constexpr int SE = SB * SPT;      // elements per scan block

// in-block exclusive scan of cnt[0..n) (4 per thread); block sums to bsum
__global__ void __launch_bounds__(SB)
k_scan_blocks(const int32_t* __restrict__ cnt, int n, int32_t* __restrict__ offs,
              int32_t* __restrict__ bsum) {
  __shared__ int sh[SB / 64 + 1];
  const int base = blockIdx.x * SE + threadIdx.x * SPT;
  int v[SPT], tot = 0;
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    v[k] = base + k < n ? cnt[base + k] : 0;
    tot += v[k];
  }
  int all;
  int pre = block_excl_scan(tot, sh, &all);
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    if (base + k < n) offs[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = all;
}

// exclusive scan of the block sums (one block; nb <= SE)
__global__ void __launch_bounds__(SB) k_scan_sums(int32_t* __restrict__ bsum, int nb) {
  __shared__ int sh[SB / 64 + 1];
  const int base = threadIdx.x * SPT;
  int v[SPT], tot = 0;
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    v[k] = base + k < nb ? bsum[base + k] : 0;
    tot += v[k];
  }
  int all;
  int pre = block_excl_scan(tot, sh, &all);
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    if (base + k < nb) bsum[base + k] = pre;
    pre += v[k];
  }
}

// offs += block prefix; cursor = offs (scatter slots)
__global__ void k_scan_add(int32_t* __restrict__ offs, int n, const int32_t* __restrict__ bsum,
                           int32_t* __restrict__ cursor) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = offs[i] + bsum[i / SE];
  offs[i] = o;
  cursor[i] = o;
}

__global__ void k_scatter(const int32_t* __restrict__ idx, int M, int32_t* __restrict__ cursor,
                          int32_t* __restrict__ ent) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < M) ent[atomicAdd(&cursor[idx[e]], 1)] = e;
}

// each bucket in ascending entry order: buckets of up to SMALL entries by one
// thread (insertion sort); longer ones are queued for k_bucket_sort_large
constexpr int SMALL = 64;
__global__ void k_bucket_sort(const int32_t* __restrict__ offs, int ncand,
                              int32_t* __restrict__ ent, int32_t* __restrict__ big,
                              int32_t* __restrict__ nbig) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncand) return;
  const int a = offs[t], b = offs[t + 1];
  if (b - a > SMALL) {
    big[atomicAdd(nbig, 1)] = t;           // queue order is irrelevant: each bucket
    return;                                // is sorted on its own
  }
  for (int i = a + 1; i < b; ++i) {
    const int v = ent[i];
    int j = i - 1;
    while (j >= a && ent[j] > v) {
      ent[j + 1] = ent[j];
      --j;
    }
    ent[j + 1] = v;
  }
}

// one block per queued bucket (grid-stride over the queue): bitonic sort in
// LDS.  A bucket holds at most one entry per group, so at most N <= LB.
constexpr int LB = 16384;
__global__ void __launch_bounds__(1024)
k_bucket_sort_large(const int32_t* __restrict__ offs, int32_t* __restrict__ ent,
                    const int32_t* __restrict__ big, const int32_t* __restrict__ nbig) {
  __shared__ int v[LB];
  const int nb = nbig[0];
  for (int k = blockIdx.x; k < nb; k += gridDim.x) {
    const int t = big[k];
    const int a = offs[t], n = offs[t + 1] - a;
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    __syncthreads();
    for (int i = threadIdx.x; i < n2; i += blockDim.x) v[i] = i < n ? ent[a + i] : 0x7fffffff;
    __syncthreads();
    for (int kk = 2; kk <= n2; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < n2; i += blockDim.x) {
          const int p = i ^ j;
          if (p > i) {
            const int x = v[i], y = v[p];
            if ((x > y) == ((i & kk) == 0)) {
              v[i] = y;
              v[p] = x;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < n; i += blockDim.x) ent[a + i] = v[i];
  }
}

constexpr int GX = 64;            // pixels per row segment
constexpr int GT = 256;           // threads per block
constexpr int CG = 32;            // channels per block (grid y covers the rest)
constexpr int LDS_FLOATS = 4096;  // staged estimate rows per chunk (16 KB: with the entry
                                  // tables 24 KB per block, six blocks per CU; 32 KB
                                  // allowed four and took 3.6 ms instead of 2.5 on the
                                  // 1024^2 x 24 workload)
constexpr int UB = 4;             // 16-byte staging loads in flight per thread
constexpr int EB = 1024;          // entries per gather slice (load balance)

// The work of a row segment (image row r, 64 pixels from c0) is the stream
// of entries that cover it: for dy = 0 .. P-1, the entries of the window of
// top-left positions (row r - dy, columns c0 - P + 1 .. c0 + GX - 1), which
// are contiguous in the CSR order.  Segments differ by orders of magnitude
// (a candidate many groups chose makes its neighbourhood heavy), so the
// stream is cut into slices of EB entries, one block each: a segment with
// one slice writes the image directly; a heavier one writes per-slice
// partial sums that k_gather_combine adds in slice order.  Every sum keeps a
// fixed order (slice, then within a slice dy, position, entry ascending): the
// output is deterministic.
__device__ __forceinline__ int seg_entries(const int32_t* __restrict__ offs, int r, int c0, int H,
                                           int W, int P) {
  const int Hc = H - P + 1, Wc = W - P + 1;
  const int tc0 = max(0, c0 - P + 1), tc1 = min(Wc - 1, c0 + GX - 1);
  int e = 0;
  for (int dy = 0; dy < P; ++dy) {
    const int tr = r - dy;
    if (tr >= 0 && tr < Hc && tc0 <= tc1) e += offs[tr * Wc + tc1 + 1] - offs[tr * Wc + tc0];
  }
  return e;
}

// slices per segment (at least one): nsub[id], id = r * nsw + segment
__global__ void k_gather_count(const int32_t* __restrict__ offs, int H, int W, int P, int nsw,
                               int32_t* __restrict__ nsub) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id > H * nsw) return;
  if (id == H * nsw) {                       // the scan's last entry: the total
    nsub[id] = 0;
    return;
  }
  const int e = seg_entries(offs, id / nsw, (id % nsw) * GX, H, W, P);
  nsub[id] = max(1, (e + EB - 1) / EB);
}

// owner[sub] = the segment of slice sub (first[]: exclusive scan of nsub)
__global__ void k_gather_expand(const int32_t* __restrict__ first, int nseg,
                                int32_t* __restrict__ owner) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nseg) return;
  for (int k = first[id]; k < first[id + 1]; ++k) owner[k] = id;
}

// One block per (slice, channel group).  Estimates are stored per member
// patch as xhat[e][dy][dx][c], so the dy-row of an entry is one contiguous
// run of P*Cp floats.  The slice's entries are staged window by window in
// LDS in chunks (all loads of a thread's batch issued before its stores) and
// every (pixel, channel) of the segment sums its covering values in the
// fixed order (dy, position, entry) ascending: the covering entries of a
// pixel are one contiguous run of the staged list, whose column is kept per
// entry.  Lanes run over the channels of a pixel, which all have the same
// trip counts.  WG: entry e weighs gw[e / K] (its group's weight) and the
// pixel is the weighted mean; otherwise every entry weighs 1.  part: per
// slice [CG][GX] sums (and weight sums), then [GX] counts, for segments of
// more than one slice.
template <bool WG>
__global__ void __launch_bounds__(GT)
k_gather(const float* __restrict__ xbar, const float* __restrict__ xhat,
         const int32_t* __restrict__ ent, const int32_t* __restrict__ offs, int Cp, int H, int W,
         int P, int D, const float* __restrict__ gw, int K, const int32_t* __restrict__ first,
         const int32_t* __restrict__ owner, int nsw, float* __restrict__ part,
         float* __restrict__ out, int32_t* __restrict__ cover) {
  __shared__ __align__(16) float lds[LDS_FLOATS];
  __shared__ int spos[GX + 17];             // window bucket starts (P <= 16), + end
  __shared__ int sent[LDS_FLOATS / 4];      // entry ids of the staged chunk
  __shared__ int scol[LDS_FLOATS / 4];      // their top-left columns
  __shared__ float swt[WG ? LDS_FLOATS / 4 : 1];   // their weights
  const int nseg = H * nsw;
  const int sub = blockIdx.x;
  if (sub >= first[nseg]) return;           // block-uniform: the grid is an upper bound
  const int id = owner[sub];
  const int k0 = sub - first[id], nsl = first[id + 1] - first[id];
  const int r = id / nsw;
  const int c0 = (id - r * nsw) * GX;
  const int cg0 = blockIdx.y * CG;
  const int ncg = min(CG, Cp - cg0);
  const int s0 = k0 * EB, s1 = s0 + EB;     // this slice of the segment's entry stream
  const int Hc = H - P + 1, Wc = W - P + 1;
  const int tid = threadIdx.x;
  const int npair = GX * ncg;
  constexpr int NPT = GX * CG / GT;         // pairs per thread (max)
  float acc[NPT];
  float wsum[NPT];
  int cnt[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    acc[k] = 0.f;
    wsum[k] = 0.f;
    cnt[k] = 0;
  }
  const int rowlen = ncg * P;               // floats staged per entry
  const int cap = min(LDS_FLOATS / rowlen, LDS_FLOATS / 4);   // entries per chunk
  // 16-byte staging when the block takes all channels (a staged row is one
  // contiguous run) and every row start and length is a multiple of 4 floats
  const bool vec4 = ncg == Cp && (rowlen & 3) == 0 && (D & 3) == 0;
  const int tc0 = max(0, c0 - P + 1);
  const int tc1 = min(Wc - 1, c0 + GX - 1);
  int pos0 = 0;                             // stream offset of this window
  for (int dy = 0; dy < P; ++dy) {
    const int tr = r - dy;
    if (tr < 0 || tr >= Hc || tc0 > tc1) continue;      // block-uniform
    const int nwin = tc1 - tc0 + 1;
    __syncthreads();                                     // previous users of spos / lds
    for (int i = tid; i <= nwin; i += GT) spos[i] = offs[tr * Wc + tc0 + i];
    __syncthreads();
    const int wa = spos[0], wb = spos[nwin];
    // the part of this window inside the slice
    const int ea = max(wa, wa + s0 - pos0), eb = min(wb, wa + s1 - pos0);
    pos0 += wb - wa;
    for (int ia = ea; ia < eb; ia += cap) {
      const int ib = min(eb, ia + cap);
      const int nrow = ib - ia;
      __syncthreads();
      for (int i = tid; i < nrow; i += GT) {
        const int e = ent[ia + i];
        sent[i] = e;
        if (WG) swt[i] = gw[e / K];
      }
      for (int k = tid; k < nwin; k += GT) {
        const int i0 = max(spos[k], ia), i1 = min(spos[k + 1], ib);
        for (int i = i0; i < i1; ++i) scol[i - ia] = tc0 + k;
      }
      __syncthreads();
      // LDS row i holds [dx][c - cg0]
      {
        const size_t roff = (size_t)dy * P * Cp;
        if (vec4) {
          const int r4 = rowlen >> 2;
          const int nw = nrow * r4;
          for (int base = tid; base < nw; base += GT * UB) {
            // every load is issued (past the end it re-reads the last word)
            // before the stores, so UB loads per thread are in flight
            float4 v[UB];
            int dst[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int q = min(base + u * GT, nw - 1);
              const int i = q / r4, w = q - i * r4;
              v[u] = *reinterpret_cast<const float4*>(xhat + (size_t)sent[i] * D + roff + 4 * w);
              dst[u] = i * rowlen + 4 * w;
            }
#pragma unroll
            for (int u = 0; u < UB; ++u)
              if (base + u * GT < nw) *reinterpret_cast<float4*>(lds + dst[u]) = v[u];
          }
        } else {
          const int nw = nrow * rowlen;
          for (int base = tid; base < nw; base += GT * UB) {
            float v[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
              const int q = min(base + u * GT, nw - 1);
              const int i = q / rowlen, w = q - i * rowlen;
              const int dx = w / ncg, c = w - dx * ncg;
              v[u] = xhat[(size_t)sent[i] * D + roff + (size_t)dx * Cp + cg0 + c];
            }
#pragma unroll
            for (int u = 0; u < UB; ++u)
              if (base + u * GT < nw) lds[base + u * GT] = v[u];
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int p = tid + k * GT;
        if (p < npair) {
          const int px = p / ncg, ch = p - px * ncg;
          const int c = c0 + px;
          const int lo = max(tc0, c - P + 1), hi = min(tc1, c);
          if (c < W && lo <= hi) {
            const int b0 = max(spos[lo - tc0], ia), b1 = min(spos[hi - tc0 + 1], ib);
            float a = acc[k];
            if (WG) {
              float ws = wsum[k];
              for (int i = b0; i < b1; ++i) {
                const float w = swt[i - ia];
                a = fmaf(w, lds[(i - ia) * rowlen + (c - scol[i - ia]) * ncg + ch], a);
                ws += w;
              }
              wsum[k] = ws;
            } else {
              for (int i = b0; i < b1; ++i)
                a += lds[(i - ia) * rowlen + (c - scol[i - ia]) * ncg + ch];
            }
            acc[k] = a;
            cnt[k] += max(b1 - b0, 0);
          }
        }
      }
    }
  }
  const size_t HW = (size_t)H * W;
  if (nsl == 1) {
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int p = tid + k * GT;
      if (p < npair) {
        const int px = p / ncg, ch = p - px * ncg;
        const int c = c0 + px;
        if (c < W) {
          const int n = cnt[k];
          if (cover && cg0 == 0 && ch == 0) cover[(size_t)r * W + c] = n;
          const size_t o = (size_t)(cg0 + ch) * HW + (size_t)r * W + c;
          out[o] = n ? acc[k] / (WG ? wsum[k] : (float)n) : xbar[o];
        }
      }
    }
    return;
  }
  // partial sums of this slice: [ch][px] sums, [ch][px] weight sums, [px] counts
  float* ps = part + ((size_t)sub * gridDim.y + blockIdx.y) * (size_t)GX * (2 * CG + 1);
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int p = tid + k * GT;
    if (p < npair) {
      const int px = p / ncg, ch = p - px * ncg;
      ps[ch * GX + px] = acc[k];
      if (WG) ps[(CG + ch) * GX + px] = wsum[k];
      if (ch == 0) ps[2 * CG * GX + px] = __int_as_float(cnt[k]);
    }
  }
}

// Segments of more than one slice: the slices' partial sums added in slice
// order, then the mean (or weighted mean).  One block per (segment, channel
// group); single-slice segments exit.
template <bool WG>
__global__ void __launch_bounds__(GT)
k_gather_combine(const float* __restrict__ xbar, const int32_t* __restrict__ first, int nsw,
                 int Cp, int H, int W, const float* __restrict__ part, float* __restrict__ out,
                 int32_t* __restrict__ cover) {
  const int id = blockIdx.x;
  const int f0 = first[id], nsl = first[id + 1] - f0;
  if (nsl == 1) return;                     // block-uniform
  const int r = id / nsw;
  const int c0 = (id - r * nsw) * GX;
  const int cg0 = blockIdx.y * CG;
  const int ncg = min(CG, Cp - cg0);
  const size_t HW = (size_t)H * W;
  const size_t stride = (size_t)gridDim.y * GX * (2 * CG + 1);
  for (int p = threadIdx.x; p < GX * ncg; p += GT) {
    const int px = p / ncg, ch = p - px * ncg;
    const int c = c0 + px;
    if (c >= W) continue;
    const float* ps = part + ((size_t)f0 * gridDim.y + blockIdx.y) * (size_t)GX * (2 * CG + 1);
    float a = 0.f, ws = 0.f;
    int n = 0;
    for (int k = 0; k < nsl; ++k, ps += stride) {
      a += ps[ch * GX + px];
      if (WG) ws += ps[(CG + ch) * GX + px];
      n += __float_as_int(ps[2 * CG * GX + px]);
    }
    if (cover && cg0 == 0 && ch == 0) cover[(size_t)r * W + c] = n;
    const size_t o = (size_t)(cg0 + ch) * HW + (size_t)r * W + c;
    out[o] = n ? a / (WG ? ws : (float)n) : xbar[o];
  }
}

}  // namespace

static int gather_nsw(const glr_plan* pl) { return (pl->W + GX - 1) / GX; }
static size_t gather_max_slices(const glr_plan* pl) {
  // every entry lies in the streams of at most P rows x 2 segments (P < GX)
  const size_t nseg = (size_t)pl->H * gather_nsw(pl);
  return nseg + (2 * (size_t)pl->P * pl->M + EB - 1) / EB;
}

size_t agg_gather_ints(const glr_plan* pl) {
  const size_t n = (size_t)pl->H * gather_nsw(pl) + 1;
  // slice counts [n], their scan [n], scan block sums, slice owners
  return 2 * ((n + 63) / 64 * 64) + (n + SE - 1) / SE + 64 + gather_max_slices(pl);
}

size_t agg_gather_part_floats(const glr_plan* pl) {
  return gather_max_slices(pl) * (size_t)((pl->Cp + CG - 1) / CG) * GX * (2 * CG + 1);
}

void launch_aggregate(const glr_plan* pl, const float* xbar, const int32_t* idx,
                      const float* xhat, const float* gw, int32_t* sortbuf, int32_t* offs,
                      int32_t* gplan, float* gpart, float* out, int32_t* cover, hipStream_t s) {
  const int M = pl->M, n = pl->Ncand + 1;
  int32_t* ent = sortbuf;                       // [M]
  int32_t* cnt = sortbuf + pl->M2;              // [Ncand + 1], later the scatter cursor
  int32_t* bsum = cnt + ((size_t)n + 63) / 64 * 64;
  const int nb = (n + SE - 1) / SE;
  hipLaunchKernelGGL(k_count, dim3((M + 255) / 256), dim3(256), 0, s, idx, M, cnt);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SB), 0, s, cnt, n, offs, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SB), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, offs, n, bsum, cnt);
  hipLaunchKernelGGL(k_scatter, dim3((M + 255) / 256), dim3(256), 0, s, idx, M, cnt, ent);
  int32_t* nbig = bsum + nb;                    // [1] queue length, then the queue
  int32_t* big = nbig + 1;
  hipLaunchKernelGGL(k_bucket_sort, dim3((pl->Ncand + 255) / 256), dim3(256), 0, s, offs,
                     pl->Ncand, ent, big, nbig);
  hipLaunchKernelGGL(k_bucket_sort_large, dim3(256), dim3(1024), 0, s, offs, ent, big, nbig);
  // slices: counts per segment, their exclusive scan, the owner of each slice
  const int nsw = gather_nsw(pl), nseg = pl->H * nsw, ns1 = nseg + 1;
  int32_t* gn = gplan;                                   // [ns1] slices per segment
  int32_t* gfirst = gn + ((size_t)ns1 + 63) / 64 * 64;   // [ns1] first slice of each
  int32_t* gbs = gfirst + ((size_t)ns1 + 63) / 64 * 64;  // scan block sums
  const int nbs = (ns1 + SE - 1) / SE;
  int32_t* gowner = gbs + nbs + 64;
  hipLaunchKernelGGL(k_gather_count, dim3((ns1 + 255) / 256), dim3(256), 0, s, offs, pl->H,
                     pl->W, pl->P, nsw, gn);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nbs), dim3(SB), 0, s, gn, ns1, gfirst, gbs);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SB), 0, s, gbs, nbs);
  hipLaunchKernelGGL(k_scan_add, dim3((ns1 + 255) / 256), dim3(256), 0, s, gfirst, ns1, gbs, gn);
  hipLaunchKernelGGL(k_gather_expand, dim3((nseg + 255) / 256), dim3(256), 0, s, gfirst, nseg,
                     gowner);
  const int ncg = (pl->Cp + CG - 1) / CG;
  const dim3 grid((unsigned)gather_max_slices(pl), ncg);
  const dim3 cgrid((unsigned)nseg, ncg);
  if (gw) {
    hipLaunchKernelGGL(k_gather<true>, grid, dim3(GT), 0, s, xbar, xhat, ent, offs, pl->Cp,
                       pl->H, pl->W, pl->P, pl->D, gw, pl->K, gfirst, gowner, nsw, gpart, out,
                       cover);
    hipLaunchKernelGGL(k_gather_combine<true>, cgrid, dim3(GT), 0, s, xbar, gfirst, nsw, pl->Cp,
                       pl->H, pl->W, gpart, out, cover);
  } else {
    hipLaunchKernelGGL(k_gather<false>, grid, dim3(GT), 0, s, xbar, xhat, ent, offs, pl->Cp,
                       pl->H, pl->W, pl->P, pl->D, gw, pl->K, gfirst, gowner, nsw, gpart, out,
                       cover);
    hipLaunchKernelGGL(k_gather_combine<false>, cgrid, dim3(GT), 0, s, xbar, gfirst, nsw, pl->Cp,
                       pl->H, pl->W, gpart, out, cover);
  }
}
