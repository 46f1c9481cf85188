// Host-side plan and the kernel launchers of libglr (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <utility>
#include <vector>

#include "../../include/glr.h"

// Device-side counters kept in the workspace.
struct DevStats {
  unsigned long long margin_sum;
  unsigned long long steps;
  unsigned long long sweeps_sum;
  int margin_max;
  int overflow;
  int sweeps_max;
  int keys_selected;
  int rematch;
  int regather;                  // keys whose margin set was re-derived from the distance row
};

#define GLR_STAGE_SLOTS 12

// Byte offsets of the workspace buffers (all 256-aligned).
struct WsLayout {
  size_t xp, xo;                 // planar copies of input / output (complex data)
  size_t xi;                     // channel-interleaved copy [H][W][Cp] for the group loads
  size_t q, gxx, gyy, gxy, r25;  // detector
  size_t cflag, slist, sval;     // detector candidate flags / survivor list, scores
  size_t keys;                   // detected keys [N]
  size_t A;                      // key matrix [N][D] f32
  size_t kmb, cmeta, cm2;        // BF16 form: centred key / candidate metadata (one mean)
  size_t kre, cre;               // BF16 form: key / candidate BF16 rounding residual norms
  size_t E, eq, egx, emax;       // edge-map score: maps, quantised channels, gradients, max
  size_t Ac, kn, kc, pn, pc, pq; // FP32 form: channel-centred keys and metadata
  size_t Ab;                     // BF16 form: centred keys in the BF16 slice layout
  size_t tsh;                    // per-key shared threshold bound [n_chunk]
  size_t tkey;                   // the bound each key's scan left, float [n_chunk]
  size_t klist, kcount;          // BF16 form: keys re-matched in FP32 [N], their count
  size_t bpos, bhi, blo;         // large-margin scratch [n_chunk][mcap]
  size_t cnn_ws, xcnn, xglr, cover, subkeys, sigv, jpart, jdelta;  // surrogate and judge
  size_t dist;                   // distance chunk [n_chunk][ldd]
  size_t lj, lu, ll, lcnt, oflag; // partial top-K lists, per-key overflow flags
  size_t idx, dd;                // groups [N][K], distances [N][K]
  size_t xhat, sv;               // group estimates [N][D][K]; singular values
  size_t gw;                     // per-group aggregation weights [N] (GLR_AGG_RANK)
  size_t gplan, gpart;           // aggregation: slice table, partial sums
  size_t yk, ipart, isig;        // inner WNNM iterations: y^(k), partial sums, sigma_k
  size_t pairs, offs;            // aggregation sort keys, CSR offsets
  size_t cplx_a, cplx_b;         // complex scratch (FFT / ADMM)
  size_t red;                    // small reduction scratch
  size_t stats;                  // DevStats
  size_t total;
};

struct glr_plan {
  int modality, H, W, C, Cp, is_complex;
  const uint8_t* mask;
  int P, N, K, T, solver, precision, timing;
  int n_corner;                   // corner exemplars (N counts the uniform grid too)
  int exemplars, uniform_step, search, window;
  int score;                      // GLR_SCORE_L2 | GLR_SCORE_EDGE
  int agg_weights;                // GLR_AGG_UNIFORM | GLR_AGG_RANK
  int wnnm_iters;                 // inner WNNM iterations per prior step (1: one shrinkage)
  float wnnm_delta, wnnm_lambda;  // their regularisation step and noise re-estimate factor
  bool lowrank_complex;           // complex data shrunk as complex groups
  int Ce;                         // edge-map channels per real channel group (score EDGE)
  float rho, wnnm_c, wnnm_eps;
  std::vector<float> sigma;
  // derived sizes
  int Hc, Wc, Ncand, D, ldd;
  int n_chunk, n_split, split_len;
  int mcap;                       // large-margin capacity per key
  int M, M2;                      // aggregation entries (N*K) and power of two
  WsLayout ws;
  hipStream_t last_stream;
  const void* stats_ws;           // workspace whose stats region is initialised
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;   // timing event pairs
  std::vector<int> ev_stage;      // stage of each recorded pair
  size_t ev_used;                 // pairs recorded since the last read
  // host-side timing accumulators (ms), one per stage
  double ms[GLR_STAGE_SLOTS];
  // CNN surrogate
  int surrogate, judge_stride;
  float surrogate_frac, judge_delta_max;
  const void* cnn_packed;
  long long sur_steps, fallback_steps;
  float judge_delta_last;
  long long match_launches;
  long long rematch_launches;     // FP32 re-match launches of the BF16 form
};

// Sets the thread-local detail string of glr_last_error_message(); returns s.
glr_status glr_set_error(glr_status s, const char* msg);

// list capacity of one top-K split (entries) and of the union per key
#define GLR_SPLIT_CAP 1024
#define GLR_UNION_CAP 4096

// ------------------------------------------------------------------ launchers
// ops.hip
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void launch_cacti_forward(const float* x, const uint8_t* m, float* y, int F, int HW, hipStream_t s);
void launch_cacti_adjoint(const float* y, const uint8_t* m, float* x, int F, int HW, hipStream_t s);
void launch_cacti_init(const float* y, const uint8_t* m, float* x, int F, int HW, hipStream_t s);
// yacc (nullable): accelerated GAP's accumulated measurement, updated when wacc
void launch_cacti_gap(const float* x, const float* y, const uint8_t* m, float* xo, int F, int HW,
                      float* yacc, int wacc, hipStream_t s);
void launch_msfa_forward(const float* x, float* y, int H, int W, hipStream_t s);
void launch_msfa_adjoint(const float* y, float* x, int H, int W, hipStream_t s);
void launch_msfa_init(const float* y, float* x, int H, int W, hipStream_t s);
void launch_msfa_gap(const float* x, const float* y, float* xo, int H, int W, float* yacc,
                     int wacc, hipStream_t s);
// Optional fusions of the 2-D FFT (see k_fft_rows / k_fft_cols): the rows pass
// transforms in + beta in2; the columns pass applies the ADMM k-space update
// (ky, lines, rho) and/or writes vp = planar(result + pu).
struct FftFuse {
  const float2* in2 = nullptr;
  float beta = 0.f;
  const float2* ky = nullptr;
  const uint8_t* lines = nullptr;
  float rho = 0.f;
  const float2* pu = nullptr;
  float* vp = nullptr;
};
void launch_fft2d(const float2* in, float2* out, int H, int W, int inverse, hipStream_t s,
                  const FftFuse* f = nullptr);
void launch_kspace_mask(const float2* in, const uint8_t* lines, float2* out, int H, int W,
                        hipStream_t s);
void launch_cplx_axpby(const float2* a, const float2* b, float2* out, float alpha, float beta,
                       int n, hipStream_t s);
// z = complex form of the planar zp, then u += x - z
void launch_admm_dual(float2* u, const float2* x, const float* zp, float2* z, int n,
                      hipStream_t s);
void launch_to_planar(const float2* z, float* p, int n, hipStream_t s);
void launch_from_planar(const float* p, float2* z, int n, hipStream_t s);

// detect.hip
// the n_sel best corner keys (n_sel <= N_cand)
void launch_detect(const glr_plan* pl, const float* xp, char* ws, int32_t* keys, int n_sel,
                   hipStream_t s);
// binary edge maps E [4 Ce][H][W] (0/1 floats) of the matching score of
// eq. 6-8, Ce = C' for real data, 1 for complex data
void launch_edges(const glr_plan* pl, const float* xp, char* ws, float* E, hipStream_t s);
// the uniform exemplar grid of interval step (ceil(Hc/step) ceil(Wc/step) keys)
void launch_uniform_keys(const glr_plan* pl, int32_t* keys, int step, hipStream_t s);

// match.hip
// also resets the top-K scan's per-key bounds tsh[0..min(n_chunk, N)) to +inf
void launch_gather_keys(const glr_plan* pl, const float* xp, const int32_t* keys, float* A,
                        uint32_t* tsh, hipStream_t s);
int bf16_key_row(int P);     // bf16 values per key and channel in the BF16 key layout
// kmb[N] float4 (||a||^2, mu_k, sum a, ||a||), kre[N] ||a - bf16(a)||; Ab
// (BF16 key slices) may be null.  raw != 0: no centring and zero norm terms
// (the BF16 matcher then returns -2 <k, p>: the edge-map score)
void launch_key_meta(const glr_plan* pl, const float* A, uint16_t* Ab, float* kmb, float* kre,
                     int raw, hipStream_t s);
// cmeta[Ncand] float4 (mu, ||pbar||^2, ||pbar||, sum pbar); cm2[Ncand] float2
// (mu, ||pbar||); cre[Ncand] ||pbar - bf16(pbar)||; raw as above
void launch_cand_meta(const glr_plan* pl, const float* xp, float* cmeta, float* cm2, float* cre,
                      int raw, hipStream_t s);
// FP32 form, channel-centred: Ac[N][D] (a~), kn[N] float4 (||a~||^2, h_k, 0, ||a~||),
// kc[N][Cp] (fl(P mu_kc)); pn[Ncand] (||p~||^2), pc[Cp][Ncand] float2
// (mu_pc, fl(P mu_pc)), pq[Ncand] float2 (h_p, ||p~||)
void launch_key_meta_pc(const glr_plan* pl, const float* A, float* Ac, float* kn, float* kc,
                        hipStream_t s);
void launch_cand_meta_pc(const glr_plan* pl, const float* xp, float* pn, float* pc, float* pq,
                         hipStream_t s);
// keys: rows g0..g0+nk of Ac, or rows kmap[g0..g0+nk) when kmap is not null
void launch_match_f32(const glr_plan* pl, const float* xp, const float* Ac, const float* kn,
                      const float* kc, const float* pn, const float* pc, const int32_t* kmap,
                      int g0, int nk, float* dist, hipStream_t s);
void launch_match_bf16(const glr_plan* pl, const float* xp, const uint16_t* Ab, const float* kmb,
                       const float* cmeta, int g0, int nk, float* dist, hipStream_t s);

// topk.hip
// bf16 = 1: BF16 form (kmb/cm2 and the residual norms kre/cre of
// launch_key_meta/launch_cand_meta); 0: the channel-centred FP32 form
// (kn/pq of launch_key_meta_pc/launch_cand_meta_pc; kre, cre null)
void launch_topk_partial(const glr_plan* pl, const float* dist, const float* kmb,
                         const float* kre, const int32_t* kmap, int g0, const float* cm2,
                         const float* cre, int nk, int bf16, uint32_t* tsh, int32_t* lj,
                         float* lu, float* ll, int32_t* lcnt, hipStream_t s);
// Global scratch of the large-margin path: per chunk key, cap entries of
// position, rescored hi and lo.
struct BigMargin {
  int32_t* pos;
  float* hi;
  float* lo;
  int cap;
};
// What the large-margin path needs to re-derive a key's margin set from its
// distance row when a range list overflowed: the chunk's d~ rows and the key
// and candidate bound terms the scan used (same arguments as
// launch_topk_partial), and tkey, where the select kernel leaves the bound
// each key's scan published.
// Padding (entries) after the arrays the top-K stage streams in chunks:
// the distance chunk, the candidate bound terms (cm2, cre, pq).  Its reads
// reach at most two chunks (2 x 768 candidates) past a range's end.
constexpr int SPAD = 2048;
struct RowBound {
  const float* dist;
  size_t ldd;
  const float* km;
  const float* kre;
  const float* cm;
  const float* cre;
  int pc;
  float coef, coef2, cz;
  float* tkey;
};
// xi: the channel-interleaved copy of the image (launch_interleave)
void launch_select_rescore(const glr_plan* pl, const float* xi, const float* A,
                           const int32_t* kmap, int g0, int nk, const int32_t* lj,
                           const float* lu, const float* ll, const int32_t* lcnt, int32_t* idx,
                           float* dd, int32_t* oflag, uint32_t* tsh, int defer,
                           const BigMargin& bm, const float* dist, const float* kmb,
                           const float* kre, const float* cm2, const float* cre, int bf16,
                           float* tkey, DevStats* st, hipStream_t s);
void launch_collect_flags(const int32_t* oflag, int g0, int nk, int32_t* klist, int32_t* kcount,
                          DevStats* st, hipStream_t s);
// groups of the edge heat map from a chunk of d = -2 H (H <= hmax <= 8192):
// the K largest H per key, lowest position first among ties
void launch_topk_heat(const glr_plan* pl, const float* dist, int g0, int nk, int hmax,
                      int32_t* idx, float* dd, hipStream_t s);
// block matching in a (2 window + 1)^2 window around each key: exact groups
// (compensated distances, (distance, position) order) for keys[0..N)
// xi: the channel-interleaved copy of the image (launch_interleave)
void launch_window_topk(const glr_plan* pl, const float* xi, const float* A, const int32_t* keys,
                        int32_t* idx, float* dd, hipStream_t s);

// lowrank.hip
// zbuf[0..zn) is set to zero (nullable); bump != 0 counts a prior step
// xi: scratch [H][W][Cp] for the channel-interleaved copy of xp
// xi[(r*W + c)*Cp + ch] = xp[ch*H*W + r*W + c]: the channel-interleaved copy
// of a planar image that the low-rank step and the exact rescoring read
void launch_interleave(const glr_plan* pl, const float* xp, float* xi, hipStream_t s);
// xi: the image's channel-interleaved copy (launch_interleave), made by the caller
void launch_wnnm(const glr_plan* pl, const float* xi, const int32_t* idx, float sigma,
                 float* xhat, float* sv, DevStats* st, int32_t* zbuf, int zn, int bump,
                 float* gw, const float* sigp, hipStream_t s);
// one inner WNNM iteration's regularisation: ynew = x + delta (xbar - yprev)
// (ynew may be yprev), and sig_out = lambda sqrt(max(sigma^2 - mean((xbar -
// ynew)^2), 0)) on the device; part holds 1024 doubles
void launch_inner_update(const float* xbar, const float* x, const float* yprev, float* ynew,
                         size_t n, float delta, float sigma, float lambda, double* part,
                         float* sig_out, hipStream_t s);

// aggregate.hip
// sortbuf: aggregation sort scratch (agg_sort_ints(pl) int32); offs [Ncand + 1];
// cover (nullable): per-pixel count of covering estimates [H][W]
// The counters at agg_zero_range(pl, sortbuf) must be zero on entry.
// gw: per-group weights [N] (weighted mean), or null (plain mean)
// gplan (agg_gather_ints(pl) int32) and gpart (agg_gather_part_floats(pl)):
// the load-balanced gather's slice table and partial sums
void launch_aggregate(const glr_plan* pl, const float* xbar, const int32_t* idx,
                      const float* xhat, const float* gw, int32_t* sortbuf, int32_t* offs,
                      int32_t* gplan, float* gpart, float* out, int32_t* cover, hipStream_t s);
size_t agg_gather_ints(const glr_plan* pl);
size_t agg_gather_part_floats(const glr_plan* pl);
// counts, block sums and queue length of the aggregation sort: one contiguous
// range of sortbuf (returns its start; *n its length)
inline int32_t* agg_zero_range(const glr_plan* pl, int32_t* sortbuf, int* n) {
  const size_t nc = (size_t)pl->Ncand + 1;
  *n = (int)((nc + 63) / 64 * 64 + (nc + 4095) / 4096 + 1);
  return sortbuf + pl->M2;
}
inline size_t agg_sort_ints(const glr_plan* pl) {
  const size_t n = (size_t)pl->Ncand + 1;
  // entries [M2], counts/cursor [n], block sums, queue length, large-bucket queue
  return (size_t)pl->M2 + (n + 63) / 64 * 64 + (n + 4095) / 4096 + 1 + (size_t)pl->M / 65 + 64;
}

// cnn.hip
size_t cnn_packed_bytes();
int cnn_param_count();
size_t cnn_workspace_bytes(int B, int h, int w, int train);
void cnn_pack(const float* params, void* packed, hipStream_t s);
void cnn_forward(const void* packed, const float* x, const float* sigma, float* out, int B, int h,
                 int w, void* ws, hipStream_t s);
void cnn_loss_grad(const void* packed, const float* x, const float* sigma, const float* tgt,
                   int B, int h, int w, float* loss, float* grad, float* out_tmp, void* ws,
                   hipStream_t s);
void cnn_adam(float* params, float* m, float* v, const float* grad, int step, float lr,
              void* packed, hipStream_t s);

// judge (ops.hip)
void launch_fill_f32(float* p, float v, size_t n, hipStream_t s);
void launch_stride_keys(const int32_t* keys, int n, int stride, int32_t* sub, hipStream_t s);
// delta = ||(a - b)|cov|| / ||b|cov|| over planar [C][HW] (inf if a is not finite or den = 0)
void launch_judge(const float* a, const float* b, const int32_t* cover, int C, int HW,
                  float* part, float* delta, hipStream_t s);
