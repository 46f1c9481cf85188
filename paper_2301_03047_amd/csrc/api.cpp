// libglr host layer: plans, validation, workspace layout and the stream-ordered
// launch sequences behind the C ABI declared in include/glr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.h"

namespace {

thread_local std::string g_err;

glr_status fail(glr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
glr_status fail(glr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

glr_status check_hip(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GLR_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
  return GLR_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = up(off + (bytes ? bytes : 1), 256);
    return o;
  }
};

#define REQUIRE_PTR(p)                                                         \
  do {                                                                         \
    if (!(p)) return fail(GLR_ERR_INVALID_ARG, "%s: %s is NULL", __func__, #p); \
    if (!aligned((p), 16))                                                     \
      return fail(GLR_ERR_ALIGNMENT, "%s: %s not 16-byte aligned", __func__, #p); \
  } while (0)

glr_status check_plan_ws(const glr_plan* pl, const void* ws, const char* fn) {
  if (!pl) return fail(GLR_ERR_INVALID_ARG, "%s: plan is NULL", fn);
  if (!ws) return fail(GLR_ERR_INVALID_ARG, "%s: workspace is NULL", fn);
  if (!aligned(ws, 256)) return fail(GLR_ERR_ALIGNMENT, "%s: workspace not 256-byte aligned", fn);
  return GLR_OK;
}

// Stats live in the workspace: clear them the first time a workspace is seen.
// (The top-K scan's per-key bounds are reset by every match call itself.)
void ensure_stats(glr_plan* pl, char* ws, hipStream_t s) {
  if (pl->stats_ws != ws) {
    launch_fill_u32((uint32_t*)(ws + pl->ws.stats), 0u, sizeof(DevStats) / 4, s);
    pl->stats_ws = ws;
  }
  pl->last_stream = s;
}

// Optional per-stage timing: an event pair is recorded around each stage on
// the caller's stream (no host synchronisation); glr_read_stats() waits for
// the stream and folds the elapsed times into per-stage totals.
struct StageTimer {
  glr_plan* pl;
  hipStream_t s;
  int stage;
  size_t slot;
  StageTimer(glr_plan* p, hipStream_t st, int stg) : pl(p), s(st), stage(stg), slot(0) {
    if (!pl->timing) return;
    slot = pl->ev_used;
    if (slot == pl->ev_pool.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      hipEventCreate(&a);
      hipEventCreate(&b);
      pl->ev_pool.push_back({a, b});
      pl->ev_stage.push_back(0);
    }
    pl->ev_stage[slot] = stage;
    pl->ev_used++;
    hipEventRecord(pl->ev_pool[slot].first, s);
  }
  ~StageTimer() {
    if (pl->timing) hipEventRecord(pl->ev_pool[slot].second, s);
  }
};

void fold_timers(glr_plan* pl) {
  for (size_t i = 0; i < pl->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pl->ev_pool[i].first, pl->ev_pool[i].second) == hipSuccess)
      pl->ms[pl->ev_stage[i]] += ms;
  }
  pl->ev_used = 0;
}
enum { T_DETECT = 0, T_MATCH, T_TOPK, T_SELECT, T_LOWRANK, T_AGG, T_DATA, T_NORMS, T_CNN, T_JUDGE,
       T_REMATCH, T_COUNT };
static_assert(T_COUNT <= GLR_STAGE_SLOTS, "stage timer slots");

// ---------------------------------------------------------------- prior step
// The N exemplar keys of one prior step (corner detection, the uniform grid,
// or corners followed by the grid of three times the interval).
void launch_exemplars(const glr_plan* pl, const float* xp, char* ws, int32_t* keys,
                      hipStream_t s) {
  if (pl->exemplars != GLR_EXEMPLAR_UNIFORM) launch_detect(pl, xp, ws, keys, pl->n_corner, s);
  if (pl->exemplars == GLR_EXEMPLAR_UNIFORM) launch_uniform_keys(pl, keys, pl->uniform_step, s);
  if (pl->exemplars == GLR_EXEMPLAR_CORNER_UNIFORM)
    launch_uniform_keys(pl, keys + pl->n_corner, 3 * pl->uniform_step, s);
}

// xp: planar [Cp][H][W]; xo: planar output; keys_in: optional caller keys.
// idx_out/dd_out: where groups go (may be the workspace buffers).
glr_status match_stage(glr_plan* pl, const float* xp, const int32_t* keys, int32_t* idx_out,
                       float* dd_out, char* ws, hipStream_t s) {
  float* A = (float*)(ws + pl->ws.A);
  float* kmb = (float*)(ws + pl->ws.kmb);
  float* cmeta = (float*)(ws + pl->ws.cmeta);
  float* cm2 = (float*)(ws + pl->ws.cm2);
  float* kre = (float*)(ws + pl->ws.kre);
  float* cre = (float*)(ws + pl->ws.cre);
  uint16_t* Ab = (uint16_t*)(ws + pl->ws.Ab);
  float* Ac = (float*)(ws + pl->ws.Ac);
  float* kn = (float*)(ws + pl->ws.kn);
  float* kc = (float*)(ws + pl->ws.kc);
  float* pn = (float*)(ws + pl->ws.pn);
  float* pc = (float*)(ws + pl->ws.pc);
  float* pq = (float*)(ws + pl->ws.pq);
  uint32_t* tsh = (uint32_t*)(ws + pl->ws.tsh);
  float* tkey = (float*)(ws + pl->ws.tkey);
  float* dist = (float*)(ws + pl->ws.dist);
  int32_t* lj = (int32_t*)(ws + pl->ws.lj);
  float* lu = (float*)(ws + pl->ws.lu);
  float* ll = (float*)(ws + pl->ws.ll);
  int32_t* lcnt = (int32_t*)(ws + pl->ws.lcnt);
  int32_t* oflag = (int32_t*)(ws + pl->ws.oflag);
  int32_t* klist = (int32_t*)(ws + pl->ws.klist);
  int32_t* kcount = (int32_t*)(ws + pl->ws.kcount);
  DevStats* st = (DevStats*)(ws + pl->ws.stats);
  const bool bf = pl->precision == GLR_PREC_BF16_RESCORE;
  const BigMargin bm = {(int32_t*)(ws + pl->ws.bpos), (float*)(ws + pl->ws.bhi),
                        (float*)(ws + pl->ws.blo), pl->mcap};
  if (pl->score == GLR_SCORE_EDGE) {
    // the stacked binary maps are matched as an image of 4 Ce channels with
    // the BF16 matcher in raw form (d = -2 H exactly), then grouped by the
    // exact integer top-K of the heat values
    float* E = (float*)(ws + pl->ws.E);
    const int Cp0 = pl->Cp, D0 = pl->D;
    const int De = 4 * pl->Ce * pl->P * pl->P;
    auto as_maps = [&](bool on) {
      pl->Cp = on ? 4 * pl->Ce : Cp0;
      pl->D = on ? De : D0;
    };
    {
      StageTimer t(pl, s, T_NORMS);
      launch_edges(pl, xp, ws, E, s);
      as_maps(true);
      launch_gather_keys(pl, E, keys, A, tsh, s);
      launch_key_meta(pl, A, Ab, kmb, kre, 1, s);
      launch_cand_meta(pl, E, cmeta, cm2, cre, 1, s);
      as_maps(false);
    }
    for (int g0 = 0; g0 < pl->N; g0 += pl->n_chunk) {
      const int nk = std::min(pl->n_chunk, pl->N - g0);
      {
        StageTimer t(pl, s, T_MATCH);
        as_maps(true);
        launch_match_bf16(pl, E, Ab, kmb, cmeta, g0, nk, dist, s);
        as_maps(false);
        if (pl->timing) pl->match_launches++;
      }
      {
        StageTimer t(pl, s, T_TOPK);
        launch_topk_heat(pl, dist, g0, nk, De, idx_out, dd_out, s);
      }
    }
    return check_hip("glr_match_topk");
  }
  // the exact rescoring reads the channel-interleaved copy of the image
  float* xi = (float*)(ws + pl->ws.xi);
  if (pl->search == GLR_SEARCH_WINDOW) {
    {
      StageTimer t(pl, s, T_NORMS);
      launch_gather_keys(pl, xp, keys, A, tsh, s);
      launch_interleave(pl, xp, xi, s);
    }
    StageTimer t(pl, s, T_MATCH);
    launch_window_topk(pl, xi, A, keys, idx_out, dd_out, s);
    return check_hip("glr_match_topk");
  }
  {
    StageTimer t(pl, s, T_NORMS);
    launch_gather_keys(pl, xp, keys, A, tsh, s);
    launch_interleave(pl, xp, xi, s);
    if (bf) {
      launch_key_meta(pl, A, Ab, kmb, kre, 0, s);
      launch_cand_meta(pl, xp, cmeta, cm2, cre, 0, s);
    } else {
      launch_key_meta_pc(pl, A, Ac, kn, kc, s);
      launch_cand_meta_pc(pl, xp, pn, pc, pq, s);
    }
  }
  // FP32 pass over keys (kmap == null: rows 0..n) or over a key list (the
  // BF16 form's re-matched keys, whose matcher time is kept apart)
  auto fp32_pass = [&](const int32_t* kmap, int n) {
    for (int g0 = 0; g0 < n; g0 += pl->n_chunk) {
      const int nk = std::min(pl->n_chunk, n - g0);
      {
        StageTimer t(pl, s, kmap ? T_REMATCH : T_MATCH);
        launch_match_f32(pl, xp, Ac, kn, kc, pn, pc, kmap, g0, nk, dist, s);
        if (pl->timing) (kmap ? pl->rematch_launches : pl->match_launches)++;
      }
      {
        StageTimer t(pl, s, T_TOPK);
        launch_topk_partial(pl, dist, kn, nullptr, kmap, g0, pq, nullptr, nk, 0, tsh, lj, lu,
                            ll, lcnt, s);
      }
      {
        StageTimer t(pl, s, T_SELECT);
        launch_select_rescore(pl, xi, A, kmap, g0, nk, lj, lu, ll, lcnt, idx_out, dd_out, oflag,
                              tsh, 0, bm, dist, kn, nullptr, pq, nullptr, 0, tkey, st, s);
      }
    }
  };
  if (!bf) {
    fp32_pass(nullptr, pl->N);
    return check_hip("glr_match_topk");
  }
  // BF16 pass; keys whose margin set or range lists overflow are re-matched
  // with the FP32 form (a bound about 15x tighter) instead of being rescored
  // against every candidate.
  launch_fill_u32((uint32_t*)kcount, 0u, 1, s);
  for (int g0 = 0; g0 < pl->N; g0 += pl->n_chunk) {
    const int nk = std::min(pl->n_chunk, pl->N - g0);
    {
      StageTimer t(pl, s, T_MATCH);
      launch_match_bf16(pl, xp, Ab, kmb, cmeta, g0, nk, dist, s);
      if (pl->timing) pl->match_launches++;
    }
    {
      StageTimer t(pl, s, T_TOPK);
      launch_topk_partial(pl, dist, kmb, kre, nullptr, g0, cm2, cre, nk, 1, tsh, lj, lu, ll,
                          lcnt, s);
    }
    {
      StageTimer t(pl, s, T_SELECT);
      launch_select_rescore(pl, xi, A, nullptr, g0, nk, lj, lu, ll, lcnt, idx_out, dd_out, oflag,
                            tsh, 1, bm, dist, kmb, kre, cm2, cre, 1, tkey, st, s);
      launch_collect_flags(oflag, g0, nk, klist, kcount, st, s);
    }
  }
  int32_t n_re = 0;
  if (hipMemcpyAsync(&n_re, kcount, sizeof(n_re), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return check_hip("glr_match_topk");
  if (n_re > 0) {
    {
      StageTimer t(pl, s, T_NORMS);
      launch_key_meta_pc(pl, A, Ac, kn, kc, s);
      launch_cand_meta_pc(pl, xp, pn, pc, pq, s);
    }
    fp32_pass(klist, n_re);
  }
  return check_hip("glr_match_topk");
}

glr_status lowrank_stage(glr_plan* pl, const float* xp, const int32_t* idx, float sigma, float* xo,
                         float* sv, char* ws, hipStream_t s, int32_t* cover = nullptr,
                         bool count_step = false, const float* sigp = nullptr) {
  float* xhat = (float*)(ws + pl->ws.xhat);
  DevStats* st = (DevStats*)(ws + pl->ws.stats);
  float* gw = pl->agg_weights == GLR_AGG_RANK ? (float*)(ws + pl->ws.gw) : nullptr;
  {
    StageTimer t(pl, s, T_LOWRANK);
    int zn = 0;
    int32_t* z = agg_zero_range(pl, (int32_t*)(ws + pl->ws.pairs), &zn);
    float* xi = (float*)(ws + pl->ws.xi);
    launch_interleave(pl, xp, xi, s);
    launch_wnnm(pl, xi, idx, sigma, xhat, sv, st, z, zn, count_step ? 1 : 0, gw, sigp, s);
  }
  {
    StageTimer t(pl, s, T_AGG);
    launch_aggregate(pl, xp, idx, xhat, gw, (int32_t*)(ws + pl->ws.pairs),
                     (int32_t*)(ws + pl->ws.offs), (int32_t*)(ws + pl->ws.gplan),
                     (float*)(ws + pl->ws.gpart), xo, cover, s);
  }
  return check_hip("glr_lowrank_aggregate");
}

glr_status prior_planar(glr_plan* pl, const float* xp, float sigma, float* xo, char* ws,
                        hipStream_t s) {
  int32_t* keys = (int32_t*)(ws + pl->ws.keys);
  int32_t* idx = (int32_t*)(ws + pl->ws.idx);
  float* dd = (float*)(ws + pl->ws.dd);
  {
    StageTimer t(pl, s, T_DETECT);
    launch_exemplars(pl, xp, ws, keys, s);
  }
  glr_status e = check_hip("detect");
  if (e) return e;
  e = match_stage(pl, xp, keys, idx, dd, ws, s);
  if (e) return e;
  e = lowrank_stage(pl, xp, idx, sigma, xo, (float*)(ws + pl->ws.sv), ws, s, nullptr, true);
  // inner WNNM iterations on the same groups: y^(k) = x^(k-1) + delta (xbar -
  // y^(k-1)) with y^(1) = xbar, the noise level re-estimated on the device
  // (no host read), x^(k) the shrinkage and aggregation of y^(k)
  float* yk = (float*)(ws + pl->ws.yk);
  float* sigk = (float*)(ws + pl->ws.isig);
  for (int k = 2; k <= pl->wnnm_iters && !e; ++k) {
    {
      StageTimer t(pl, s, T_LOWRANK);
      launch_inner_update(xp, xo, k == 2 ? xp : yk, yk, (size_t)pl->Cp * pl->H * pl->W,
                          pl->wnnm_delta, sigma, pl->wnnm_lambda, (double*)(ws + pl->ws.ipart),
                          sigk, s);
    }
    e = lowrank_stage(pl, yk, idx, sigma, xo, (float*)(ws + pl->ws.sv), ws, s, nullptr, false,
                      sigk);
  }
  if (e) return e;
  return check_hip("prior step");
}

// The surrogate in place of the prior step on planar xp (Cp slices of H x W):
// x_cnn = xp + f(xp, sigma); unless the judge is off, GLR on every
// judge_stride-th detected key gives x_glr on the covered pixels and the
// relative deviation decides.  *accepted: the CNN estimate was used (xo);
// otherwise xo is the full GLR step.  One host read of the deviation.
glr_status surrogate_prior(glr_plan* pl, const float* xp, float sigma, float* xo, char* ws,
                           hipStream_t s, bool* accepted) {
  const int HW = pl->H * pl->W;
  float* xcnn = (float*)(ws + pl->ws.xcnn);
  float* sigv = (float*)(ws + pl->ws.sigv);
  {
    StageTimer t(pl, s, T_CNN);
    launch_fill_f32(sigv, sigma, (size_t)pl->Cp, s);
    cnn_forward(pl->cnn_packed, xp, sigv, xcnn, pl->Cp, pl->H, pl->W, ws + pl->ws.cnn_ws, s);
  }
  glr_status e = check_hip("surrogate forward");
  if (e) return e;
  float delta = 0.f;
  const bool judged = !std::isinf(pl->judge_delta_max);
  if (judged) {
    int32_t* keys = (int32_t*)(ws + pl->ws.keys);
    int32_t* sub = (int32_t*)(ws + pl->ws.subkeys);
    int32_t* idx = (int32_t*)(ws + pl->ws.idx);
    float* dd = (float*)(ws + pl->ws.dd);
    float* xglr = (float*)(ws + pl->ws.xglr);
    int32_t* cover = (int32_t*)(ws + pl->ws.cover);
    float* dptr = (float*)(ws + pl->ws.jdelta);
    const int N = pl->N, M = pl->M, M2 = pl->M2;
    const int ns = (N + pl->judge_stride - 1) / pl->judge_stride;
    {
      StageTimer t(pl, s, T_DETECT);
      launch_exemplars(pl, xp, ws, keys, s);
      launch_stride_keys(keys, N, pl->judge_stride, sub, s);
    }
    // the subset step reuses the plan's buffers with N = ns keys
    pl->N = ns;
    pl->M = ns * pl->K;
    pl->M2 = 2048;
    while (pl->M2 < pl->M) pl->M2 <<= 1;
    e = match_stage(pl, xp, sub, idx, dd, ws, s);
    if (!e) e = lowrank_stage(pl, xp, idx, sigma, xglr, (float*)(ws + pl->ws.sv), ws, s, cover);
    pl->N = N;
    pl->M = M;
    pl->M2 = M2;
    if (e) return e;
    {
      StageTimer t(pl, s, T_JUDGE);
      launch_judge(xcnn, xglr, cover, pl->Cp, HW, (float*)(ws + pl->ws.jpart), dptr, s);
    }
    if (hipMemcpyAsync(&delta, dptr, sizeof delta, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return check_hip("judge");
    pl->judge_delta_last = delta;
  }
  if (!judged || delta <= pl->judge_delta_max) {
    hipMemcpyAsync(xo, xcnn, (size_t)pl->Cp * HW * 4, hipMemcpyDeviceToDevice, s);
    pl->sur_steps++;
    *accepted = true;
    return check_hip("surrogate");
  }
  pl->fallback_steps++;
  *accepted = false;
  return prior_planar(pl, xp, sigma, xo, ws, s);
}

// input image (modality layout) -> planar pointer (complex data is split into ws.xp)
const float* planar_in(glr_plan* pl, const void* x, char* ws, hipStream_t s) {
  if (!pl->is_complex) return (const float*)x;
  float* xp = (float*)(ws + pl->ws.xp);
  launch_to_planar((const float2*)x, xp, pl->H * pl->W, s);
  return xp;
}

// For MRI with vp, also vp = planar form of x_out + u (the prior's input).
// yacc: accelerated GAP's accumulated measurement (null: plain GAP), updated
// when wacc != 0.
glr_status data_step_impl(glr_plan* pl, const void* y, const void* x, const void* z,
                          const void* u, void* x_out, char* ws, hipStream_t s,
                          float* vp = nullptr, float* yacc = nullptr, int wacc = 0) {
  StageTimer t(pl, s, T_DATA);
  const int H = pl->H, W = pl->W, HW = H * W;
  if (pl->modality == GLR_CACTI) {
    launch_cacti_gap((const float*)x, (const float*)y, pl->mask, (float*)x_out, pl->C, HW, yacc,
                     wacc, s);
  } else if (pl->modality == GLR_MSFA) {
    launch_msfa_gap((const float*)x, (const float*)y, (float*)x_out, H, W, yacc, wacc, s);
  } else {
    // F(z - u) with the k-space update fused into the transform's passes
    float2* a = (float2*)(ws + pl->ws.cplx_a);
    FftFuse fw;
    fw.in2 = (const float2*)u;
    fw.beta = -1.0f;
    fw.ky = (const float2*)y;
    fw.lines = pl->mask;
    fw.rho = pl->rho;
    launch_fft2d((const float2*)z, a, H, W, 0, s, &fw);
    FftFuse iv;
    if (vp) {
      iv.pu = (const float2*)u;
      iv.vp = vp;
    }
    launch_fft2d(a, (float2*)x_out, H, W, 1, s, &iv);
  }
  return check_hip("glr_data_step");
}

}  // namespace

glr_status glr_set_error(glr_status s, const char* msg) {
  g_err = msg ? msg : "";
  return s;
}

// ================================================================== ABI
extern "C" {

int32_t glr_version(void) { return 100; }

const char* glr_status_string(glr_status s) {
  switch (s) {
    case GLR_OK: return "GLR_OK";
    case GLR_ERR_INVALID_ARG: return "GLR_ERR_INVALID_ARG";
    case GLR_ERR_SHAPE: return "GLR_ERR_SHAPE";
    case GLR_ERR_ALIGNMENT: return "GLR_ERR_ALIGNMENT";
    case GLR_ERR_UNSUPPORTED: return "GLR_ERR_UNSUPPORTED";
    case GLR_ERR_WORKSPACE_TOO_SMALL: return "GLR_ERR_WORKSPACE_TOO_SMALL";
    case GLR_ERR_HIP: return "GLR_ERR_HIP";
    default: return "GLR_ERR_UNKNOWN";
  }
}

const char* glr_last_error_message(void) { return g_err.c_str(); }

void glr_params_default(glr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->solver = GLR_SOLVER_GAP;
  p->rho = 1.0f;
  p->wnnm_c = 2.0f * std::sqrt(2.0f);
  p->wnnm_eps = 1e-16f;
  p->precision = GLR_PREC_FP32;
  p->dist_chunk_mb = 16384;
  p->timing = 0;
  p->surrogate = 0;
  p->surrogate_frac = 0.6f;
  p->judge_stride = 8;
  p->judge_delta_max = 0.02f;
  p->cnn_packed = nullptr;
  p->exemplars = GLR_EXEMPLAR_CORNER;
  p->uniform_step = 4;
  p->search = GLR_SEARCH_GLOBAL;
  p->window = 20;
  p->score = GLR_SCORE_L2;
  p->agg_weights = GLR_AGG_UNIFORM;
  p->wnnm_iters = 1;
  p->wnnm_delta = 0.1f;
  p->wnnm_lambda = 0.54f;
  p->lowrank = GLR_LOWRANK_STACKED;
}

glr_status glr_plan_create(glr_plan** out, const glr_problem* pb, const glr_params* pr,
                           size_t* workspace_bytes) {
  g_err.clear();
  if (!out || !pb || !pr) return fail(GLR_ERR_INVALID_ARG, "glr_plan_create: NULL argument");
  *out = nullptr;
  if (pb->modality < GLR_CACTI || pb->modality > GLR_MSFA)
    return fail(GLR_ERR_INVALID_ARG, "unknown modality %d", pb->modality);
  if (pb->H <= 0 || pb->W <= 0 || pb->C <= 0)
    return fail(GLR_ERR_SHAPE, "image size must be positive (H=%d W=%d C=%d)", pb->H, pb->W, pb->C);
  if (pb->H > 65535 || pb->W > 65535 || (long long)pb->H * pb->W > (1LL << 26))
    return fail(GLR_ERR_UNSUPPORTED, "image side > 65535 or more than 2^26 pixels");
  const int P = pr->patch;
  if (P < 1 || P > std::min(pb->H, pb->W))
    return fail(GLR_ERR_SHAPE, "patch %d must be in [1, min(H, W)]", P);
  if (P > 16) return fail(GLR_ERR_UNSUPPORTED, "patch %d > 16", P);
  const int Cp = pb->modality == GLR_MRI ? 2 : pb->C;
  const int D = Cp * P * P;
  if (D > 4096) return fail(GLR_ERR_UNSUPPORTED, "patch dimension %d > 4096", D);
  const int Hc = pb->H - P + 1, Wc = pb->W - P + 1;
  const long long Ncand = (long long)Hc * Wc;
  if (pr->k < 1 || pr->k > Ncand) return fail(GLR_ERR_SHAPE, "K=%d must be in [1, N_cand=%lld]", pr->k, Ncand);
  if (pr->k > 64) return fail(GLR_ERR_UNSUPPORTED, "K=%d > 64", pr->k);
  if (pr->exemplars < GLR_EXEMPLAR_CORNER || pr->exemplars > GLR_EXEMPLAR_CORNER_UNIFORM)
    return fail(GLR_ERR_INVALID_ARG, "unknown exemplar selection %d", pr->exemplars);
  if (pr->search != GLR_SEARCH_GLOBAL && pr->search != GLR_SEARCH_WINDOW)
    return fail(GLR_ERR_INVALID_ARG, "unknown search %d", pr->search);
  if (pr->score != GLR_SCORE_L2 && pr->score != GLR_SCORE_EDGE)
    return fail(GLR_ERR_INVALID_ARG, "unknown score %d", pr->score);
  if (pr->agg_weights != GLR_AGG_UNIFORM && pr->agg_weights != GLR_AGG_RANK)
    return fail(GLR_ERR_INVALID_ARG, "unknown aggregation weights %d", pr->agg_weights);
  if (pr->wnnm_iters < 1 || pr->wnnm_iters > 16)
    return fail(GLR_ERR_INVALID_ARG, "wnnm_iters %d not in [1, 16]", pr->wnnm_iters);
  if (pr->wnnm_iters > 1 &&
      !(pr->wnnm_delta >= 0.f && pr->wnnm_delta <= 1.f && pr->wnnm_lambda > 0.f &&
        std::isfinite(pr->wnnm_lambda)))
    return fail(GLR_ERR_INVALID_ARG, "wnnm_delta must lie in [0, 1] and wnnm_lambda be positive");
  if (pr->lowrank != GLR_LOWRANK_STACKED && pr->lowrank != GLR_LOWRANK_COMPLEX)
    return fail(GLR_ERR_INVALID_ARG, "unknown low-rank form %d", pr->lowrank);
  if (pr->lowrank == GLR_LOWRANK_COMPLEX && pb->modality != GLR_MRI)
    return fail(GLR_ERR_INVALID_ARG, "the complex low-rank form needs complex (MRI) data");
  if (pr->wnnm_iters > 1 && pr->surrogate)
    return fail(GLR_ERR_UNSUPPORTED, "inner WNNM iterations are not combined with the surrogate");
  const int Ce = pb->modality == GLR_MRI ? 1 : Cp;
  if (pr->score == GLR_SCORE_EDGE) {
    if (pr->search != GLR_SEARCH_GLOBAL)
      return fail(GLR_ERR_UNSUPPORTED, "the edge-map score needs global search");
    if (4LL * Ce * P * P > 8192)
      return fail(GLR_ERR_UNSUPPORTED, "edge patch length 4*%d*%d^2 above 8192", Ce, P);
  }
  const bool corners = pr->exemplars != GLR_EXEMPLAR_UNIFORM;
  if (corners && (pr->n_keys < 1 || pr->n_keys > Ncand))
    return fail(GLR_ERR_SHAPE, "n_keys=%d must be in [1, N_cand=%lld]", pr->n_keys, Ncand);
  long long n_total = corners ? pr->n_keys : 0;
  if (pr->exemplars != GLR_EXEMPLAR_CORNER) {
    if (pr->uniform_step < 1) return fail(GLR_ERR_INVALID_ARG, "uniform_step must be >= 1");
    const long long st = pr->exemplars == GLR_EXEMPLAR_UNIFORM ? pr->uniform_step
                                                                : 3LL * pr->uniform_step;
    n_total += ((Hc + st - 1) / st) * ((Wc + st - 1) / st);
  }
  // (a candidate's aggregation bucket holds one entry per group: at most N)
  if (n_total > 16384)
    return fail(GLR_ERR_UNSUPPORTED, "%lld exemplar keys above 16384", n_total);
  if (pr->search == GLR_SEARCH_WINDOW) {
    if (pr->window < 1 || pr->window > 4096)
      return fail(GLR_ERR_INVALID_ARG, "window must be in [1, 4096]");
    const long long corner_win =
        (long long)std::min(pr->window + 1, Hc) * std::min(pr->window + 1, Wc);
    if (corner_win < pr->k)
      return fail(GLR_ERR_SHAPE, "a window of %d at a grid corner holds %lld < K=%d candidates",
                  pr->window, corner_win, pr->k);
  }
  if (Ncand + 1 > 4096LL * 4096LL)
    return fail(GLR_ERR_UNSUPPORTED, "N_cand=%lld above 4096^2 - 1", Ncand);
  if (n_total * pr->k > (1LL << 30))
    return fail(GLR_ERR_UNSUPPORTED, "n_keys*K too large");
  if (pr->iters < 0) return fail(GLR_ERR_INVALID_ARG, "iters < 0");
  if (pr->iters > 0 && !pr->sigma) return fail(GLR_ERR_INVALID_ARG, "sigma is NULL");
  if (pr->precision != GLR_PREC_FP32 && pr->precision != GLR_PREC_BF16_RESCORE)
    return fail(GLR_ERR_INVALID_ARG, "unknown precision %d", pr->precision);
  if (!(pr->wnnm_c >= 0.f) || !(pr->wnnm_eps > 0.f) || !(pr->rho > 0.f))
    return fail(GLR_ERR_INVALID_ARG, "wnnm_c >= 0, wnnm_eps > 0 and rho > 0 required");
  if (pr->surrogate) {
    if (!pr->cnn_packed) return fail(GLR_ERR_INVALID_ARG, "surrogate needs cnn_packed");
    if (!aligned(pr->cnn_packed, 256))
      return fail(GLR_ERR_ALIGNMENT, "cnn_packed not 256-byte aligned");
    if (pr->judge_stride < 1) return fail(GLR_ERR_INVALID_ARG, "judge_stride must be >= 1");
    if (!(pr->surrogate_frac >= 0.f && pr->surrogate_frac <= 1.f))
      return fail(GLR_ERR_INVALID_ARG, "surrogate_frac must be in [0, 1]");
    if (!(pr->judge_delta_max >= 0.f)) return fail(GLR_ERR_INVALID_ARG, "judge_delta_max >= 0");
  }
  if (pb->modality == GLR_MRI) {
    if (pb->C != 1) return fail(GLR_ERR_SHAPE, "MRI plans take C = 1 (complex image)");
    if (!pow2(pb->H) || !pow2(pb->W) || pb->H < 4 || pb->W < 4 || pb->H > 2048 || pb->W > 2048)
      return fail(GLR_ERR_UNSUPPORTED, "MRI needs H, W powers of two in [4, 2048]");
    if (pr->solver != GLR_SOLVER_ADMM) return fail(GLR_ERR_INVALID_ARG, "MRI uses the ADMM solver");
  } else if (pr->solver != GLR_SOLVER_GAP && pr->solver != GLR_SOLVER_GAP_ACC) {
    return fail(GLR_ERR_INVALID_ARG, "CACTI/MSFA use the GAP or accelerated GAP solver");
  }
  if (pb->modality == GLR_MSFA) {
    if (pb->C != 16) return fail(GLR_ERR_UNSUPPORTED, "MSFA needs 16 bands");
    if (pb->H % 4 || pb->W % 4) return fail(GLR_ERR_SHAPE, "MSFA needs H, W multiples of 4");
  } else if (!pb->mask) {
    return fail(GLR_ERR_INVALID_ARG, "mask is NULL");
  }
  if (pb->mask && !aligned(pb->mask, 16)) return fail(GLR_ERR_ALIGNMENT, "mask not 16-byte aligned");

  glr_plan* pl = new (std::nothrow) glr_plan();
  if (!pl) return fail(GLR_ERR_INVALID_ARG, "out of host memory");
  pl->modality = pb->modality;
  pl->H = pb->H;
  pl->W = pb->W;
  pl->C = pb->C;
  pl->Cp = Cp;
  pl->is_complex = pb->modality == GLR_MRI;
  pl->mask = pb->mask;
  pl->P = P;
  pl->N = (int)n_total;
  pl->n_corner = corners ? pr->n_keys : 0;
  pl->exemplars = pr->exemplars;
  pl->uniform_step = pr->uniform_step;
  pl->search = pr->search;
  pl->window = pr->window;
  pl->score = pr->score;
  pl->agg_weights = pr->agg_weights;
  pl->wnnm_iters = pr->wnnm_iters;
  pl->wnnm_delta = pr->wnnm_delta;
  pl->wnnm_lambda = pr->wnnm_lambda;
  pl->lowrank_complex = pr->lowrank == GLR_LOWRANK_COMPLEX;
  pl->Ce = Ce;
  pl->K = pr->k;
  pl->T = pr->iters;
  pl->solver = pr->solver;
  pl->precision = pr->precision;
  pl->timing = pr->timing;
  pl->rho = pr->rho;
  pl->wnnm_c = pr->wnnm_c;
  pl->wnnm_eps = pr->wnnm_eps;
  pl->surrogate = pr->surrogate ? 1 : 0;
  pl->surrogate_frac = pr->surrogate_frac;
  pl->judge_stride = pr->judge_stride;
  pl->judge_delta_max = pr->judge_delta_max;
  pl->cnn_packed = pr->cnn_packed;
  pl->sur_steps = pl->fallback_steps = 0;
  pl->judge_delta_last = 0.f;
  if (pr->iters > 0) pl->sigma.assign(pr->sigma, pr->sigma + pr->iters);
  pl->Hc = Hc;
  pl->Wc = Wc;
  pl->Ncand = (int)Ncand;
  pl->D = D;
  pl->ldd = (int)up((size_t)Ncand, 64);
  size_t chunk_bytes = (size_t)(pr->dist_chunk_mb > 0 ? pr->dist_chunk_mb : 16384) << 20;
  long long nch = (long long)(chunk_bytes / ((size_t)pl->ldd * 4));
  if (nch < 1) nch = 1;
  if (nch >= 128) nch = nch / 128 * 128;
  pl->n_chunk = (int)std::min<long long>(nch, pl->N);
  // window search needs no distance chunks or candidate-range lists
  if (pl->search == GLR_SEARCH_WINDOW) pl->n_chunk = 1;
  // ranges per key: enough waves to fill the chip; more for the BF16 form,
  // whose larger margin sets need the combined capacity of more range lists
  // (on the 1024^2 x 24 workload, 16 GiB chunks of 4096 keys with 16 ranges
  // each: no list overflow over the run, and half the launches, hence half
  // the per-launch tails, of 8 GiB chunks)
  const int target = pr->precision == GLR_PREC_BF16_RESCORE ? 65536 : 8192;
  int ns = (target + pl->n_chunk - 1) / pl->n_chunk;
  ns = std::min(ns, 64);
  ns = std::min<long long>(ns, (Ncand + 1023) / 1024);
  if (ns < 1) ns = 1;
  pl->split_len = (int)up((size_t)((Ncand + ns - 1) / ns), 256);
  pl->n_split = (int)((Ncand + pl->split_len - 1) / pl->split_len);
  pl->M = pl->N * pl->K;
  pl->M2 = 2048;
  while (pl->M2 < pl->M) pl->M2 <<= 1;

  const size_t HW = (size_t)pl->H * pl->W;
  Carver c;
  WsLayout& L = pl->ws;
  L.xp = c.take(HW * Cp * 4);
  L.xo = c.take(HW * Cp * 4);
  L.xi = c.take(HW * Cp * 4);
  L.q = c.take(HW);
  L.gxx = c.take(HW * 4);
  L.gyy = c.take(HW * 4);
  L.gxy = c.take(HW * 4);
  L.r25 = c.take(HW * 8);
  L.cflag = c.take((size_t)Ncand);
  L.slist = c.take((size_t)Ncand * 4);
  L.sval = c.take((size_t)Ncand * 8);
  L.keys = c.take((size_t)pl->N * 4);
  const bool edge = pr->score == GLR_SCORE_EDGE;
  const int De = 4 * Ce * P * P;                 // edge patch length
  L.A = c.take((size_t)pl->N * (edge ? std::max(D, De) : D) * 4);
  // the BF16 buffers serve the BF16 form and the edge score alike
  const bool bf = pr->precision == GLR_PREC_BF16_RESCORE || edge;
  L.kmb = c.take(bf ? (size_t)pl->N * 16 : 0);
  L.cmeta = c.take(bf ? (size_t)Ncand * 16 : 0);
  // arrays the top-K stage streams carry SPAD entries of padding, so its
  // chunked loads stay in bounds without a ragged-edge path
  L.cm2 = c.take(bf ? ((size_t)Ncand + SPAD) * 8 : 0);
  L.kre = c.take(bf ? (size_t)pl->N * 4 : 0);
  L.cre = c.take(bf ? ((size_t)Ncand + SPAD) * 4 : 0);
  L.E = c.take(edge ? (size_t)4 * Ce * HW * 4 : 0);
  L.eq = c.take(edge ? (size_t)Ce * HW : 0);
  L.egx = c.take(edge ? (size_t)2 * Ce * HW * 2 : 0);
  L.emax = c.take(edge ? 4 : 0);
  L.Ac = c.take((size_t)pl->N * D * 4);
  L.kn = c.take((size_t)pl->N * 16);
  L.kc = c.take((size_t)pl->N * Cp * 4);
  L.pn = c.take((size_t)Ncand * 4);
  L.pc = c.take((size_t)Cp * Ncand * 8);
  L.pq = c.take(((size_t)Ncand + SPAD) * 8);
  L.Ab = c.take(bf ? (size_t)pl->N * (edge ? std::max(Cp, 4 * Ce) : Cp) * bf16_key_row(P) * 2 : 0);
  L.tsh = c.take((size_t)pl->n_chunk * 4);
  L.tkey = c.take((size_t)pl->n_chunk * 4);
  L.klist = c.take(bf ? (size_t)pl->N * 4 : 0);
  L.kcount = c.take(bf ? 4 : 0);
  pl->mcap = (int)std::min<long long>(Ncand, 32768);
  L.bpos = c.take((size_t)pl->n_chunk * pl->mcap * 4);
  L.bhi = c.take((size_t)pl->n_chunk * pl->mcap * 4);
  L.blo = c.take((size_t)pl->n_chunk * pl->mcap * 4);
  L.dist = c.take(((size_t)pl->n_chunk * pl->ldd + SPAD) * 4);
  const size_t nlist = (size_t)pl->n_chunk * pl->n_split;
  L.lj = c.take(nlist * GLR_SPLIT_CAP * 4);
  L.lu = c.take(nlist * GLR_SPLIT_CAP * 4);
  L.ll = c.take(nlist * GLR_SPLIT_CAP * 4);
  L.lcnt = c.take(nlist * 4);
  L.oflag = c.take((size_t)pl->n_chunk * 4);
  L.idx = c.take((size_t)pl->M * 4);
  L.dd = c.take((size_t)pl->M * 4);
  L.xhat = c.take((size_t)pl->M * D * 4);
  L.sv = c.take((size_t)pl->M * 4);
  L.gw = c.take(pr->agg_weights == GLR_AGG_RANK ? (size_t)pl->N * 4 : 0);
  const bool inner = pr->wnnm_iters > 1;
  L.yk = c.take(inner ? HW * Cp * 4 : 0);
  L.ipart = c.take(inner ? 1024 * 8 : 0);
  L.isig = c.take(inner ? 4 : 0);
  L.pairs = c.take(agg_sort_ints(pl) * 4);
  L.offs = c.take(((size_t)Ncand + 1) * 4);
  L.gplan = c.take(agg_gather_ints(pl) * 4);
  L.gpart = c.take(agg_gather_part_floats(pl) * 4);
  L.cplx_a = c.take(pl->is_complex ? HW * 8 : 0);
  L.cplx_b = c.take(pl->is_complex ? HW * 8 : 0);
  L.red = c.take(1024);
  const bool sur = pl->surrogate != 0;
  L.cnn_ws = c.take(sur ? cnn_workspace_bytes(Cp, pl->H, pl->W, 0) : 0);
  L.xcnn = c.take(sur ? HW * Cp * 4 : 0);
  L.xglr = c.take(sur ? HW * Cp * 4 : 0);
  L.cover = c.take(sur ? HW * 4 : 0);
  L.subkeys = c.take(sur ? (size_t)pl->N * 4 : 0);
  L.sigv = c.take(sur ? (size_t)Cp * 4 : 0);
  L.jpart = c.take(sur ? 512 * 3 * 4 : 0);
  L.jdelta = c.take(sur ? 4 : 0);
  L.stats = c.take(sizeof(DevStats));
  L.total = c.off;

  pl->ev_used = 0;
  pl->stats_ws = nullptr;
  pl->last_stream = nullptr;
  for (double& m : pl->ms) m = 0.0;
  pl->match_launches = 0;
  pl->rematch_launches = 0;
  if (workspace_bytes) *workspace_bytes = L.total;
  *out = pl;
  return GLR_OK;
}

glr_status glr_plan_destroy(glr_plan* pl) {
  if (!pl) return fail(GLR_ERR_INVALID_ARG, "glr_plan_destroy: NULL plan");
  for (auto& e : pl->ev_pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  delete pl;
  return GLR_OK;
}

glr_status glr_plan_keys(const glr_plan* pl, int32_t* n_keys) {
  if (!pl || !n_keys) return fail(GLR_ERR_INVALID_ARG, "glr_plan_keys: NULL argument");
  *n_keys = pl->N;
  return GLR_OK;
}

glr_status glr_workspace_size(const glr_plan* pl, size_t* bytes) {
  if (!pl || !bytes) return fail(GLR_ERR_INVALID_ARG, "glr_workspace_size: NULL argument");
  *bytes = pl->ws.total;
  return GLR_OK;
}

glr_status glr_forward(glr_plan* pl, const void* x, void* y, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x);
  REQUIRE_PTR(y);
  hipStream_t s = (hipStream_t)stream;
  ensure_stats(pl, (char*)ws, s);
  const int H = pl->H, W = pl->W;
  if (pl->modality == GLR_CACTI)
    launch_cacti_forward((const float*)x, pl->mask, (float*)y, pl->C, H * W, s);
  else if (pl->modality == GLR_MSFA)
    launch_msfa_forward((const float*)x, (float*)y, H, W, s);
  else {
    float2* a = (float2*)((char*)ws + pl->ws.cplx_a);
    launch_fft2d((const float2*)x, a, H, W, 0, s);
    launch_kspace_mask(a, pl->mask, (float2*)y, H, W, s);
  }
  return check_hip(__func__);
}

glr_status glr_adjoint(glr_plan* pl, const void* y, void* x, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x);
  REQUIRE_PTR(y);
  hipStream_t s = (hipStream_t)stream;
  ensure_stats(pl, (char*)ws, s);
  const int H = pl->H, W = pl->W;
  if (pl->modality == GLR_CACTI)
    launch_cacti_adjoint((const float*)y, pl->mask, (float*)x, pl->C, H * W, s);
  else if (pl->modality == GLR_MSFA)
    launch_msfa_adjoint((const float*)y, (float*)x, H, W, s);
  else {
    float2* a = (float2*)((char*)ws + pl->ws.cplx_a);
    launch_kspace_mask((const float2*)y, pl->mask, a, H, W, s);
    launch_fft2d(a, (float2*)x, H, W, 1, s);
  }
  return check_hip(__func__);
}

glr_status glr_fft2d(glr_plan* pl, const void* in, void* out, int32_t inverse, void* ws,
                     void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(in);
  REQUIRE_PTR(out);
  if (!pl->is_complex) return fail(GLR_ERR_UNSUPPORTED, "glr_fft2d needs an MRI plan");
  hipStream_t s = (hipStream_t)stream;
  launch_fft2d((const float2*)in, (float2*)out, pl->H, pl->W, inverse ? 1 : 0, s);
  return check_hip(__func__);
}

glr_status glr_data_step(glr_plan* pl, const void* y, const void* x, const void* z, const void* u,
                         void* x_out, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(y);
  REQUIRE_PTR(x_out);
  if (pl->is_complex) {
    REQUIRE_PTR(z);
    REQUIRE_PTR(u);
  } else {
    REQUIRE_PTR(x);
  }
  hipStream_t s = (hipStream_t)stream;
  ensure_stats(pl, (char*)ws, s);
  return data_step_impl(pl, y, x, z, u, x_out, (char*)ws, s);
}

glr_status glr_detect_keys(glr_plan* pl, const void* x, int32_t* keys, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x);
  REQUIRE_PTR(keys);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const float* xp = planar_in(pl, x, w, s);
  {
    StageTimer t(pl, s, T_DETECT);
    launch_exemplars(pl, xp, w, keys, s);
  }
  return check_hip(__func__);
}

glr_status glr_match_topk(glr_plan* pl, const void* x, const int32_t* keys, int32_t* idx,
                          float* dist, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x);
  REQUIRE_PTR(keys);
  REQUIRE_PTR(idx);
  REQUIRE_PTR(dist);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const float* xp = planar_in(pl, x, w, s);
  return match_stage(pl, xp, keys, idx, dist, w, s);
}

glr_status glr_lowrank_aggregate(glr_plan* pl, const void* x_in, const int32_t* idx, float sigma,
                                 void* x_out, float* sv, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x_in);
  REQUIRE_PTR(idx);
  REQUIRE_PTR(x_out);
  if (sv && !aligned(sv, 16)) return fail(GLR_ERR_ALIGNMENT, "sv not 16-byte aligned");
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return fail(GLR_ERR_INVALID_ARG, "sigma must be finite and >= 0");
  if (x_in == x_out) return fail(GLR_ERR_INVALID_ARG, "x_out must not alias x_in");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const float* xp = planar_in(pl, x_in, w, s);
  float* xo = pl->is_complex ? (float*)(w + pl->ws.xo) : (float*)x_out;
  e = lowrank_stage(pl, xp, idx, sigma, xo, sv, w, s);
  if (e) return e;
  if (pl->is_complex) launch_from_planar(xo, (float2*)x_out, pl->H * pl->W, s);
  return check_hip(__func__);
}

glr_status glr_prior_step(glr_plan* pl, const void* x_in, float sigma, void* x_out, void* ws,
                          void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(x_in);
  REQUIRE_PTR(x_out);
  if (!(sigma >= 0.f) || !std::isfinite(sigma)) return fail(GLR_ERR_INVALID_ARG, "sigma must be finite and >= 0");
  if (x_in == x_out) return fail(GLR_ERR_INVALID_ARG, "x_out must not alias x_in");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const float* xp = planar_in(pl, x_in, w, s);
  float* xo = pl->is_complex ? (float*)(w + pl->ws.xo) : (float*)x_out;
  e = prior_planar(pl, xp, sigma, xo, w, s);
  if (e) return e;
  if (pl->is_complex) launch_from_planar(xo, (float2*)x_out, pl->H * pl->W, s);
  return check_hip(__func__);
}

// Loop state: the iterate (MRI: x, z, u), accelerated GAP's accumulated
// measurement [H][W], then the surrogate-active flag (int32).
size_t state_yacc_offset(const glr_plan* pl) {
  const size_t HW = (size_t)pl->H * pl->W;
  return pl->is_complex ? 3 * HW * 8 : (size_t)pl->C * HW * 4;
}
size_t state_flag_offset(const glr_plan* pl) {
  const size_t HW = (size_t)pl->H * pl->W;
  return state_yacc_offset(pl) + (pl->solver == GLR_SOLVER_GAP_ACC ? HW * 4 : 0);
}

glr_status glr_state_bytes(const glr_plan* pl, size_t* bytes) {
  if (!pl || !bytes) return fail(GLR_ERR_INVALID_ARG, "glr_state_bytes: NULL argument");
  *bytes = state_flag_offset(pl);
  if (pl->surrogate) *bytes += 256;              // surrogate-active flag (int32)
  return GLR_OK;
}

glr_status glr_reconstruct(glr_plan* pl, const void* y, void* state, int32_t t_begin,
                           int32_t t_end, void* x_out, void* ws, void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(y);
  REQUIRE_PTR(state);
  REQUIRE_PTR(x_out);
  if (t_begin < 0 || t_end < t_begin || t_end > pl->T)
    return fail(GLR_ERR_INVALID_ARG, "need 0 <= t_begin <= t_end <= iters (%d)", pl->T);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const int H = pl->H, W = pl->W, HW = H * W;
  // surrogate-active flag in the state tail
  int32_t* flag = (int32_t*)((char*)state + state_flag_offset(pl));
  float* yacc = pl->solver == GLR_SOLVER_GAP_ACC ? (float*)((char*)state + state_yacc_offset(pl))
                                                 : nullptr;
  int active = 0;
  // ceil(frac * T) with frac taken to 6 decimals (0.6f must give 3 of 5, not 4)
  const long long fr = std::llround((double)pl->surrogate_frac * 1e6);
  const int t_sur = pl->surrogate ? (int)((fr * pl->T + 999999) / 1000000) : 0;
  if (pl->surrogate) {
    if (t_begin == 0) {
      launch_fill_u32((uint32_t*)flag, 1u, 1, s);
      active = 1;
    } else if (hipMemcpyAsync(&active, flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
               hipStreamSynchronize(s) != hipSuccess) {
      return check_hip(__func__);
    }
  }
  // prior step of iteration t: the surrogate while allowed, else GLR
  auto prior = [&](int t, const float* in, float* out) -> glr_status {
    if (!(active && t < t_sur)) return prior_planar(pl, in, pl->sigma[t], out, w, s);
    bool ok = false;
    glr_status st = surrogate_prior(pl, in, pl->sigma[t], out, w, s, &ok);
    if (!st && !ok) {
      active = 0;
      launch_fill_u32((uint32_t*)flag, 0u, 1, s);
    }
    return st;
  };
  if (!pl->is_complex) {
    float* x = (float*)state;
    float* xb = (float*)(w + pl->ws.xp);
    if (t_begin == 0) {
      if (pl->modality == GLR_CACTI) launch_cacti_init((const float*)y, pl->mask, x, pl->C, HW, s);
      else launch_msfa_init((const float*)y, x, H, W, s);
      if (yacc) hipMemcpyAsync(yacc, y, (size_t)HW * 4, hipMemcpyDeviceToDevice, s);
    }
    for (int t = t_begin; t < t_end; ++t) {
      e = data_step_impl(pl, y, x, nullptr, nullptr, xb, w, s, nullptr, yacc, 1);
      if (e) return e;
      e = prior(t, xb, x);
      if (e) return e;
    }
    hipMemcpyAsync(x_out, x, (size_t)pl->C * HW * 4, hipMemcpyDeviceToDevice, s);
  } else {
    float2* x = (float2*)state;
    float2* z = x + HW;
    float2* u = z + HW;
    float* vp = (float*)(w + pl->ws.xp);
    float* zp = (float*)(w + pl->ws.xo);
    if (t_begin == 0) {
      float2* a = (float2*)(w + pl->ws.cplx_a);
      launch_kspace_mask((const float2*)y, pl->mask, a, H, W, s);
      launch_fft2d(a, z, H, W, 1, s);
      launch_cplx_axpby(z, z, x, 1.0f, 0.0f, HW, s);
      launch_cplx_axpby(z, z, u, 0.0f, 0.0f, HW, s);
    }
    for (int t = t_begin; t < t_end; ++t) {
      e = data_step_impl(pl, y, nullptr, z, u, x, w, s, vp);     // also vp = planar(x + u)
      if (e) return e;
      e = prior(t, vp, zp);
      if (e) return e;
      launch_admm_dual(u, x, zp, z, HW, s);
    }
    hipMemcpyAsync(x_out, z, (size_t)HW * 8, hipMemcpyDeviceToDevice, s);
  }
  return check_hip(__func__);
}

glr_status glr_pre_prior(glr_plan* pl, const void* y, const void* state, void* v_out, void* ws,
                         void* stream) {
  glr_status e = check_plan_ws(pl, ws, __func__);
  if (e) return e;
  REQUIRE_PTR(y);
  REQUIRE_PTR(state);
  REQUIRE_PTR(v_out);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  ensure_stats(pl, w, s);
  const int HW = pl->H * pl->W;
  if (!pl->is_complex) {
    if (v_out == state) return fail(GLR_ERR_INVALID_ARG, "v_out must not alias the state");
    float* yacc = pl->solver == GLR_SOLVER_GAP_ACC
                      ? (float*)((char*)state + state_yacc_offset(pl)) : nullptr;
    // the accumulated measurement is read, not advanced
    return data_step_impl(pl, y, state, nullptr, nullptr, v_out, w, s, nullptr, yacc, 0);
  }
  // ADMM: x = F^H((M y + rho F(z - u)) / (M + rho)) into the complex scratch,
  // v = x + u in planar form (the prior's input), then interleaved into v_out
  const float2* st = (const float2*)state;
  float2* xs = (float2*)(w + pl->ws.cplx_b);
  float* vp = (float*)(w + pl->ws.xp);
  e = data_step_impl(pl, y, nullptr, st + HW, st + 2 * (size_t)HW, xs, w, s, vp);
  if (e) return e;
  launch_from_planar(vp, (float2*)v_out, HW, s);
  return check_hip(__func__);
}

glr_status glr_read_stats(glr_plan* pl, glr_stats* out, int32_t reset) {
  if (!pl || !out) return fail(GLR_ERR_INVALID_ARG, "glr_read_stats: NULL argument");
  std::memset(out, 0, sizeof *out);
  if (pl->stats_ws) {
    if (hipStreamSynchronize(pl->last_stream) != hipSuccess)
      return fail(GLR_ERR_HIP, "hipStreamSynchronize failed");
    fold_timers(pl);
    DevStats d;
    if (hipMemcpy(&d, (const char*)pl->stats_ws + pl->ws.stats, sizeof d, hipMemcpyDeviceToHost) !=
        hipSuccess)
      return fail(GLR_ERR_HIP, "stats copy failed");
    out->prior_steps = (int64_t)d.steps;
    out->margin_sum = (int64_t)d.margin_sum;
    out->margin_max = d.margin_max;
    out->overflow_keys = d.overflow;
    out->jacobi_sweeps_max = d.sweeps_max;
    out->jacobi_sweeps_sum = (int64_t)d.sweeps_sum;
    out->keys_selected = d.keys_selected;
    out->rematch_keys = (int64_t)d.rematch;
    out->regather_keys = (int64_t)d.regather;
    if (reset) {
      launch_fill_u32((uint32_t*)((char*)pl->stats_ws + pl->ws.stats), 0u, sizeof(DevStats) / 4,
                      pl->last_stream);
      hipStreamSynchronize(pl->last_stream);
    }
  }
  out->ms_detect = (float)pl->ms[T_DETECT];
  out->ms_match = (float)pl->ms[T_MATCH];
  out->ms_topk = (float)pl->ms[T_TOPK];
  out->ms_select = (float)pl->ms[T_SELECT];
  out->ms_lowrank = (float)pl->ms[T_LOWRANK];
  out->ms_aggregate = (float)pl->ms[T_AGG];
  out->ms_data = (float)pl->ms[T_DATA];
  out->ms_norms = (float)pl->ms[T_NORMS];
  out->ms_cnn = (float)pl->ms[T_CNN];
  out->ms_judge = (float)pl->ms[T_JUDGE];
  out->ms_rematch = (float)pl->ms[T_REMATCH];
  out->rematch_launches = pl->rematch_launches;
  out->match_launches = pl->match_launches;
  out->surrogate_steps = pl->sur_steps;
  out->fallback_steps = pl->fallback_steps;
  out->judge_delta_last = pl->judge_delta_last;
  if (reset) {
    for (double& m : pl->ms) m = 0.0;
    pl->match_launches = 0;
    pl->rematch_launches = 0;
    pl->sur_steps = pl->fallback_steps = 0;
  }
  return GLR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- CNN surrogate
namespace {
glr_status cnn_shape(const char* fn, int32_t B, int32_t h, int32_t w) {
  if (B < 1 || h < 1 || w < 1) return fail(GLR_ERR_SHAPE, "%s: B, h, w must be >= 1", fn);
  if ((long long)B * h * w > (1LL << 31) / 64)
    return fail(GLR_ERR_UNSUPPORTED, "%s: B*h*w too large", fn);
  return GLR_OK;
}
}  // namespace

int32_t glr_cnn_param_count(void) { return cnn_param_count(); }
size_t glr_cnn_packed_bytes(void) { return cnn_packed_bytes(); }

glr_status glr_cnn_workspace_size(int32_t B, int32_t h, int32_t w, int32_t train, size_t* bytes) {
  if (!bytes) return fail(GLR_ERR_INVALID_ARG, "glr_cnn_workspace_size: NULL bytes");
  glr_status e = cnn_shape(__func__, B, h, w);
  if (e) return e;
  *bytes = cnn_workspace_bytes(B, h, w, train ? 1 : 0);
  return GLR_OK;
}

glr_status glr_cnn_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return fail(GLR_ERR_INVALID_ARG, "glr_cnn_pack: NULL argument");
  if (!aligned(params, 16) || !aligned(packed, 256))
    return fail(GLR_ERR_ALIGNMENT, "glr_cnn_pack: params 16-byte, packed 256-byte alignment");
  cnn_pack(params, packed, (hipStream_t)stream);
  return check_hip(__func__);
}

glr_status glr_cnn_forward(const void* packed, const float* x, const float* sigma, float* out,
                           int32_t B, int32_t h, int32_t w, void* ws, void* stream) {
  if (!packed || !x || !sigma || !out || !ws)
    return fail(GLR_ERR_INVALID_ARG, "glr_cnn_forward: NULL argument");
  glr_status e = cnn_shape(__func__, B, h, w);
  if (e) return e;
  if (!aligned(packed, 256) || !aligned(ws, 256) || !aligned(x, 16) || !aligned(out, 16))
    return fail(GLR_ERR_ALIGNMENT, "glr_cnn_forward: packed/ws 256-byte, x/out 16-byte alignment");
  cnn_forward(packed, x, sigma, out, B, h, w, ws, (hipStream_t)stream);
  return check_hip(__func__);
}

glr_status glr_cnn_loss_grad(const void* packed, const float* x, const float* sigma,
                             const float* target, int32_t B, int32_t h, int32_t w, float* loss,
                             float* grad, float* out, void* ws, void* stream) {
  if (!packed || !x || !sigma || !target || !loss || !grad || !out || !ws)
    return fail(GLR_ERR_INVALID_ARG, "glr_cnn_loss_grad: NULL argument");
  glr_status e = cnn_shape(__func__, B, h, w);
  if (e) return e;
  if (!aligned(packed, 256) || !aligned(ws, 256) || !aligned(x, 16) || !aligned(out, 16) ||
      !aligned(grad, 16))
    return fail(GLR_ERR_ALIGNMENT, "glr_cnn_loss_grad: packed/ws 256-byte, arrays 16-byte");
  cnn_loss_grad(packed, x, sigma, target, B, h, w, loss, grad, out, ws, (hipStream_t)stream);
  return check_hip(__func__);
}

glr_status glr_cnn_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                        float lr, void* packed, void* stream) {
  if (!params || !m || !v || !grad || !packed)
    return fail(GLR_ERR_INVALID_ARG, "glr_cnn_adam: NULL argument");
  if (step < 1) return fail(GLR_ERR_INVALID_ARG, "glr_cnn_adam: step counts from 1");
  if (!(lr > 0.f)) return fail(GLR_ERR_INVALID_ARG, "glr_cnn_adam: lr must be > 0");
  if (!aligned(packed, 256)) return fail(GLR_ERR_ALIGNMENT, "glr_cnn_adam: packed 256-byte");
  cnn_adam(params, m, v, grad, step, lr, packed, (hipStream_t)stream);
  return check_hip(__func__);
}
