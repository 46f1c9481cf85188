/*
 * glr.h - C ABI of libglr, the MI355X (gfx950) implementation of the global
 * low-rank (GLR) prior step and of its data-fidelity loop, after
 * "Large-scale Global Low-rank Optimization for Computational Compressed
 * Imaging" (Li, Xu, Cao, Yuan, Brady, Bian; arXiv 2301.03047).
 *
 * The calls follow the paper's problem statement: a measurement y of an
 * image x through a sensing matrix Phi (the low-rank objective of the Method
 * section: minimise sum_i rank(R_i x) subject to y = Phi x), a patch size P
 * and a number N of exemplar (key) patches (the heat-map sizes given with
 * eq. 8), a group size K (the KNN grouping of block matching), and an
 * iterative solver (GAP or ADMM, named with the objective).
 *
 * Conventions for every call
 * - Array arguments are DEVICE pointers unless marked "host".  The caller
 *   owns all device memory (inputs, outputs, workspace); the library never
 *   allocates device memory.  A plan holds host metadata only.
 * - Every compute call is asynchronous on the given HIP stream (except for
 *   the one host read-back of the BF16 form, see precision); results are
 *   valid once the stream has completed.  Calls on one plan must not overlap
 *   (plans are not thread-safe); separate plans may run on separate streams.
 * - Arguments are validated on the host before anything is enqueued.  On an
 *   error nothing is launched, inputs are untouched and outputs are
 *   unspecified; the status is returned and a detail string is available from
 *   glr_last_error_message().  No C++ exception crosses this interface.
 * - Device pointers must be 16-byte aligned; the workspace 256-byte aligned.
 * - The workspace carries one piece of state from one call of a plan to the
 *   next: the statistics read by glr_read_stats().  A plan clears them the
 *   first time it is given a workspace (a pointer different from the last
 *   one it saw); every other buffer is written by a call before it is read.
 *   Between calls the caller may reuse the workspace for anything else, at
 *   the cost of those statistics.
 * - Image layouts: real data is planar float32 [C][H][W] (C = frames for
 *   CACTI, bands for MSFA); MRI data is complex64 interleaved [H][W]
 *   (re, im pairs).  "Real channels" C' is C for real data and 2 for MRI.
 * - Patch vectors are ordered d = (c*P + dy)*P + dx (channel slowest); a
 *   complex patch is stacked [Re; Im].  Candidate patches are all stride-1
 *   top-left positions of the (H-P+1) x (W-P+1) grid (the heat-map size of
 *   eq. 8); a position is the linear index t = r*(W-P+1) + c.
 */
#ifndef GLR_H
#define GLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GLR_API __attribute__((visibility("default")))

typedef int32_t glr_status;
enum {
  GLR_OK = 0,
  GLR_ERR_INVALID_ARG = 1,        /* null pointer, bad enum, bad scalar      */
  GLR_ERR_SHAPE = 2,              /* sizes inconsistent (K > N_cand, P > H)  */
  GLR_ERR_ALIGNMENT = 3,          /* pointer not aligned as required         */
  GLR_ERR_UNSUPPORTED = 4,        /* valid but outside this build's limits   */
  GLR_ERR_WORKSPACE_TOO_SMALL = 5,
  GLR_ERR_HIP = 6                 /* a HIP runtime call or launch failed     */
};

enum { GLR_CACTI = 0, GLR_MRI = 1, GLR_MSFA = 2 };   /* eq. 2, eq. 3, eq. 4-5 */
/* GAP_ACC: accelerated GAP, the measurement replaced by an accumulated one,
 * y_acc <- y_acc + (y - Phi x) (y_acc = y at the start), before each
 * projection (a reading: the paper names GAP without the variant). */
enum { GLR_SOLVER_GAP = 0, GLR_SOLVER_ADMM = 1, GLR_SOLVER_GAP_ACC = 2 };
enum { GLR_PREC_FP32 = 0, GLR_PREC_BF16_RESCORE = 1 };
/* Exemplar selection (Method section: corners of the edge map instead of the
 * traditional uniform grid; Results, CACTI: corners plus a modest uniform
 * grid at three times the vanilla interval). */
enum { GLR_EXEMPLAR_CORNER = 0, GLR_EXEMPLAR_UNIFORM = 1, GLR_EXEMPLAR_CORNER_UNIFORM = 2 };
/* Search region: global matching over the whole candidate grid (eq. 8), or
 * block matching in a local window around each key (eq. 1, vanilla BM). */
enum { GLR_SEARCH_GLOBAL = 0, GLR_SEARCH_WINDOW = 1 };
/* Matching score: the squared L2 distance of the patches (eq. 1, the reading
 * the plan defaults to), or the paper's edge-map correlation (eq. 6-8): the
 * heat value of key and candidate is the number of coinciding pixels of
 * their binary rising/falling, horizontal/vertical Sobel edge patches
 * (larger = more similar). */
enum { GLR_SCORE_L2 = 0, GLR_SCORE_EDGE = 1 };
enum { GLR_AGG_UNIFORM = 0, GLR_AGG_RANK = 1 };
/* Form of the low-rank step for complex data (MRI).  STACKED: each member's
 * P^2 complex values enter the group as 2 P^2 real rows [Re; Im] and the real
 * group is shrunk.  COMPLEX: the group is the P^2 x K complex matrix Z and
 * WNNM runs on its complex SVD Z - mu 1^T = U S V^H (mu the complex row
 * mean; the same weights and threshold, K the member count, sigma the noise
 * level per real component).  Real modalities take STACKED only. */
enum { GLR_LOWRANK_STACKED = 0, GLR_LOWRANK_COMPLEX = 1 };

/* Sensing problem (eq. 2-5). */
typedef struct glr_problem {
  int32_t modality;      /* GLR_CACTI | GLR_MRI | GLR_MSFA                      */
  int32_t H, W;          /* image size                                          */
  int32_t C;             /* CACTI: frames per snapshot; MSFA: bands (16); MRI: 1 */
  const uint8_t* mask;   /* device. CACTI: [C][H][W] in {0,1} (the coded
                            apertures A_t of eq. 2). MRI: [H] k_y-line mask in
                            {0,1}, expanded along k_x (M of eq. 3). MSFA: NULL
                            (4x4 periodic array, band 4*(r%4)+(c%4), eq. 4-5). */
} glr_problem;

/* Method parameters.  Fields the paper leaves open are readings; their
 * defaults are those of glr_params_default(). */
typedef struct glr_params {
  int32_t patch;         /* P, patch side (heat-map sizes with eq. 8)           */
  int32_t n_keys;        /* N, exemplar (key) patches per prior step            */
  int32_t k;             /* K, group size (K nearest patches), 1..64            */
  int32_t iters;         /* T, outer iterations of glr_reconstruct              */
  int32_t solver;        /* GAP or GAP_ACC for CACTI/MSFA, ADMM for MRI         */
  float rho;             /* ADMM penalty                                        */
  const float* sigma;    /* host [iters]: noise level per iteration (copied)    */
  float wnnm_c;          /* WNNM weight constant c (default 2*sqrt(2))          */
  float wnnm_eps;        /* WNNM weight regulariser (default 1e-16)             */
  int32_t precision;     /* matcher contraction on mean-centred key and
                            candidate patches: GLR_PREC_FP32 (FP32 MFMA) or
                            GLR_PREC_BF16_RESCORE (BF16 MFMA, FP32 sums, with
                            its own certified error bound; keys whose margin
                            set would not fit are re-matched in FP32).  The
                            groups are the same exact top-K with either; only
                            the work spent on the margin sets differs.  The
                            BF16 form reads the re-match count back to the
                            host once per match (a synchronisation of the
                            stream inside glr_match_topk, glr_prior_step and
                            each iteration of glr_reconstruct)              */
  int32_t dist_chunk_mb; /* max size of one distance-matrix chunk (MiB)         */
  int32_t timing;        /* nonzero: record per-stage HIP event pairs on the
                            stream (no host sync); glr_read_stats() sums them */
  /* CNN surrogate (glr_cnn_*; not part of the paper's method).  With
   * surrogate != 0, glr_reconstruct uses the network for the prior step
   * while t < ceil(surrogate_frac * iters) and the surrogate is active; each
   * use is judged: GLR runs on every judge_stride-th detected key and
   *   delta = ||(x_cnn - x_glr)|cov|| / ||x_glr|cov||
   * over the pixels those groups cover; delta > judge_delta_max or a
   * non-finite estimate makes that iteration run the full GLR step and
   * deactivates the surrogate for the rest of the run (the active flag is
   * part of the loop state).  judge_delta_max = +inf skips the judge. */
  int32_t surrogate;
  float surrogate_frac;  /* default 0.6 (taken to 6 decimals)                    */
  int32_t judge_stride;  /* default 8                                            */
  float judge_delta_max; /* default 0.02                                         */
  const void* cnn_packed; /* device, glr_cnn_packed_bytes(), from glr_cnn_pack()  */
  /* Block-matching baselines (the paper's comparison).  exemplars: CORNER
   * takes the n_keys corner keys; UNIFORM the grid of top-left positions
   * (s a, s b), s = uniform_step (n_keys is then ignored); CORNER_UNIFORM the
   * n_keys corners followed by the grid of interval 3 s.  The plan's key
   * count N is reported by glr_plan_keys() (at most 16384).  search: GLOBAL
   * (every candidate) or WINDOW (candidates within `window` rows and columns
   * of the key; (window + 1)^2 >= K required).  The groups are exact either
   * way: the window's distances are all computed exactly (FP64 sums). */
  int32_t exemplars;      /* default GLR_EXEMPLAR_CORNER                         */
  int32_t uniform_step;   /* default 4                                           */
  int32_t search;         /* default GLR_SEARCH_GLOBAL                           */
  int32_t window;         /* default 20 (a 41 x 41 window)                        */
  /* Matching score (default GLR_SCORE_L2).  GLR_SCORE_EDGE: edge maps per real
   * channel of the quantised image (complex data: of the detection image),
   * th = ceil(max |gradient| / 10); the heat values are exact integers (BF16
   * MFMA on 0/1 operands), the group is the K largest, the lowest position
   * winning ties, and glr_match_topk's dist holds the heat values.  Needs
   * GLR_SEARCH_GLOBAL and 4 C'' P^2 <= 8192 (C'' = C' real, 1 complex). */
  int32_t score;
  /* Aggregation weights (default GLR_AGG_UNIFORM: every member estimate
   * weighs 1, a pixel is the mean of its covering estimates).  GLR_AGG_RANK:
   * every estimate of group g weighs 1 / max(r_g, 1), r_g the number of
   * singular values the WNNM shrinkage keeps non-zero, and a pixel is the
   * weighted mean (a variant of the aggregation of the Method section). */
  int32_t agg_weights;
  /* Inner WNNM iterations per prior step (default 1: one shrinkage).  With
   * wnnm_iters = J > 1 the groups of the step's one matching are shrunk J
   * times (the iterative regularisation of WNNM [Gu et al. 2014]):
   *   y1 = xbar, yk = x(k-1) + wnnm_delta (xbar - y(k-1)),
   *   sigma1 = sigma, sigmak = wnnm_lambda sqrt(max(sigma^2 - mean((xbar - yk)^2), 0)),
   *   xk = aggregation of the WNNM estimates of the groups of yk at sigmak
   * (uncovered pixels keep yk); the step returns xJ.  1 <= J <= 16;
   * wnnm_delta in [0, 1] (default 0.1), wnnm_lambda > 0 (default 0.54).
   * Not combined with the surrogate. */
  int32_t wnnm_iters;
  float wnnm_delta;
  float wnnm_lambda;
  int32_t lowrank;       /* default GLR_LOWRANK_STACKED; COMPLEX for MRI only     */
} glr_params;

/* Counters of the last prior steps, read by glr_read_stats(). */
typedef struct glr_stats {
  int64_t prior_steps;        /* prior steps since the plan was created/reset   */
  int64_t margin_sum;         /* sum over keys of the certified margin-set size  */
  int32_t margin_max;         /* largest margin set                              */
  int32_t overflow_keys;      /* keys that took the exact full-row path          */
  int32_t jacobi_sweeps_max;  /* most Jacobi sweeps any group needed             */
  int32_t keys_selected;      /* corner keys in the last step (before any fill)  */
  /* with params.timing: milliseconds summed over all prior steps, per stage */
  float ms_detect, ms_match, ms_topk, ms_select, ms_lowrank, ms_aggregate, ms_data;
  float ms_norms;             /* key gather and candidate norms                  */
  int64_t match_launches;     /* matcher kernel launches timed in ms_match       */
  int64_t jacobi_sweeps_sum;  /* Jacobi sweeps summed over all groups            */
  int64_t rematch_keys;       /* BF16 form: keys re-matched with the FP32 form   */
  int64_t surrogate_steps;    /* iterations whose prior step was the CNN         */
  int64_t fallback_steps;     /* judged iterations that fell back to GLR         */
  float judge_delta_last;     /* deviation measured by the last judge            */
  float ms_cnn, ms_judge;     /* with timing: CNN forward, judge (subset GLR)    */
  int64_t regather_keys;      /* keys whose margin set was re-derived from their
                                 distance row (a candidate-range list of the
                                 top-K scan overflowed)                          */
  float ms_rematch;           /* with timing: the BF16 form's FP32 re-match
                                 matcher launches (not in ms_match)              */
  int64_t rematch_launches;   /* those launches                                  */
} glr_stats;

typedef struct glr_plan glr_plan;

/* --------------------------------------------------------------- basics */
GLR_API int32_t glr_version(void);                    /* 100*major + minor          */
GLR_API const char* glr_status_string(glr_status s);
/* Thread-local detail of the last failed call on this thread ("" if none). */
GLR_API const char* glr_last_error_message(void);
/* Fill *p with the defaults (c = 2*sqrt(2), eps = 1e-16, rho = 1, FP32,
 * 16384 MiB chunks, GAP, no timing); patch/n_keys/k/iters are set to 0. */
GLR_API void glr_params_default(glr_params* p);

/* Create a plan for one problem shape.  Validates everything that does not
 * depend on data pointers and reports the workspace size every later call
 * needs (*workspace_bytes, 256-byte aligned buffer owned by the caller).
 * problem->mask is recorded (the caller keeps it alive).  Limits: K <= 64,
 * 1 <= N <= min(N_cand, 16384), K <= N_cand, N_cand < 4096^2,
 * P <= min(H, W), P <= 16, D = C'*P*P <= 4096;
 * MRI needs H, W powers of two in [4, 2048]; MSFA needs C == 16 and H, W
 * multiples of 4. */
GLR_API glr_status glr_plan_create(glr_plan** out, const glr_problem* problem,
                           const glr_params* params, size_t* workspace_bytes);
GLR_API glr_status glr_plan_destroy(glr_plan* plan);
GLR_API glr_status glr_workspace_size(const glr_plan* plan, size_t* bytes);
/* Exemplar keys per prior step (the length of keys, idx and dist): n_keys
 * for CORNER, the uniform grid's size for UNIFORM, both for CORNER_UNIFORM. */
GLR_API glr_status glr_plan_keys(const glr_plan* plan, int32_t* n_keys);

/* --------------------------------------------------------------- operators
 * y = Phi x (eq. 2, eq. 3, eq. 4).  x in the image layout; y: CACTI/MSFA
 * float32 [H][W], MRI complex64 [H][W] (k-space, orthonormal DFT, unshifted,
 * zero outside the sampled lines). */
GLR_API glr_status glr_forward(glr_plan* plan, const void* x, void* y, void* ws, void* stream);
/* x = Phi^T y (Phi^H for MRI).  Same layouts. */
GLR_API glr_status glr_adjoint(glr_plan* plan, const void* y, void* x, void* ws, void* stream);
/* Orthonormal 2-D DFT of a complex64 [H][W] array (MRI plans only);
 * inverse != 0 gives the inverse transform.  In-place allowed. */
GLR_API glr_status glr_fft2d(glr_plan* plan, const void* in, void* out, int32_t inverse,
                     void* ws, void* stream);
/* Data step.  GAP (CACTI, MSFA): x_out = x + Phi^T((y - Phi x) / R~) with
 * R = diag(Phi Phi^T) and zeros of R replaced by 1.  ADMM (MRI): x_out =
 * F^H((M y + rho F(z - u)) / (M + rho)); z and u are complex64 [H][W] and
 * ignored for GAP (may be NULL).  In-place (x_out == x) allowed.  (Always
 * the plain GAP step: the accelerated one needs the loop state's
 * accumulated measurement, see glr_reconstruct / glr_pre_prior.) */
GLR_API glr_status glr_data_step(glr_plan* plan, const void* y, const void* x, const void* z,
                         const void* u, void* x_out, void* ws, void* stream);

/* --------------------------------------------------------------- prior step
 * Key detection (corner exemplars, Method section / Fig. 1a): keys[N] int32,
 * ascending top-left positions.  Reading: integer Harris on a u8 detection
 * image, 3x3 non-maximum suppression, best N by score, uniform raster fill
 * when fewer corners exist.  With params.exemplars UNIFORM the keys are the
 * uniform grid; with CORNER_UNIFORM the n_keys corners followed by the grid
 * of three times the interval (N = glr_plan_keys()). */
GLR_API glr_status glr_detect_keys(glr_plan* plan, const void* x, int32_t* keys, void* ws,
                           void* stream);
/* Global matching and grouping (eq. 1 made global; eq. 8 candidate grid):
 * for each key g, idx[g][0..K) are the K candidates with the smallest
 * squared L2 patch distance, ordered by (distance, position) ascending, and
 * dist[g][q] those distances (float32).  keys: device int32 [N] (any order,
 * each < N_cand).  The distance contraction runs on MFMA; candidates within a
 * certified error margin of the K-th distance are rescored in FP64 (exact
 * differences, FP64 sums) so that the selection equals the exact one.
 * With params.search WINDOW the candidates are those of the key's window
 * (block matching), all scored in FP64. */
GLR_API glr_status glr_match_topk(glr_plan* plan, const void* x, const int32_t* keys,
                          int32_t* idx, float* dist, void* ws, void* stream);
/* Low-rank step and aggregation (WNNM on each group, the low-rank objective
 * of the Method section): each group Y (D x K, column q = patch idx[g][q]) is
 * mean-centred, decomposed by a one-sided Jacobi SVD (QR-preconditioned),
 * its singular values shrunk by the WNNM weights for noise level sigma, and
 * the member estimates averaged back per pixel; pixels no member covers keep
 * x_in (weighted per group with params.agg_weights RANK).  One shrinkage:
 * params.wnnm_iters applies to glr_prior_step and glr_reconstruct only.
 * With params.lowrank COMPLEX the group is the P^2 x K complex matrix and the
 * SVD complex (Hermitian rotations).
 * sv: optional device float32 [N][K], singular values descending (NULL to
 * skip; the complex form has at most min(P^2, K) non-zero ones).  x_out must
 * not alias x_in. */
GLR_API glr_status glr_lowrank_aggregate(glr_plan* plan, const void* x_in, const int32_t* idx,
                                 float sigma, void* x_out, float* sv, void* ws,
                                 void* stream);
/* The whole prior step: detect, match, group, shrink, aggregate. x_out must
 * not alias x_in. */
GLR_API glr_status glr_prior_step(glr_plan* plan, const void* x_in, float sigma, void* x_out,
                          void* ws, void* stream);

/* Allocation-free glr_prior_step, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a library-owned static device array
 * of GLR_STATIC_SCRATCH_BYTES per GPU (held from the library's load on that
 * GPU until the process ends), looked up on the CURRENT device at the first
 * call there; stream must belong to that device.  The caller still passes
 * x_in and x_out (layouts as for glr_prior_step; x_out must not alias x_in).
 * The call reaches no hipMalloc, hipFree or allocating library routine.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (any plans, any streams) race and must be serialised by the caller.
 * The statistics region is cleared by each call, so glr_read_stats() after
 * it reports that call alone, until the next call on the same GPU.
 * BF16-form plans read one 4-byte counter back to the host (a stream
 * synchronisation), as glr_prior_step does.
 * Errors: GLR_ERR_WORKSPACE_TOO_SMALL when the plan's workspace
 * (glr_workspace_size) exceeds GLR_STATIC_SCRATCH_BYTES; GLR_ERR_UNSUPPORTED
 * for plans created with timing != 0 (their event pairs are created on
 * demand); GLR_ERR_HIP if the array's address cannot be obtained; otherwise
 * as glr_prior_step.  Nothing is launched on an error. */
#define GLR_STATIC_SCRATCH_BYTES (64u << 20)
GLR_API glr_status glr_prior_step_static(glr_plan* plan, const void* x_in, float sigma,
                                         void* x_out, void* stream);

/* --------------------------------------------------------------- loop
 * Run outer iterations t_begin .. t_end-1 of the GAP/ADMM loop with the GLR
 * prior (sigma[t] per iteration).  state: device buffer of
 * glr_state_bytes() holding the loop state (iterate; MRI: x, z, u;
 * GAP_ACC: then the accumulated measurement [H][W]); when
 * t_begin == 0 it is initialised from y (CACTI: Phi^T(y / R~); MSFA: 4x4
 * cell replication; MRI: x = z = F^H(M y), u = 0; y_acc = y), otherwise it must hold
 * the state left by a previous call, so a run may be split and resumed.
 * x_out receives the current estimate (CACTI/MSFA: the last prior output;
 * MRI: z). */
GLR_API glr_status glr_state_bytes(const glr_plan* plan, size_t* bytes);
GLR_API glr_status glr_reconstruct(glr_plan* plan, const void* y, void* state, int32_t t_begin,
                           int32_t t_end, void* x_out, void* ws, void* stream);

/* The pre-prior iterate of the next iteration, from a loop state (as left by
 * glr_reconstruct, or initialised by it with t_begin = t_end = 0): the image
 * the prior step of that iteration receives.  CACTI/MSFA: the GAP data step
 * x + Phi^T((y - Phi x) / R~) of the state's iterate; MRI: v = x + u with
 * x = F^H((M y + rho F(z - u)) / (M + rho)) from the state's z and u.
 * v_out in the image layout, not aliasing the state; the state is not
 * changed. */
GLR_API glr_status glr_pre_prior(glr_plan* plan, const void* y, const void* state, void* v_out,
                                 void* ws, void* stream);

/* Synchronise the plan's last stream and copy the counters; reset != 0 zeroes
 * them afterwards. */
GLR_API glr_status glr_read_stats(glr_plan* plan, glr_stats* host_out, int32_t reset);

/* --------------------------------------------------------------- CNN surrogate
 * A learned stand-in for the prior step (not part of the paper's method; it
 * is judged against the GLR step, see glr_params.surrogate):
 *   x_out = x + f(x, sigma),  f = 3x3 conv 2->64, ReLU, 3 x (3x3 conv
 *   64->64, ReLU), 3x3 conv 64->1, zero padding, cross-correlation taps.
 * A slice is one 2-D image [h][w] (a CACTI frame, an MRI real or imaginary
 * plane, an MSFA band); the network input is (slice, constant sigma map).
 * params: device float [glr_cnn_param_count()] in the order W1 [64][2][3][3],
 * b1 [64], W2 [64][64][3][3], b2, W3, b3, W4, b4, W5 [1][64][3][3], b5 [1].
 * packed: device buffer of glr_cnn_packed_bytes() (256-byte aligned) holding
 * the BF16 weights and FP32 biases the kernels read; glr_cnn_pack() fills
 * it from params.  Weights and activations are BF16, sums FP32.  All
 * buffers are caller-owned; ws is a workspace of glr_cnn_workspace_size(). */
GLR_API int32_t glr_cnn_param_count(void);
GLR_API size_t glr_cnn_packed_bytes(void);
/* train != 0 sizes the workspace for glr_cnn_loss_grad. */
GLR_API glr_status glr_cnn_workspace_size(int32_t B, int32_t h, int32_t w, int32_t train,
                                          size_t* bytes);
GLR_API glr_status glr_cnn_pack(const float* params, void* packed, void* stream);
/* out[B][h][w] = x + f(x, sigma[b]) for slices x [B][h][w] (device float);
 * sigma: device float [B]. */
GLR_API glr_status glr_cnn_forward(const void* packed, const float* x, const float* sigma,
                                   float* out, int32_t B, int32_t h, int32_t w, void* ws,
                                   void* stream);
/* Mean squared error loss of the surrogate estimate against target
 * [B][h][w] into *loss (device float) and its gradient with respect to every
 * parameter into grad (device float [param_count], the params layout);
 * out [B][h][w] receives the surrogate estimate. */
GLR_API glr_status glr_cnn_loss_grad(const void* packed, const float* x, const float* sigma,
                                     const float* target, int32_t B, int32_t h, int32_t w,
                                     float* loss, float* grad, float* out, void* ws,
                                     void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
 * params with moments m, v (device float [param_count]); repacks packed. */
GLR_API glr_status glr_cnn_adam(float* params, float* m, float* v, const float* grad,
                                int32_t step, float lr, void* packed, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GLR_H */
