"""GPU parity of every step of the GLR prior step against the CPU oracle,
through the C ABI.  Same FP32 inputs on both sides (the oracle upcasts
exactly).  Bar: keys and groups bit-exact (up to certified numerical ties,
see gpu_util.check_groups), images and singular values within 1e-5 relative."""
import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from synth.workloads import random_image
from oracle import detector as odet, matching as om, lowrank as olr, aggregate as oag
from oracle import prior as opr, metrics
from gpu_util import require_gpu, gpu, host, planar, ones_mask, check_groups, WNNM_C, WNNM_EPS

pytestmark = pytest.mark.gpu


def _plan(C, H, W, P, N, K, **kw):
    return glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), **kw)


MATCH_CASES = [
    # C, H, W, P, N, K, kind          (ragged key tiles / candidate tiles / odd P)
    (2, 12, 12, 3, 5, 5, "uniform"),
    (2, 21, 150, 3, 17, 5, "smooth"),
    (8, 40, 41, 6, 130, 32, "smooth"),
    (3, 37, 29, 7, 50, 64, "uniform"),
    (1, 64, 300, 5, 257, 45, "smooth"),
    (2, 30, 30, 1, 40, 9, "uniform"),
    (1, 40, 40, 16, 20, 8, "smooth"),
    (4, 24, 24, 4, 30, 11, "dup"),
    # stage heights of the tiled FP32 matcher for P2 = 10 and 12, and the
    # small-patch (persistent) matcher with P2 = 8
    (2, 40, 60, 9, 40, 10, "smooth"),
    (1, 40, 40, 11, 30, 8, "uniform"),
    (1, 45, 140, 7, 70, 12, "smooth"),
    # more than 32 channels: the epilogue's channel-mean term in two passes
    (40, 36, 44, 4, 30, 16, "smooth"),
    (40, 30, 30, 3, 25, 9, "uniform"),
]


@pytest.mark.parametrize("case", MATCH_CASES, ids=lambda c: "x".join(map(str, c[:6])) + c[6])
def test_match_topk_vs_oracle(case):
    require_gpu()
    C, H, W, P, N, K, kind = case
    print("case", case, flush=True)
    x = random_image(C, H, W, seed=H * W + P, kind=kind)
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.sort(np.random.default_rng(7).choice(n_cand, size=N, replace=False))
    plan = _plan(C, H, W, P, N, K)
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    idx, dist = host(idx), host(dist)
    ref_idx, ref_dist = om.topk_exact(x.astype(np.float64), P, keys, K)
    ties = check_groups(x.astype(np.float64), P, keys, idx, ref_idx)
    assert ties == 0, f"{ties} numerical-tie rows"
    np.testing.assert_allclose(dist, ref_dist, rtol=1e-6, atol=1e-30)


def test_match_topk_small_chunks_and_splits():
    # force several distance chunks (1 MiB) and many splits
    require_gpu()
    C, H, W, P, N, K = 3, 64, 200, 5, 300, 20
    x = random_image(C, H, W, seed=3, kind="smooth")
    keys = np.arange(0, N * 37, 37)
    plan = _plan(C, H, W, P, N, K, dist_chunk_mb=1)
    idx, _ = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    ref, _ = om.topk_exact(x.astype(np.float64), P, keys, K)
    assert check_groups(x.astype(np.float64), P, keys, host(idx), ref) == 0


@pytest.mark.parametrize("H,W", [(40, 50), (200, 200)])
def test_match_topk_constant_image_exact_path(H, W):
    # every distance is exactly 0: the certified margin holds every candidate
    # and the range lists overflow.  With at most 32768 candidates the margin
    # set is re-derived from the distance row and rescored from global memory
    # (40 x 50); above that the exact full-row path runs (200 x 200, 38809
    # candidates).  Ties resolve to the lowest positions either way.
    require_gpu()
    C, P, N, K = 2, 4, 6, 10
    x = np.full((C, H, W), 0.3, dtype=np.float32)
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.linspace(0, n_cand - 1, N).astype(np.int64)
    plan = _plan(C, H, W, P, N, K)
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    st = plan.read_stats()
    np.testing.assert_array_equal(host(idx), np.tile(np.arange(K), (N, 1)))
    assert np.all(host(dist) == 0)
    if n_cand <= 32768:
        assert st["regather_keys"] == N and st["overflow_keys"] == 0
        assert st["margin_max"] == n_cand
    else:
        assert st["overflow_keys"] == N


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_match_topk_list_overflow_regather(precision):
    # the top 16 rows are one constant value, the rest is random: keys up
    # there see ~2000 exact ties, most of them in the first candidate range,
    # whose list overflows; their margin sets are re-derived from the
    # distance rows.  Keys below keep the ordinary paths.
    require_gpu()
    C, H, W, P, N, K = 2, 128, 192, 4, 24, 32
    x = random_image(C, H, W, seed=77, kind="uniform")
    x[:, :16, :] = np.float32(0.4)
    Wc = W - P + 1
    n_cand = (H - P + 1) * Wc
    top = np.array([r * Wc + c for r in (0, 3, 7, 12) for c in (0, 50, 100)])
    rest = np.random.default_rng(9).choice(np.arange(13 * Wc, n_cand), size=N - len(top),
                                           replace=False)
    keys = np.sort(np.concatenate([top, rest]))
    plan = _plan(C, H, W, P, N, K, precision=precision)
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    st = plan.read_stats()
    print("regather", st["regather_keys"], "overflow", st["overflow_keys"], "margin max",
          st["margin_max"], "rematch", st["rematch_keys"], flush=True)
    ref_idx, ref_dist = om.topk_exact(x.astype(np.float64), P, keys, K)
    np.testing.assert_array_equal(host(idx), ref_idx)
    np.testing.assert_allclose(host(dist), ref_dist, rtol=1e-6, atol=1e-30)
    assert st["regather_keys"] >= len(top) and st["overflow_keys"] == 0


def test_detect_keys_real_vs_oracle():
    require_gpu()
    for (C, H, W, P, N, kind, seed) in [(1, 20, 23, 4, 9, "uniform", 1), (8, 128, 128, 6, 128, "scene", 0),
                                         (3, 50, 61, 5, 400, "smooth", 2), (2, 16, 16, 3, 50, "const", 0)]:
        print("detect", C, H, W, P, N, kind, flush=True)
        if kind == "scene":
            x = synth.make_instance(synth.WORKLOADS["cacti_128"])["x_true"]
        elif kind == "const":
            x = np.full((C, H, W), 0.25, np.float32)
        else:
            x = random_image(C, H, W, seed=seed, kind=kind)
        plan = _plan(C, H, W, P, N, 4)
        keys = host(plan.detect_keys(gpu(x)))
        ref = odet.detect_keys(x, P, N)
        np.testing.assert_array_equal(keys, ref)


def test_detect_keys_complex_vs_oracle():
    require_gpu()
    wl = synth.WORKLOADS["mri_256"]
    inst = synth.make_instance(wl)
    z = inst["x_true"]
    plan = glr.Plan("mri", wl.H, wl.W, 1, wl.patch, wl.n_keys, wl.k, mask=gpu(inst["mask"]))
    keys = host(plan.detect_keys(gpu(z)))
    ref = odet.detect_keys(planar(z), wl.patch, wl.n_keys, is_complex=True)
    np.testing.assert_array_equal(keys, ref)


@pytest.mark.parametrize("shape", [(8, 40, 40, 6, 60, 32), (2, 30, 33, 5, 40, 45),
                                   (16, 32, 32, 6, 20, 64), (1, 20, 20, 3, 10, 1),
                                   (1, 24, 24, 3, 12, 16),
                                   # the 1024^2 x 24 CACTI group shape: D = 1536, K = 64
                                   (24, 64, 64, 8, 40, 64)])
def test_lowrank_aggregate_vs_oracle(shape):
    require_gpu()
    C, H, W, P, N, K = shape
    print("lowrank", shape, flush=True)
    x = random_image(C, H, W, seed=C + H, kind="smooth")
    x64 = x.astype(np.float64)
    keys = odet.detect_keys(x, P, N)
    idx, _ = om.topk_exact(x64, P, keys, K)
    sigma = 0.05
    plan = _plan(C, H, W, P, N, K)
    out, sv = plan.lowrank_aggregate(gpu(x), gpu(idx.astype(np.int32)), sigma, want_sv=True)
    Xhat, sv_ref = olr.shrink_groups(x64, P, idx, sigma, WNNM_C, WNNM_EPS)
    ref, _ = oag.aggregate(x64, P, idx, Xhat)
    err = metrics.rel_l2(host(out), ref)
    assert err <= 1e-5, err
    svg = host(sv)[:, :sv_ref.shape[1]]
    assert np.abs(svg - sv_ref).max() <= 1e-5 * sv_ref.max()


@pytest.mark.parametrize("shape", [(8, 40, 40, 6, 60, 32), (16, 32, 32, 6, 20, 64)])
def test_lowrank_tiny_scale_image(shape):
    # an image scaled by 2^-66: column norms near 1e-20, squared norms
    # subnormal in FP32.  A Householder reflector scaled by 2 / ||v||^2
    # overflows there; the unit-leading form must stay finite and match the
    # oracle on the same scaled input (to the precision subnormal squares
    # leave, about 2^-17 of the largest singular value)
    require_gpu()
    C, H, W, P, N, K = shape
    print("tiny scale", shape, flush=True)
    s = 2.0 ** -66
    x = (random_image(C, H, W, seed=C + H, kind="smooth") * np.float32(s)).astype(np.float32)
    x64 = x.astype(np.float64)
    keys = odet.detect_keys(x, P, N)
    idx, _ = om.topk_exact(x64, P, keys, K)
    sigma = 0.05 * s
    plan = _plan(C, H, W, P, N, K)
    out, sv = plan.lowrank_aggregate(gpu(x), gpu(idx.astype(np.int32)), sigma, want_sv=True)
    out, svg = host(out), host(sv)[:, :K]
    assert np.isfinite(out).all() and np.isfinite(svg).all()
    Xhat, sv_ref = olr.shrink_groups(x64, P, idx, sigma, WNNM_C, WNNM_EPS)
    ref, _ = oag.aggregate(x64, P, idx, Xhat)
    err = metrics.rel_l2(out, ref)
    sv_err = np.abs(svg - sv_ref).max() / sv_ref.max()
    print(f"  rel-L2 {err:.2e}, sv err {sv_err:.2e}", flush=True)
    assert err <= 1e-5 and sv_err <= 1e-3


@pytest.mark.parametrize("shape", [(8, 40, 40, 6, 60, 32), (2, 30, 33, 5, 40, 45),
                                   (24, 64, 64, 8, 40, 64)])
def test_rank_weighted_aggregation_vs_oracle(shape):
    # per-group weights 1 / (kept WNNM rank): the GPU takes the kept/not
    # decision in FP32 on its own singular values, so the seeded inputs are
    # checked to hold no value near its threshold (the oracle's decisions do
    # not move under a 1e-4 change of sigma)
    require_gpu()
    C, H, W, P, N, K = shape
    print("rank weights", shape, flush=True)
    x = random_image(C, H, W, seed=C + H + 1, kind="smooth")
    x64 = x.astype(np.float64)
    keys = odet.detect_keys(x, P, N)
    idx, _ = om.topk_exact(x64, P, keys, K)
    sigma = 0.05
    Xhat, sv_ref = olr.shrink_groups(x64, P, idx, sigma, WNNM_C, WNNM_EPS)
    w = olr.group_weights(sv_ref, K, sigma, WNNM_C, WNNM_EPS)
    for f in (1 - 1e-4, 1 + 1e-4):
        np.testing.assert_array_equal(w, olr.group_weights(sv_ref, K, sigma * f, WNNM_C, WNNM_EPS))
    assert len(np.unique(w)) > 1
    plan = _plan(C, H, W, P, N, K, agg_weights="rank")
    out = host(plan.lowrank_aggregate(gpu(x), gpu(idx.astype(np.int32)), sigma))
    ref, _ = oag.aggregate(x64, P, idx, Xhat, weights=w)
    uni, _ = oag.aggregate(x64, P, idx, Xhat)
    err = metrics.rel_l2(out, ref)
    print(f"  rel-L2 {err:.2e} (uniform vs weighted {metrics.rel_l2(uni, ref):.2e})", flush=True)
    assert err <= 1e-5
    assert metrics.rel_l2(uni, ref) > 100 * max(err, 1e-8)


def test_rank_weighted_prior_step_vs_oracle():
    require_gpu()
    C, H, W, P, N, K = 8, 64, 72, 6, 80, 32
    x = random_image(C, H, W, seed=77, kind="smooth")
    sigma = 0.04
    plan = _plan(C, H, W, P, N, K, agg_weights="rank")
    out = host(plan.prior_step(gpu(x), sigma))
    ref = opr.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, WNNM_EPS,
                         agg_weights="rank")
    for f in (1 - 1e-4, 1 + 1e-4):       # no kept/not decision near its threshold
        np.testing.assert_array_equal(
            ref["weights"], olr.group_weights(ref["sv"], K, sigma * f, WNNM_C, WNNM_EPS))
    err = metrics.rel_l2(out, ref["x_out"])
    print("rank-weighted prior step rel-L2", err, flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("J", [2, 3])
def test_inner_wnnm_iterations_prior_step_vs_oracle(J):
    # the same groups shrunk J times with iterative regularisation; the noise
    # level of iterations 2..J is estimated on the device
    require_gpu()
    C, H, W, P, N, K = 8, 56, 60, 6, 60, 32
    print("inner iterations", J, flush=True)
    x = random_image(C, H, W, seed=91, kind="smooth")
    sigma = 0.05
    plan = _plan(C, H, W, P, N, K, wnnm_iters=J)
    out = host(plan.prior_step(gpu(x), sigma))
    ref = opr.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, WNNM_EPS, inner=J)
    one = opr.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, WNNM_EPS)
    err = metrics.rel_l2(out, ref["x_out"])
    print(f"  rel-L2 {err:.2e}, sigmas {ref['sigmas']}, "
          f"vs one shrinkage {metrics.rel_l2(one['x_out'], ref['x_out']):.2e}", flush=True)
    assert err <= 1e-5
    assert metrics.rel_l2(one["x_out"], ref["x_out"]) > 100 * max(err, 1e-8)


def test_identity_shrink_returns_input_exactly():
    require_gpu()
    C, H, W, P, N, K = 3, 30, 30, 4, 40, 12
    x = (np.random.default_rng(3).integers(0, 256, size=(C, H, W)) / 256.0).astype(np.float32)
    plan = _plan(C, H, W, P, N, K)
    out = plan.prior_step(gpu(x), 0.0)
    np.testing.assert_array_equal(host(out), x)


def test_prior_step_cacti_iterate_vs_oracle():
    require_gpu()
    wl = synth.WORKLOADS["cacti_128"]
    inst = synth.make_instance(wl)
    m = inst["mask"]
    from oracle import operators as ops
    y = ops.cacti_forward(inst["x_true"].astype(np.float64), m)
    R = ops.cacti_mask_sum(m)
    x0 = ops.cacti_adjoint(y / np.where(R == 0, 1, R), m)
    xb = ops.gap_update(x0, y, lambda v: ops.cacti_forward(v, m), lambda r: ops.cacti_adjoint(r, m), R)
    x = xb.astype(np.float32)
    sigma = float(synth.sigma_schedule(wl)[0])
    plan = glr.Plan("cacti", wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, mask=gpu(m))
    xg = gpu(x)
    keys = host(plan.detect_keys(xg))
    idx, _ = plan.match_topk(xg, gpu(keys))
    out = host(plan.prior_step(xg, sigma))
    ref = opr.prior_step(x.astype(np.float64), wl.patch, wl.n_keys, wl.k, sigma, WNNM_C, WNNM_EPS)
    np.testing.assert_array_equal(keys, ref["keys"])
    assert check_groups(x.astype(np.float64), wl.patch, keys, host(idx), ref["idx"]) == 0
    err = metrics.rel_l2(out, ref["x_out"])
    assert err <= 1e-5, err
    st = plan.read_stats()
    print("stats", st)


def test_prior_step_mri_full_size_vs_oracle():
    require_gpu()
    wl = synth.WORKLOADS["mri_256"]
    inst = synth.make_instance(wl)
    rng = np.random.default_rng(5)
    z = (inst["x_true"] + 0.03 * (rng.standard_normal((wl.H, wl.W)) + 1j * rng.standard_normal((wl.H, wl.W)))).astype(np.complex64)
    sigma = 0.03
    plan = glr.Plan("mri", wl.H, wl.W, 1, wl.patch, wl.n_keys, wl.k, mask=gpu(inst["mask"]))
    zg = gpu(z)
    keys = host(plan.detect_keys(zg))
    idx, dist = plan.match_topk(zg, gpu(keys))
    out = host(plan.prior_step(zg, sigma))
    ref = opr.prior_step(planar(z), wl.patch, wl.n_keys, wl.k, sigma, WNNM_C, WNNM_EPS, is_complex=True)
    np.testing.assert_array_equal(keys, ref["keys"])
    ties = check_groups(planar(z), wl.patch, keys, host(idx), ref["idx"])
    assert ties == 0, ties
    err = metrics.rel_l2(out, opr.from_planar(ref["x_out"]))
    assert err <= 1e-5, err
    print("stats", plan.read_stats())


def test_prior_step_deterministic():
    require_gpu()
    C, H, W, P, N, K = 8, 64, 64, 6, 100, 32
    x = random_image(C, H, W, seed=9, kind="smooth")
    plan = _plan(C, H, W, P, N, K)
    a = host(plan.prior_step(gpu(x), 0.04))
    b = host(plan.prior_step(gpu(x), 0.04))
    np.testing.assert_array_equal(a, b)


def test_msfa_512_full_size_prior_step_vs_oracle():
    # the 512 x 512 x 16-band MSFA workload at its real size (4096 keys over
    # 507^2 candidates, FP32 matcher), first GAP iterate: keys bit-exact,
    # every group equal to the oracle's exact top-K except rows whose
    # differing members tie within 1e-9 of the row's distances (the GPU's
    # FP64 sums and the oracle's FP64 sums, in their own orders, order such near-ties
    # by their own roundings; check_groups verifies those rows' distance
    # profiles), the whole prior step within rel-L2 1e-5 of the oracle's
    require_gpu()
    from oracle import operators as ops
    wl = synth.WORKLOADS["msfa_512"]
    inst = synth.make_instance(wl)
    y = ops.msfa_forward(inst["x_true"].astype(np.float64))
    x0 = ops.msfa_init(y, wl.C)
    xb = ops.gap_update(x0, y, ops.msfa_forward, lambda r: ops.msfa_adjoint(r, wl.C),
                        np.ones_like(y)).astype(np.float32)
    sigma = float(synth.sigma_schedule(wl)[0])
    plan = glr.Plan("msfa", wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k)
    xg = gpu(xb)
    keys = host(plan.detect_keys(xg))
    idx = host(plan.match_topk(xg, gpu(keys))[0])
    out = host(plan.prior_step(xg, sigma))
    print("oracle prior step of msfa_512 ...", flush=True)
    ref = opr.prior_step(xb.astype(np.float64), wl.patch, wl.n_keys, wl.k, sigma, WNNM_C, WNNM_EPS)
    np.testing.assert_array_equal(keys, ref["keys"])
    ties = check_groups(xb.astype(np.float64), wl.patch, keys, idx, ref["idx"])
    err = metrics.rel_l2(out, ref["x_out"])
    print(f"msfa_512: {ties} numerical-tie rows of {wl.n_keys}, prior step rel-L2 {err:.3e}",
          flush=True)
    assert ties <= wl.n_keys // 100, ties
    assert err <= 1e-5, err


def test_msfa_512_full_size_sampled_keys():
    # the 512 x 512 x 16-band MSFA workload at its real size (4096 keys over
    # 507^2 candidates, FP32 matcher): sampled keys against the oracle's
    # direct-sum distance map; the prior step of the whole image is finite
    # and moves the iterate
    require_gpu()
    from oracle import operators as ops
    wl = synth.WORKLOADS["msfa_512"]
    inst = synth.make_instance(wl)
    y = ops.msfa_forward(inst["x_true"].astype(np.float64))
    x0 = ops.msfa_init(y, wl.C)
    xb = ops.gap_update(x0, y, ops.msfa_forward, lambda r: ops.msfa_adjoint(r, wl.C),
                        np.ones_like(y)).astype(np.float32)
    plan = glr.Plan("msfa", wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k)
    xg = gpu(xb)
    keys = host(plan.detect_keys(xg))
    np.testing.assert_array_equal(keys, odet.detect_keys(xb.astype(np.float64), wl.patch,
                                                         wl.n_keys))
    idx, dist = plan.match_topk(xg, gpu(keys))
    idx, dist = host(idx), host(dist)
    st = plan.read_stats()
    print("msfa_512 margins mean", st["margin_sum"] / wl.n_keys, "max", st["margin_max"],
          "overflow", st["overflow_keys"], flush=True)
    x64 = xb.astype(np.float64)
    rng = np.random.default_rng(23)
    for a in sorted(rng.choice(wl.n_keys, size=4, replace=False).tolist()):
        ref_idx, ref_d, _ = om.topk_one(x64, wl.patch, int(keys[a]), wl.k)
        if not np.array_equal(idx[a], ref_idx):
            dmap = om.distance_map(x64, wl.patch, int(keys[a]))
            assert np.abs(np.sort(dmap[idx[a]]) - ref_d).max() <= 1e-9 * float(ref_d.max()), a
        np.testing.assert_allclose(dist[a], ref_d, rtol=1e-6, atol=1e-30)
    out = host(plan.prior_step(xg, float(synth.sigma_schedule(wl)[0])))
    assert np.isfinite(out).all() and metrics.rel_l2(out, xb) > 0
