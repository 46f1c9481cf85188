"""The paper's edge-map matching score (eq. 6-8) on the GPU against the
oracle: groups and heat values exact (integers), the prior step and a
short loop built on them."""
import numpy as np
import pytest

import paper_2301_03047_amd as glr
import synth
from synth.workloads import random_image, small
from oracle import edges as oe, prior as opr, reconstruct as orc, metrics, detector as odet
from gpu_util import require_gpu, gpu, host, planar, ones_mask, WNNM_C, WNNM_EPS

pytestmark = pytest.mark.gpu

EDGE_CASES = [
    # C, H, W, P, N, K, kind
    (1, 40, 44, 5, 30, 12, "smooth"),
    (3, 37, 29, 7, 20, 9, "uniform"),
    (8, 64, 72, 6, 64, 32, "smooth"),
    (4, 24, 24, 4, 20, 11, "dup"),
    (24, 48, 56, 8, 40, 64, "smooth"),
    (2, 30, 30, 3, 25, 64, "flat"),
]


@pytest.mark.parametrize("case", EDGE_CASES, ids=lambda c: "x".join(map(str, c[:6])) + c[6])
def test_edge_score_groups_vs_oracle(case):
    require_gpu()
    C, H, W, P, N, K, kind = case
    print("edge case", case, flush=True)
    if kind == "flat":
        x = np.full((C, H, W), 0.4, np.float32)
    else:
        x = random_image(C, H, W, seed=H * W + C, kind=kind)
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.sort(np.random.default_rng(3).choice(n_cand, size=N, replace=False))
    plan = glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), score="edge")
    idx, heat = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    ref_idx, ref_heat = oe.topk_edge(x, P, keys, K)
    np.testing.assert_array_equal(host(idx), ref_idx)
    np.testing.assert_array_equal(host(heat), ref_heat)


def test_edge_score_complex_image():
    require_gpu()
    wl = synth.WORKLOADS["mri_256"]
    z = synth.make_instance(wl)["x_true"][64:192, 64:192].copy()
    P, N, K = 6, 100, 45
    plan = glr.Plan("mri", 128, 128, 1, P, N, K, mask=gpu(np.ones(128, np.uint8)), score="edge")
    zg = gpu(z)
    keys = host(plan.detect_keys(zg))
    idx, heat = plan.match_topk(zg, gpu(keys))
    ref_idx, ref_heat = oe.topk_edge(planar(z), P, keys, K, is_complex=True)
    np.testing.assert_array_equal(host(idx), ref_idx)
    np.testing.assert_array_equal(host(heat), ref_heat)


def test_edge_score_prior_step_and_loop_vs_oracle():
    require_gpu()
    C, H, W, P, N, K = 8, 48, 52, 6, 40, 16
    x = random_image(C, H, W, seed=41, kind="smooth")
    sigma = 0.05
    plan = glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), score="edge")
    out = host(plan.prior_step(gpu(x), sigma))
    ref = opr.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, WNNM_EPS, score="edge")
    err = metrics.rel_l2(out, ref["x_out"])
    print("edge-score prior step rel-L2", err, flush=True)
    assert err <= 1e-5
    wl = small(synth.WORKLOADS["cacti_128"], H=64, W=64, n_keys=48, k=16, iters=3, score="edge")
    x_true = synth.cacti_video(wl.C, wl.H, wl.W, 21)
    m = synth.cacti_masks(wl.C, wl.H, wl.W, 22)
    pl = glr.Plan.for_workload(wl, mask=gpu(m))
    y = pl.forward(gpu(x_true))
    g, _ = pl.reconstruct(y, 0, wl.iters)
    r = orc.reconstruct(small(wl, wnnm_c=WNNM_C), host(y).astype(np.float64), m,
                        synth.sigma_schedule(wl).astype(np.float64))
    e2 = metrics.rel_l2(host(g), r)
    print("edge-score loop rel-L2", e2, flush=True)
    assert e2 <= 1e-3
