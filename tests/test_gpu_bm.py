"""The block-matching baselines on the GPU against the oracle: uniform and
corner-plus-uniform exemplars, local-window matching (eq. 1, vanilla BM)
with exact groups, and the prior step and loop built on them."""
import numpy as np
import pytest

import paper_2301_03047_amd as glr
import synth
from synth.workloads import random_image, small
from oracle import detector as odet, matching as om, prior as opr, reconstruct as orc, metrics
from gpu_util import require_gpu, gpu, host, ones_mask, check_groups, WNNM_C, WNNM_EPS

pytestmark = pytest.mark.gpu


def _plan(C, H, W, P, N, K, **kw):
    return glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), **kw)


WINDOW_CASES = [
    # C, H, W, P, K, radius, kind   (windows clipped at every border, odd/even P)
    (2, 40, 44, 5, 12, 6, "smooth"),
    (3, 37, 29, 7, 9, 4, "uniform"),
    (4, 24, 24, 4, 11, 5, "dup"),
    (8, 64, 80, 6, 32, 20, "smooth"),
    (1, 30, 30, 16, 6, 3, "smooth"),
    (24, 48, 56, 8, 64, 10, "smooth"),
]


@pytest.mark.parametrize("case", WINDOW_CASES, ids=lambda c: "x".join(map(str, c[:6])) + c[6])
def test_window_topk_vs_oracle(case):
    require_gpu()
    C, H, W, P, K, R, kind = case
    print("window case", case, flush=True)
    x = random_image(C, H, W, seed=H + W + P, kind=kind)
    Hc, Wc = H - P + 1, W - P + 1
    rng = np.random.default_rng(5)
    keys = np.sort(rng.choice(Hc * Wc, size=min(40, Hc * Wc), replace=False))
    keys = np.unique(np.concatenate([keys, [0, Wc - 1, (Hc - 1) * Wc, Hc * Wc - 1]]))
    plan = _plan(C, H, W, P, len(keys), K, search="window", window=R)
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    idx, dist = host(idx), host(dist)
    ref_idx, ref_dist = om.window_topk(x.astype(np.float64), P, keys, K, R)
    assert check_groups(x.astype(np.float64), P, keys, idx, ref_idx) == 0
    np.testing.assert_allclose(dist, ref_dist, rtol=1e-6, atol=1e-30)


def test_exemplar_keys_vs_oracle():
    require_gpu()
    x = random_image(4, 60, 70, seed=12, kind="smooth")
    P, N, s = 5, 20, 3
    for mode in ("uniform", "corner_uniform", "corner"):
        plan = _plan(4, 60, 70, P, N, 8, exemplars=mode, uniform_step=s)
        keys = host(plan.detect_keys(gpu(x)))
        ref = odet.exemplar_keys(x, P, N, mode, s)
        assert plan.n_keys == len(ref), mode
        np.testing.assert_array_equal(keys, ref)


@pytest.mark.parametrize("mode", ["uniform", "corner_uniform"])
def test_block_matching_prior_step_vs_oracle(mode):
    require_gpu()
    C, H, W, P, N, K, R, s = 8, 48, 52, 6, 24, 16, 8, 4
    x = random_image(C, H, W, seed=31, kind="smooth")
    sigma = 0.05
    plan = _plan(C, H, W, P, N, K, exemplars=mode, uniform_step=s, search="window", window=R)
    xg = gpu(x)
    keys = host(plan.detect_keys(xg))
    idx = host(plan.match_topk(xg, gpu(keys))[0])
    out = host(plan.prior_step(xg, sigma))
    ref = opr.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, WNNM_EPS,
                         exemplars=mode, step=s, search="window", radius=R)
    np.testing.assert_array_equal(keys, ref["keys"])
    assert check_groups(x.astype(np.float64), P, keys, idx, ref["idx"]) == 0
    err = metrics.rel_l2(out, ref["x_out"])
    print(mode, "prior step rel-L2", err, flush=True)
    assert err <= 1e-5


def test_block_matching_loop_vs_oracle():
    # three GAP iterations of the corner-plus-uniform block-matching variant
    require_gpu()
    wl = small(synth.WORKLOADS["cacti_256"], H=64, W=64, n_keys=32, k=16, iters=3,
               exemplars="corner_uniform", uniform_step=4, search="window", window=10)
    x_true = synth.cacti_video(wl.C, wl.H, wl.W, 17)
    m = synth.cacti_masks(wl.C, wl.H, wl.W, 18)
    plan = glr.Plan.for_workload(wl, mask=gpu(m))
    y = plan.forward(gpu(x_true))
    out, _ = plan.reconstruct(y, 0, wl.iters)
    out = host(out)
    wl64 = small(wl, wnnm_c=WNNM_C)
    ref = orc.reconstruct(wl64, host(y).astype(np.float64), m,
                          synth.sigma_schedule(wl).astype(np.float64))
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, x_true) - metrics.psnr(ref, x_true)
    print("block-matching loop rel-L2", err, "dPSNR", dp, flush=True)
    assert err <= 1e-3 and abs(dp) <= 0.01
