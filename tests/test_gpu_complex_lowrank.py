"""GPU parity of the complex-Hermitian low-rank form (complex MRI data shrunk
as complex P^2 x K groups) against the oracle, through the C ABI.  Bar: images
and singular values within 1e-5 relative (one step), 1e-3 after three ADMM
iterations (the FP32 loop's drift, as for the other loop tests)."""
import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from synth.workloads import random_image, small
from oracle import matching as om, lowrank as olr, aggregate as oag
from oracle import prior as opr, reconstruct as orc, metrics
from gpu_util import require_gpu, gpu, host, planar, check_groups, WNNM_C, WNNM_EPS

pytestmark = pytest.mark.gpu


def _image(H, W, seed):
    x = random_image(2, H, W, seed=seed, kind="smooth")
    return (x[0] - 0.5 + 1j * (x[1] - 0.5)).astype(np.complex64)


def _keys(H, W, P, N, seed):
    n_cand = (H - P + 1) * (W - P + 1)
    return np.sort(np.random.default_rng(seed).choice(n_cand, size=N, replace=False))


@pytest.mark.parametrize("shape", [
    # H, W, P, N, K: K > P^2 (rank-deficient Gram matrix), K < P^2, the
    # 64-member form with P^2 = 9, one member, two row chunks (P = 8), one
    # partial chunk (P = 2); MRI image sides are powers of two
    (32, 32, 6, 60, 45), (32, 64, 5, 40, 20), (16, 32, 3, 12, 64), (16, 16, 4, 10, 1),
    (32, 32, 8, 16, 33), (16, 16, 2, 20, 7)])
def test_complex_lowrank_aggregate_vs_oracle(shape):
    require_gpu()
    H, W, P, N, K = shape
    print("complex lowrank", shape, flush=True)
    z = _image(H, W, H + W + P)
    zp = planar(z)
    keys = _keys(H, W, P, N, K)
    idx, _ = om.topk_exact(zp, P, keys, K)
    sigma = 0.05
    mask = torch.ones(H, dtype=torch.uint8, device="cuda")
    plan = glr.Plan("mri", H, W, 1, P, N, K, mask=mask, lowrank="complex")
    out, sv = plan.lowrank_aggregate(gpu(z), gpu(idx.astype(np.int32)), sigma, want_sv=True)
    Xhat, sv_ref = olr.shrink_groups(zp, P, idx, sigma, WNNM_C, WNNM_EPS, complex_groups=True)
    ref, _ = oag.aggregate(zp, P, idx, Xhat)
    ref = opr.from_planar(ref)
    Xs, _ = olr.shrink_groups(zp, P, idx, sigma, WNNM_C, WNNM_EPS)
    stacked = opr.from_planar(oag.aggregate(zp, P, idx, Xs)[0])
    out = host(out)
    err = metrics.rel_l2(out, ref)
    svg = host(sv)[:, :sv_ref.shape[1]]
    sv_err = np.abs(svg - sv_ref).max() / max(sv_ref.max(), 1e-30)    # K = 1: all zero
    print(f"  rel-L2 {err:.2e}, sv err {sv_err:.2e}, "
          f"stacked vs complex {metrics.rel_l2(stacked, ref):.2e}", flush=True)
    assert err <= 1e-5 and sv_err <= 1e-5
    if K > 1:
        assert metrics.rel_l2(stacked, ref) > 100 * max(err, 1e-8)


def test_complex_lowrank_phase_equivariance():
    # a global phase e^{i theta} on the image turns the estimate by the same
    # phase (the groups do not change: distances are phase-invariant)
    require_gpu()
    H, W, P, N, K = 32, 32, 6, 60, 45
    z = _image(H, W, 5)
    keys = _keys(H, W, P, N, 6)
    idx, _ = om.topk_exact(planar(z), P, keys, K)
    mask = torch.ones(H, dtype=torch.uint8, device="cuda")
    plan = glr.Plan("mri", H, W, 1, P, N, K, mask=mask, lowrank="complex")
    ig = gpu(idx.astype(np.int32))
    ph = np.complex64(np.exp(0.9j))
    a = host(plan.lowrank_aggregate(gpu(z), ig, 0.05))
    b = host(plan.lowrank_aggregate(gpu((z * ph).astype(np.complex64)), ig, 0.05))
    err = metrics.rel_l2(b, a * ph)
    print("phase equivariance rel-L2", err, flush=True)
    assert err <= 1e-5


def test_complex_prior_step_mri_full_size_vs_oracle():
    require_gpu()
    wl = synth.WORKLOADS["mri_256"]
    inst = synth.make_instance(wl)
    rng = np.random.default_rng(5)
    z = (inst["x_true"] + 0.03 * (rng.standard_normal((wl.H, wl.W)) +
                                  1j * rng.standard_normal((wl.H, wl.W)))).astype(np.complex64)
    sigma = 0.03
    plan = glr.Plan("mri", wl.H, wl.W, 1, wl.patch, wl.n_keys, wl.k, mask=gpu(inst["mask"]),
                    lowrank="complex")
    zg = gpu(z)
    keys = host(plan.detect_keys(zg))
    idx, _ = plan.match_topk(zg, gpu(keys))
    out = host(plan.prior_step(zg, sigma))
    ref = opr.prior_step(planar(z), wl.patch, wl.n_keys, wl.k, sigma, WNNM_C, WNNM_EPS,
                         is_complex=True, lowrank="complex")
    np.testing.assert_array_equal(keys, ref["keys"])
    assert check_groups(planar(z), wl.patch, keys, host(idx), ref["idx"]) == 0
    err = metrics.rel_l2(out, opr.from_planar(ref["x_out"]))
    st = plan.read_stats()
    print(f"complex prior step rel-L2 {err:.2e}, sweeps max {st['jacobi_sweeps_max']}", flush=True)
    assert err <= 1e-5


def test_complex_lowrank_admm_loop_vs_oracle():
    # three ADMM iterations with the complex form against the oracle's loop
    require_gpu()
    wl = small(synth.WORKLOADS["mri_256"], H=64, W=64, n_keys=64, k=40, iters=3,
               lowrank="complex")
    x_true = synth.mri_phantom(wl.H, wl.W, 31)
    m = synth.mri_line_mask(wl.H, 32)
    plan = glr.Plan.for_workload(wl, mask=gpu(m))
    y = plan.forward(gpu(x_true))
    out, _ = plan.reconstruct(y, 0, wl.iters)
    out = host(out)
    yh = host(y).astype(np.complex128)
    sig = synth.sigma_schedule(wl).astype(np.float64)
    ref = orc.reconstruct(small(wl, wnnm_c=WNNM_C), yh, m, sig)
    st = orc.reconstruct(small(wl, wnnm_c=WNNM_C, lowrank="stacked"), yh, m, sig)
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, x_true) - metrics.psnr(ref, x_true)
    print(f"complex ADMM loop rel-L2 {err:.2e} dPSNR {dp:.4f}; "
          f"vs stacked {metrics.rel_l2(st, ref):.2e}", flush=True)
    assert err <= 1e-3 and abs(dp) <= 0.01
    assert metrics.rel_l2(st, ref) > 10 * err
