"""GPU parity of the sensing operators, FFT, data steps and the full loop."""
import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from synth.workloads import small
from oracle import operators as ops, reconstruct as orc, metrics
from gpu_util import require_gpu, gpu, host, planar, WNNM_C

pytestmark = pytest.mark.gpu


def test_fft2d_vs_numpy():
    require_gpu()
    for H, W in [(256, 256), (8, 32), (64, 16)]:
        rng = np.random.default_rng(H + W)
        z = (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64)
        m = np.ones(H, np.uint8)
        plan = glr.Plan("mri", H, W, 1, 2, 4, 2, mask=gpu(m))
        f = host(plan.fft2d(gpu(z)))
        ref = np.fft.fft2(z.astype(np.complex128), norm="ortho")
        assert metrics.rel_l2(f, ref) <= 2e-6
        b = host(plan.fft2d(gpu(f), inverse=True))
        assert metrics.rel_l2(b, z) <= 2e-6


def test_mri_forward_adjoint_data_step():
    require_gpu()
    wl = synth.WORKLOADS["mri_256"]
    inst = synth.make_instance(wl)
    m = inst["mask"]
    x = inst["x_true"]
    plan = glr.Plan("mri", wl.H, wl.W, 1, wl.patch, wl.n_keys, wl.k, mask=gpu(m))
    y = host(plan.forward(gpu(x)))
    yref = ops.mri_forward(x.astype(np.complex128), m)
    assert metrics.rel_l2(y, yref) <= 2e-6
    y32 = yref.astype(np.complex64)
    xa = host(plan.adjoint(gpu(y32)))
    assert metrics.rel_l2(xa, ops.mri_adjoint(y32.astype(np.complex128), m)) <= 2e-6
    rng = np.random.default_rng(1)
    z = (x + 0.05 * rng.standard_normal(x.shape)).astype(np.complex64)
    u = (0.01 * rng.standard_normal(x.shape)).astype(np.complex64)
    xn = host(plan.data_step(gpu(y32), z=gpu(z), u=gpu(u)))
    ref = ops.admm_x_update(y32.astype(np.complex128), z.astype(np.complex128), u.astype(np.complex128), m, 1.0)
    assert metrics.rel_l2(xn, ref) <= 2e-6


def test_pre_prior_iterate():
    # the image the next prior step receives, from a loop state: the ADMM
    # x-update plus u (MRI), the GAP data step (CACTI); against the oracle's
    # operators on the state's own values
    require_gpu()
    wl = small(synth.WORKLOADS["mri_256"], H=64, W=64, n_keys=64, k=16, iters=3)
    inst = synth.make_instance(synth.WORKLOADS["mri_256"])
    x = inst["x_true"][96:160, 96:160].copy()
    m = synth.mri_line_mask(64, 5)
    sig = synth.sigma_schedule(wl)
    plan = glr.Plan("mri", wl.H, wl.W, 1, wl.patch, wl.n_keys, wl.k, iters=wl.iters, sigma=sig,
                    mask=gpu(m))
    y = plan.forward(gpu(x.astype(np.complex64)))
    state = plan.new_state()
    plan.reconstruct(y, 0, 2, state=state)
    v = host(plan.pre_prior(y, state))
    st = host(state)[: 3 * 64 * 64 * 8].view(np.complex64)
    z, u = st[4096:8192].reshape(64, 64), st[8192:].reshape(64, 64)
    xr = ops.admm_x_update(host(y).astype(np.complex128), z.astype(np.complex128),
                           u.astype(np.complex128), m, 1.0)
    assert metrics.rel_l2(v, xr + u) <= 2e-6
    F, H, W = 8, 48, 40
    mc = synth.cacti_masks(F, H, W, 2)
    xc = synth.workloads.random_image(F, H, W, seed=3)
    pc = glr.Plan("cacti", H, W, F, 4, 8, 4, iters=2, sigma=np.full(2, 0.05, np.float32),
                  mask=gpu(mc))
    yc = pc.forward(gpu(xc))
    sc = pc.new_state()
    pc.reconstruct(yc, 0, 1, state=sc)
    vc = host(pc.pre_prior(yc, sc))
    x1 = host(sc)[: F * H * W * 4].view(np.float32).reshape(F, H, W).astype(np.float64)
    ref = ops.gap_update(x1, host(yc).astype(np.float64), lambda q: ops.cacti_forward(q, mc),
                         lambda r: ops.cacti_adjoint(r, mc), ops.cacti_mask_sum(mc))
    assert np.abs(vc - ref).max() <= 1e-5


def test_gap_steps():
    require_gpu()
    F, H, W = 8, 48, 40
    m = synth.cacti_masks(F, H, W, 2)
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(F, H, W)).astype(np.float32)
    y = ops.cacti_forward(rng.uniform(size=(F, H, W)), m).astype(np.float32)
    plan = glr.Plan("cacti", H, W, F, 4, 8, 4, mask=gpu(m))
    xb = host(plan.data_step(gpu(y), x=gpu(x)))
    ref = ops.gap_update(x.astype(np.float64), y.astype(np.float64), lambda v: ops.cacti_forward(v, m),
                         lambda r: ops.cacti_adjoint(r, m), ops.cacti_mask_sum(m))
    assert np.abs(xb - ref).max() <= 1e-5
    # MSFA
    H, W = 32, 36
    x = rng.uniform(size=(16, H, W)).astype(np.float32)
    y = rng.uniform(size=(H, W)).astype(np.float32)
    plan = glr.Plan("msfa", H, W, 16, 4, 8, 4)
    yf = host(plan.forward(gpu(x)))
    np.testing.assert_array_equal(yf, ops.msfa_forward(x.astype(np.float64)).astype(np.float32))
    xb = host(plan.data_step(gpu(y), x=gpu(x)))
    ref = ops.gap_update(x.astype(np.float64), y.astype(np.float64), ops.msfa_forward,
                         lambda r: ops.msfa_adjoint(r, 16), np.ones((H, W)))
    assert np.abs(xb - ref).max() <= 1e-6


def _run_both(wl, iters):
    inst = synth.make_instance(wl)
    m = inst["mask"]
    y = orc.measure(wl, inst["x_true"], m)
    y32 = y.astype(np.complex64 if wl.modality == "mri" else np.float32)
    sig = synth.sigma_schedule(wl)
    plan = glr.Plan(wl.modality, wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, iters=wl.iters,
                    sigma=sig, mask=None if m is None else gpu(m))
    out, state = plan.reconstruct(gpu(y32), 0, iters)
    wl2 = small(wl, wnnm_c=WNNM_C)
    ref = orc.reconstruct(wl2, y32.astype(np.complex128 if wl.modality == "mri" else np.float64), m,
                          sig.astype(np.float64), iters=iters)
    return host(out), ref, inst["x_true"], plan, y32


def _real_per_iteration_parity(wl, plan, y32):
    """For t >= 1: the GPU prior step on the GPU's own pre-prior iterate
    (data step applied to the state) against the oracle's prior step on the
    same iterate: keys and groups exact, image within 1e-5."""
    from oracle import prior as opr
    from gpu_util import check_groups
    sig = synth.sigma_schedule(wl)
    yg = gpu(y32)
    state = plan.new_state()
    for t in range(wl.iters):
        if t > 0:
            x_t = state.view(torch.float32).view(wl.C, wl.H, wl.W)
            xb = plan.data_step(yg, x=x_t.contiguous())
            keys = host(plan.detect_keys(xb))
            idx, _ = plan.match_topk(xb, gpu(keys))
            pv = host(plan.prior_step(xb, float(sig[t])))
            xh = host(xb).astype(np.float64)
            r = opr.prior_step(xh, wl.patch, wl.n_keys, wl.k, float(sig[t]), WNNM_C, 1e-16)
            np.testing.assert_array_equal(keys, r["keys"])
            assert check_groups(xh, wl.patch, keys, host(idx), r["idx"]) == 0
            e = metrics.rel_l2(pv, r["x_out"])
            print(f"  t={t}: prior-step rel-L2 on the GPU iterate {e:.2e}")
            assert e <= 1e-5
        _, state = plan.reconstruct(yg, t, t + 1, state=state)


def test_reconstruct_cacti_small_vs_oracle():
    """Per iteration, the prior step on the GPU iterate matches the oracle
    (exact groups, 1e-5); the whole trajectory agrees with the oracle's FP64
    run up to the FP32 drift of the data steps (rel-L2 <= 1e-3,
    |dPSNR| <= 0.01 dB)."""
    require_gpu()
    wl = synth.WORKLOADS["cacti_128"]
    out, ref, xt, plan, y32 = _run_both(wl, wl.iters)
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, xt) - metrics.psnr(ref, xt)
    print(f"cacti_128: rel-L2 {err:.2e}, dPSNR {dp:.4f} dB, psnr {metrics.psnr(out, xt):.3f}")
    assert err <= 1e-3 and abs(dp) <= 0.01
    _real_per_iteration_parity(wl, plan, y32)


def test_reconstruct_msfa_small_vs_oracle():
    require_gpu()
    wl = small(synth.WORKLOADS["msfa_512"], H=64, W=64, n_keys=200, k=32, iters=3)
    out, ref, xt, plan, y32 = _run_both(wl, wl.iters)
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, xt) - metrics.psnr(ref, xt)
    print(f"msfa_64: rel-L2 {err:.2e}, dPSNR {dp:.4f} dB")
    assert err <= 1e-3 and abs(dp) <= 0.01
    _real_per_iteration_parity(wl, plan, y32)


def test_reconstruct_mri_per_iteration_parity_and_resume():
    """Every iteration: the oracle's prior step on the GPU's own pre-prior
    iterate v_t = x_t + u_t gives the same keys and groups and an image within
    1e-5.  The whole trajectory then agrees with the oracle's FP64 run up to
    the FP32 drift of the data steps (rel-L2 <= 1e-3, |dPSNR| <= 0.01 dB)."""
    require_gpu()
    from oracle import prior as opr
    wl = small(synth.WORKLOADS["mri_256"], iters=4)
    out, ref, xt, plan, y32 = _run_both(wl, wl.iters)
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, xt) - metrics.psnr(ref, xt)
    print(f"mri_256 (4 it): rel-L2 {err:.2e}, dPSNR {dp:.4f}")
    assert err <= 1e-3 and abs(dp) <= 0.01
    sig = synth.sigma_schedule(wl)
    HW = wl.H * wl.W
    state = plan.new_state()
    yg = gpu(y32)
    for t in range(wl.iters):
        if t > 0:
            st = state.view(torch.complex64)
            z, u = st[HW:2 * HW].view(wl.H, wl.W), st[2 * HW:].view(wl.H, wl.W)
            x_next = plan.data_step(yg, z=z.contiguous(), u=u.contiguous())
            v = (x_next + u).contiguous()
            keys = host(plan.detect_keys(v))
            idx, _ = plan.match_topk(v, gpu(keys))
            pv = host(plan.prior_step(v, float(sig[t])))
            vh = host(v)
            r = opr.prior_step(planar(vh), wl.patch, wl.n_keys, wl.k, float(sig[t]), WNNM_C,
                               1e-16, is_complex=True)
            np.testing.assert_array_equal(keys, r["keys"])
            from gpu_util import check_groups
            assert check_groups(planar(vh), wl.patch, keys, host(idx), r["idx"]) == 0
            e = metrics.rel_l2(pv, opr.from_planar(r["x_out"]))
            print(f"  t={t}: prior-step rel-L2 on the GPU iterate {e:.2e}")
            assert e <= 1e-5
        _, state = plan.reconstruct(yg, t, t + 1, state=state)
    # a run split at t=2 and resumed equals the straight run bit for bit
    a, st = plan.reconstruct(yg, 0, 2)
    b, _ = plan.reconstruct(yg, 2, wl.iters, state=st)
    np.testing.assert_array_equal(host(b), out)


@pytest.mark.parametrize("modality", ["cacti", "msfa"])
def test_accelerated_gap_loop_vs_oracle(modality):
    # accelerated GAP: every pre-prior iterate against the oracle's step on
    # the GPU's own state, and a three-iteration loop against the oracle's
    require_gpu()
    if modality == "cacti":
        wl = small(synth.WORKLOADS["cacti_128"], H=48, W=56, n_keys=24, k=16, iters=3,
                   gap_acc=True)
        x_true = synth.cacti_video(wl.C, wl.H, wl.W, 7)
        m = synth.cacti_masks(wl.C, wl.H, wl.W, 8)
        fwd = lambda v: ops.cacti_forward(v, m)
        adj = lambda r: ops.cacti_adjoint(r, m)
        R = ops.cacti_mask_sum(m)
        mask = gpu(m)
    else:
        wl = small(synth.WORKLOADS["msfa_512"], H=48, W=48, n_keys=24, k=16, iters=3,
                   gap_acc=True)
        x_true = synth.msfa_cube(wl.C, wl.H, wl.W, 9)
        m = None
        fwd = ops.msfa_forward
        adj = lambda r: ops.msfa_adjoint(r, wl.C)
        R = np.ones((wl.H, wl.W))
        mask = None
    plan = glr.Plan.for_workload(wl, mask=mask)
    y = plan.forward(gpu(x_true))
    y64 = host(y).astype(np.float64)
    state = plan.new_state()
    plan.reconstruct(y, 0, 0, state=state)
    n = wl.C * wl.H * wl.W
    for t in range(wl.iters):
        st = host(state)
        x = st[: 4 * n].view(np.float32).reshape(wl.C, wl.H, wl.W).astype(np.float64)
        ya = st[4 * n: 4 * n + 4 * wl.H * wl.W].view(np.float32).reshape(wl.H, wl.W)
        xb_ref, _ = ops.gap_acc_update(x, y64, ya.astype(np.float64), fwd, adj, R)
        xb = host(plan.pre_prior(y, state))
        assert np.abs(xb - xb_ref).max() <= 1e-5, (modality, t)
        plan.reconstruct(y, t, t + 1, state=state)
    out, _ = plan.reconstruct(y, 0, wl.iters)
    ref = orc.reconstruct(small(wl, wnnm_c=WNNM_C), y64, m,
                          synth.sigma_schedule(wl).astype(np.float64))
    err = metrics.rel_l2(host(out), ref)
    print(modality, "accelerated GAP loop rel-L2", err, flush=True)
    assert err <= 1e-3


@pytest.mark.parametrize("modality", ["cacti", "mri"])
def test_inner_wnnm_iterations_loop_vs_oracle(modality):
    # three outer iterations with two inner WNNM iterations per prior step
    # (MRI: the complex iterate's planar form) against the oracle's loop
    require_gpu()
    if modality == "cacti":
        wl = small(synth.WORKLOADS["cacti_128"], H=48, W=56, n_keys=24, k=16, iters=3,
                   wnnm_iters=2)
        x_true = synth.cacti_video(wl.C, wl.H, wl.W, 21)
        m = synth.cacti_masks(wl.C, wl.H, wl.W, 22)
    else:
        wl = small(synth.WORKLOADS["mri_256"], H=64, W=64, n_keys=64, k=16, iters=3,
                   wnnm_iters=2)
        x_true = synth.mri_phantom(wl.H, wl.W, 23)
        m = synth.mri_line_mask(wl.H, 24)
    plan = glr.Plan.for_workload(wl, mask=gpu(m))
    y = plan.forward(gpu(x_true))
    out, _ = plan.reconstruct(y, 0, wl.iters)
    out = host(out)
    yh = host(y).astype(np.complex128 if modality == "mri" else np.float64)
    ref = orc.reconstruct(small(wl, wnnm_c=WNNM_C), yh, m,
                          synth.sigma_schedule(wl).astype(np.float64))
    one = orc.reconstruct(small(wl, wnnm_c=WNNM_C, wnnm_iters=1), yh, m,
                          synth.sigma_schedule(wl).astype(np.float64))
    err = metrics.rel_l2(out, ref)
    dp = metrics.psnr(out, x_true) - metrics.psnr(ref, x_true)
    print(f"{modality} inner x2 loop rel-L2 {err:.2e} dPSNR {dp:.4f}; "
          f"vs one shrinkage {metrics.rel_l2(one, ref):.2e}", flush=True)
    assert err <= 1e-3 and abs(dp) <= 0.01
    assert metrics.rel_l2(one, ref) > 10 * err
