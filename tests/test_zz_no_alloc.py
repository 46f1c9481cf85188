"""The allocation-free prior step (glr_prior_step_static) against the
workspace form (glr_prior_step) on the same plans and inputs: both run the
same kernels, so outputs must be bitwise equal, call after call, while the
shared static scratch still holds what the previous call (another plan, a
larger or a differently laid out problem) left in it."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from paper_2301_03047_amd.glr import GlrError

from gpu_util import require_gpu, gpu, host, ones_mask, WNNM_C
from oracle import prior as oprior, metrics

pytestmark = pytest.mark.gpu


def _cacti_plan(C, H, W, P, N, K, precision="fp32"):
    return glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), precision=precision)


def _check_pair(plan, x, sigma, oracle_check=None):
    print(f"static prior step: {plan.C}x{plan.H}x{plan.W} P={plan.patch} N={plan.n_keys} "
          f"K={plan.k} ws={plan.workspace_bytes}", flush=True)
    assert plan.workspace_bytes <= glr.STATIC_SCRATCH_BYTES
    ref = plan.prior_step(x, sigma)
    out = plan.prior_step_static(x, sigma)
    a, b = host(ref), host(out)
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), "static and workspace forms differ"
    if oracle_check is not None:
        oracle_check(b)
    return b


def test_static_prior_step_matches_workspace_form_twice_then_smaller():
    require_gpu()
    torch.cuda.set_device(0)
    sigma = 0.05
    # first call: 4 x 48 x 52, 40 keys
    xa = synth.workloads.random_image(4, 48, 52, seed=31, kind="smooth")
    pa = _cacti_plan(4, 48, 52, 5, 40, 12)

    def vs_oracle(P, N, K, x):
        def chk(out):
            ref = oprior.prior_step(x.astype(np.float64), P, N, K, sigma, WNNM_C, 1e-16)
            err = metrics.rel_l2(out, ref["x_out"])
            assert err <= 1e-5, f"rel-L2 vs oracle {err:.3e}"
        return chk

    _check_pair(pa, gpu(xa), sigma, vs_oracle(5, 40, 12, xa))
    # second call on the same GPU: a smaller problem (3 x 32 x 36, 16 keys)
    # whose scratch region still holds the first call's buffers
    xb = synth.workloads.random_image(3, 32, 36, seed=32, kind="uniform")
    pb = _cacti_plan(3, 32, 36, 4, 16, 8)
    _check_pair(pb, gpu(xb), sigma, vs_oracle(4, 16, 8, xb))
    # and back to the first plan after the smaller one
    _check_pair(pa, gpu(xa), sigma)


def test_static_prior_step_mri_and_bf16_plans():
    require_gpu()
    torch.cuda.set_device(0)
    rng = np.random.default_rng(41)
    H = W = 64
    z = (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64)
    lines = torch.ones(H, dtype=torch.uint8, device="cuda")
    pm = glr.Plan("mri", H, W, 1, 6, 64, 16, mask=lines)
    _check_pair(pm, gpu(z), 0.1)
    x = synth.workloads.random_image(4, 48, 52, seed=33, kind="smooth")
    pbf = _cacti_plan(4, 48, 52, 5, 40, 12, precision="bf16")
    _check_pair(pbf, gpu(x), 0.05)


def test_static_prior_step_rejects_plans_above_the_scratch_size():
    require_gpu()
    C, H, W = 8, 256, 256
    p = glr.Plan("cacti", H, W, C, 6, 512, 32, mask=ones_mask(C, H, W), allocate=False)
    assert p.workspace_bytes > glr.STATIC_SCRATCH_BYTES
    x = torch.zeros((C, H, W), dtype=torch.float32, device="cuda")
    with pytest.raises(GlrError) as ei:
        p.prior_step_static(x, 0.05)
    assert ei.value.status == 5                      # GLR_ERR_WORKSPACE_TOO_SMALL
