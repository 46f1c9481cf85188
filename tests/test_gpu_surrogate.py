"""The CNN surrogate inside the reconstruction loop, through the C ABI:
fallback rules (delta_max = 0 and NaN weights reduce to the plain loop bit
for bit), the judge's deviation against the oracle on the same iterate, a
surrogate-only trajectory against the oracle's, and resume."""
import math

import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from synth.workloads import small
from synth.cnn import cnn_params
from oracle import reconstruct as orc, surrogate as osur, metrics, prior as opr
from gpu_util import require_gpu, gpu, host, planar, WNNM_C

pytestmark = pytest.mark.gpu


def _setup(name, **kw):
    wl = small(synth.WORKLOADS[name], **kw)
    inst = synth.make_instance(wl)
    y = orc.measure(wl, inst["x_true"], inst["mask"])
    y32 = y.astype(np.complex64 if wl.modality == "mri" else np.float32)
    return wl, inst, y32, synth.sigma_schedule(wl)


def _plan(wl, inst, sig, cnn=None, **kw):
    m = inst["mask"]
    return glr.Plan(wl.modality, wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, iters=wl.iters,
                    sigma=sig, mask=None if m is None else gpu(m), cnn=cnn, **kw)


CASES = [("cacti_128", dict(iters=5)), ("mri_256", dict(iters=4, n_keys=128))]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_delta_zero_and_nan_weights_equal_plain(name, kw):
    require_gpu()
    wl, inst, y32, sig = _setup(name, **kw)
    yg = gpu(y32)
    plain, _ = _plan(wl, inst, sig).reconstruct(yg)
    plain = host(plain)
    # delta_max = 0: the first judged step falls back and the surrogate stops
    net = glr.Cnn(cnn_params(0))
    p0 = _plan(wl, inst, sig, cnn=net, judge_delta_max=0.0)
    a, _ = p0.reconstruct(yg)
    st = p0.read_stats()
    assert st["fallback_steps"] == 1 and st["surrogate_steps"] == 0
    np.testing.assert_array_equal(host(a), plain)
    # NaN weights: non-finite estimate -> deviation +inf -> fallback
    th = cnn_params(0)
    th[7] = np.nan
    pn = _plan(wl, inst, sig, cnn=glr.Cnn(th))
    b, _ = pn.reconstruct(yg)
    st = pn.read_stats()
    assert st["fallback_steps"] == 1 and math.isinf(st["judge_delta_last"])
    np.testing.assert_array_equal(host(b), plain)


def test_judge_deviation_vs_oracle():
    # first iteration of a judged run: the deviation the GPU measured against
    # the oracle's on the GPU's own pre-prior iterate (same CNN, BF16 roundings)
    require_gpu()
    wl, inst, y32, sig = _setup("cacti_128", iters=5)
    th = cnn_params(3, out_scale=0.02)
    p = _plan(wl, inst, sig, cnn=glr.Cnn(th), judge_delta_max=1e9)
    yg = gpu(y32)
    state = p.new_state()
    p.reconstruct(yg, 0, 1, state=state)
    d_gpu = p.read_stats()["judge_delta_last"]
    # the pre-prior iterate of t = 0 from the data step on the initial estimate
    p2 = _plan(wl, inst, sig)
    st2 = p2.new_state()
    p2.reconstruct(yg, 0, 0, state=st2)               # t_begin == 0 initialises x0 only
    x0 = st2.view(torch.float32).view(wl.C, wl.H, wl.W)
    xb = host(p2.data_step(yg, x=x0.contiguous())).astype(np.float64)
    wl2 = small(wl, wnnm_c=WNNM_C)
    _, ok, d_ref = osur.surrogate_prior(xb, wl2, float(sig[0]), th.astype(np.float64), 8, 1e9)
    print(f"judge delta gpu {d_gpu:.6f} oracle {d_ref:.6f}", flush=True)
    assert ok and abs(d_gpu - d_ref) <= 2e-3 * d_ref


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_surrogate_only_trajectory_vs_oracle_and_resume(name, kw):
    require_gpu()
    wl, inst, y32, sig = _setup(name, **kw)
    th = cnn_params(5, out_scale=0.02)
    p = _plan(wl, inst, sig, cnn=glr.Cnn(th), judge_delta_max=float("inf"))
    yg = gpu(y32)
    out, _ = p.reconstruct(yg)
    st = p.read_stats()
    assert st["surrogate_steps"] == math.ceil(0.6 * wl.iters)
    out = host(out)
    wl2 = small(wl, wnnm_c=WNNM_C)
    ydt = np.complex128 if wl.modality == "mri" else np.float64
    ref = osur.reconstruct_surrogate(wl2, y32.astype(ydt), inst["mask"], sig.astype(np.float64),
                                     th.astype(np.float64), delta_max=float("inf"))
    e = metrics.rel_l2(out, ref)
    xt = inst["x_true"]
    dp = metrics.psnr(out, xt) - metrics.psnr(ref, xt)
    print(f"{name}: surrogate-only trajectory rel-L2 {e:.2e}, dPSNR {dp:.4f} dB", flush=True)
    # BF16 activations that round to the neighbouring value (see the CNN
    # parity tests) plus the FP32 data steps; the PSNR must not move
    assert e <= 5e-3 and abs(dp) <= 0.02
    # split at t = 2 (inside the surrogate phase) and resumed: bit for bit
    a, stt = p.reconstruct(yg, 0, 2)
    b, _ = p.reconstruct(yg, 2, wl.iters, state=stt)
    np.testing.assert_array_equal(host(b), out)
