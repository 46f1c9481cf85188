"""Pins for the oracle's surrogate loop: delta_max = 0 reduces to the plain
loop, a network with a zero output layer is the identity prior while the
surrogate runs, NaN weights always fall back."""
import math

import numpy as np

import synth
from synth.workloads import small
from synth.cnn import cnn_params
from oracle import reconstruct as orc, surrogate as osur, operators as ops, prior as opr, metrics


def _wl():
    return small(synth.WORKLOADS["cacti_128"], H=32, W=32, C=4, n_keys=24, k=8, iters=4)


def _inst(wl):
    inst = synth.make_instance(wl)
    y = orc.measure(wl, inst["x_true"], inst["mask"])
    return inst, y, synth.sigma_schedule(wl)


def test_delta_zero_is_the_plain_loop():
    wl = _wl()
    inst, y, sig = _inst(wl)
    used = []
    a = osur.reconstruct_surrogate(wl, y, inst["mask"], sig, cnn_params(0).astype(np.float64),
                                   delta_max=0.0, callback=lambda t, u, d: used.append(u))
    b = orc.reconstruct(wl, y, inst["mask"], sig)
    np.testing.assert_array_equal(a, b)
    assert not any(used)


def test_zero_output_layer_is_identity_prior_while_active():
    wl = _wl()
    inst, y, sig = _inst(wl)
    theta = cnn_params(1).astype(np.float64)
    theta[-577:] = 0.0                     # W5, b5 = 0  ->  f = 0
    a = osur.reconstruct_surrogate(wl, y, inst["mask"], sig, theta, frac=0.5,
                                   delta_max=float("inf"))
    m = inst["mask"]
    R = ops.cacti_mask_sum(m)
    x = ops.cacti_adjoint(y / np.where(R == 0, 1.0, R), m)
    for t in range(wl.iters):
        xb = ops.gap_update(x, y, lambda v: ops.cacti_forward(v, m),
                            lambda r: ops.cacti_adjoint(r, m), R)
        if t < 2:
            x = xb                         # identity prior, up to the BF16 path (x + 0)
        else:
            x = opr.prior_step(xb, wl.patch, wl.n_keys, wl.k, float(sig[t]), wl.wnnm_c,
                               wl.wnnm_eps)["x_out"]
    np.testing.assert_allclose(a, x, rtol=0, atol=1e-12)


def test_nan_weights_fall_back():
    wl = _wl()
    inst, y, sig = _inst(wl)
    theta = cnn_params(2).astype(np.float64)
    theta[5] = np.nan
    log = []
    a = osur.reconstruct_surrogate(wl, y, inst["mask"], sig, theta,
                                   callback=lambda t, u, d: log.append((u, d)))
    assert log[0] == (False, float("inf"))
    np.testing.assert_array_equal(a, orc.reconstruct(wl, y, inst["mask"], sig))


def test_ssim_pins():
    from oracle import metrics as om
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(2, 20, 24))
    assert abs(om.ssim(x, x) - 1.0) <= 1e-12
    y = np.clip(x + 0.1 * rng.standard_normal(x.shape), 0, 1)
    assert abs(om.ssim(x, y) - om.ssim(y, x)) <= 1e-12 and om.ssim(x, y) < 0.99
    # constant images: the structure term is C2 / C2 = 1, the luminance term
    # (2 a b + C1) / (a^2 + b^2 + C1)
    a, b = np.full((1, 15, 15), 0.3), np.full((1, 15, 15), 0.7)
    C1 = 0.01 ** 2
    assert abs(om.ssim(a, b) - (2 * 0.3 * 0.7 + C1) / (0.09 + 0.49 + C1)) <= 1e-12
    # a pure-Python window loop on a 13 x 14 image (three positions per row)
    u = rng.uniform(size=(13, 14))
    v = rng.uniform(size=(13, 14))
    t = np.arange(11) - 5.0
    g = [math.exp(-tt * tt / 4.5) for tt in t]
    s = sum(gi * gj for gi in g for gj in g)
    tot, n = 0.0, 0
    for i in range(3):
        for j in range(4):
            ma = mb = aa = bb = ab = 0.0
            for k in range(11):
                for l in range(11):
                    wk = g[k] * g[l] / s
                    p, q = u[i + k, j + l], v[i + k, j + l]
                    ma += wk * p
                    mb += wk * q
                    aa += wk * p * p
                    bb += wk * q * q
                    ab += wk * p * q
            va, vb, cab = aa - ma * ma, bb - mb * mb, ab - ma * mb
            C2 = 0.03 ** 2
            tot += ((2 * ma * mb + C1) * (2 * cab + C2)) / ((ma * ma + mb * mb + C1) * (va + vb + C2))
            n += 1
    assert abs(om.ssim(u, v) - tot / n) <= 1e-12


def test_package_metrics_match_the_oracle():
    # the package's evaluation metrics (separable filters) against the
    # oracle's definitions (explicit windows) on real and complex images
    from paper_2301_03047_amd import metrics as pm
    rng = np.random.default_rng(9)
    x = rng.uniform(size=(3, 40, 36))
    y = np.clip(x + 0.05 * rng.standard_normal(x.shape), 0, 1)
    assert abs(pm.ssim(y, x) - metrics.ssim(y, x)) <= 1e-10
    assert abs(pm.psnr(y, x) - metrics.psnr(y, x)) <= 1e-10
    z = x[0] * np.exp(1j * x[1])
    w = y[0] * np.exp(1j * y[1])
    assert abs(pm.ssim(w, z) - metrics.ssim(w, z)) <= 1e-10
