"""Pins for the oracle's surrogate loop: delta_max = 0 reduces to the plain
loop, a network with a zero output layer is the identity prior while the
surrogate runs, NaN weights always fall back."""
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
