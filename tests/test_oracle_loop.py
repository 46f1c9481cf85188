"""Sanity checks of the oracle's reconstruction loop (parity of the loop
itself is unpinned beyond its parts: there is no printed example)."""
import numpy as np

import synth
from synth.workloads import small
from oracle import reconstruct as rc, metrics, operators as ops


def test_mri_loop_improves_on_zero_filled():
    wl = small(synth.WORKLOADS["mri_256"], H=64, W=64, n_keys=160, k=16, iters=4,
               sigma0=0.02, sigma1=0.01)
    inst = synth.make_instance(wl)
    y = rc.measure(wl, inst["x_true"], inst["mask"])
    x0 = ops.mri_adjoint(y, inst["mask"])
    x = rc.reconstruct(wl, y, inst["mask"], synth.sigma_schedule(wl))
    assert metrics.psnr(x, inst["x_true"]) > metrics.psnr(x0, inst["x_true"])


def test_cacti_loop_runs_and_is_consistent():
    wl = small(synth.WORKLOADS["cacti_128"], H=48, W=48, C=4, n_keys=64, k=12, iters=2)
    inst = synth.make_instance(wl)
    y = rc.measure(wl, inst["x_true"], inst["mask"])
    seen = []
    rc.reconstruct(wl, y, inst["mask"], synth.sigma_schedule(wl),
                   callback=lambda t, a, b: seen.append((a, b)))
    R = ops.cacti_mask_sum(inst["mask"])
    # every pre-prior iterate satisfies the measurement where a mask is open
    for a, _ in seen:
        np.testing.assert_allclose(ops.cacti_forward(a, inst["mask"])[R > 0], y[R > 0], atol=1e-12)


def test_msfa_loop_keeps_measured_samples():
    wl = small(synth.WORKLOADS["msfa_512"], H=32, W=32, n_keys=48, k=10, iters=2)
    inst = synth.make_instance(wl)
    y = rc.measure(wl, inst["x_true"], None)
    seen = []
    rc.reconstruct(wl, y, None, synth.sigma_schedule(wl),
                   callback=lambda t, a, b: seen.append(a))
    for a in seen:
        np.testing.assert_allclose(ops.msfa_forward(a), y, atol=1e-15)
