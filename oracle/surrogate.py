"""The data-fidelity loop with the CNN surrogate and its GLR judge (oracle;
test infrastructure).

While t < ceil(frac * T) and the surrogate is active, the prior step is the
network's estimate x + f(x, sigma_t) on every slice (planar channel).  The
judge runs the GLR prior step on every ``stride``-th detected key and
measures the deviation on the pixels those groups cover; a deviation above
``delta_max`` (or a non-finite estimate) makes that iteration use the full
GLR step and deactivates the surrogate for the rest of the run.
``delta_max = inf`` skips the judge.  The network runs with the GPU's BF16
roundings (``cnn.forward(..., bf16=True)``).
"""
import math

import numpy as np

from . import operators as ops
from . import cnn
from .detector import detect_keys
from .prior import prior_step, to_planar, from_planar


def surrogate_prior(xp, wl, sigma, theta, stride, delta_max, is_complex=False):
    """Returns (x_out planar, accepted, delta)."""
    xp = np.asarray(xp, np.float64)
    x_cnn = cnn.forward(theta, xp, np.full(xp.shape[0], sigma), bf16=True)
    if math.isinf(delta_max):
        return x_cnn, True, None
    keys = detect_keys(xp, wl.patch, wl.n_keys, is_complex=is_complex)
    sub = keys[::stride]
    r = prior_step(xp, wl.patch, len(sub), wl.k, sigma, wl.wnnm_c, wl.wnnm_eps,
                   is_complex=is_complex, keys=sub)
    delta = cnn.judge_deviation(x_cnn, r["x_out"], r["count"] > 0)
    if delta <= delta_max:
        return x_cnn, True, delta
    full = prior_step(xp, wl.patch, wl.n_keys, wl.k, sigma, wl.wnnm_c, wl.wnnm_eps,
                      is_complex=is_complex)["x_out"]
    return full, False, delta


def reconstruct_surrogate(wl, y, mask, sigmas, theta, frac=0.6, stride=8, delta_max=0.02,
                          iters=None, callback=None):
    """Like ``reconstruct.reconstruct`` with the surrogate in early iterations.
    ``callback(t, used_cnn, delta)`` is called for every iteration."""
    T = wl.iters if iters is None else iters
    t_sur = math.ceil(frac * wl.iters)
    active = True

    def prior(t, xp, is_complex):
        nonlocal active
        if active and t < t_sur:
            out, ok, delta = surrogate_prior(xp, wl, sigmas[t], theta, stride, delta_max,
                                             is_complex)
            active = ok
            if callback:
                callback(t, ok, delta)
            return out
        if callback:
            callback(t, False, None)
        return prior_step(xp, wl.patch, wl.n_keys, wl.k, float(sigmas[t]), wl.wnnm_c,
                          wl.wnnm_eps, is_complex=is_complex)["x_out"]

    if wl.modality == "cacti":
        R = ops.cacti_mask_sum(mask)
        x = ops.cacti_adjoint(y / np.where(R == 0, 1.0, R), mask)
        for t in range(T):
            xb = ops.gap_update(x, y, lambda v: ops.cacti_forward(v, mask),
                                lambda r: ops.cacti_adjoint(r, mask), R)
            x = prior(t, xb, False)
        return x
    if wl.modality == "msfa":
        x = ops.msfa_init(y, wl.C)
        for t in range(T):
            xb = ops.gap_update(x, y, ops.msfa_forward, lambda r: ops.msfa_adjoint(r, wl.C),
                                np.ones_like(y))
            x = prior(t, xb, False)
        return x
    if wl.modality == "mri":
        z = ops.mri_adjoint(y, mask)
        u = np.zeros_like(z)
        for t in range(T):
            x = ops.admm_x_update(y, z, u, mask, wl.rho)
            v = x + u
            z = from_planar(prior(t, to_planar(v), True))
            u = u + x - z
        return z
    raise ValueError(wl.modality)
