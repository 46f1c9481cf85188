"""The data-fidelity loop around the prior (oracle).

x = argmin sum_i rank(R_i x) s.t. y = Phi x, solved by GAP (CACTI, MSFA) or
ADMM (MRI) alternating a data step with the GLR prior step (Method section).

Readings: plain GAP, x0 = Phi^T(y / R~) for CACTI and the 4x4-cell replication
for MSFA; ADMM with x0 = z0 = F^H(M y), u0 = 0, then per iteration
x = F^H((M y + rho F(z - u)) / (M + rho)), v = x + u, z = prior(v),
u = u + x - z.  One prior step per iteration, keys re-detected every
iteration on the current pre-prior iterate.
"""
import numpy as np

from . import operators as ops
from .prior import prior_step, to_planar, from_planar


def _prior(xp, wl, sigma, is_complex):
    return prior_step(xp, wl.patch, wl.n_keys, wl.k, float(sigma), wl.wnnm_c,
                      wl.wnnm_eps, is_complex=is_complex,
                      exemplars=getattr(wl, "exemplars", "corner"),
                      step=getattr(wl, "uniform_step", 4),
                      search=getattr(wl, "search", "global"),
                      radius=getattr(wl, "window", 20),
                      score=getattr(wl, "score", "l2"),
                      agg_weights=getattr(wl, "agg_weights", "uniform"),
                      inner=getattr(wl, "wnnm_iters", 1),
                      delta=getattr(wl, "wnnm_delta", 0.1),
                      lam=getattr(wl, "wnnm_lambda", 0.54),
                      lowrank=getattr(wl, "lowrank", "stacked"))["x_out"]


def reconstruct(wl, y, mask, sigmas, iters=None, callback=None):
    """Run ``iters`` (default ``wl.iters``) outer iterations.

    ``y``: measurement (float64 ``[H][W]`` or complex ``[H][W]`` for mri);
    ``mask``: cacti ``[F][H][W]`` u8, mri ``[H]`` u8, msfa None.
    ``callback(t, pre_prior, post_prior)`` is called each iteration.
    Returns the final estimate (real ``[C][H][W]`` or complex ``[H][W]``)."""
    T = wl.iters if iters is None else iters
    acc = getattr(wl, "gap_acc", False)
    if wl.modality in ("cacti", "msfa"):
        if wl.modality == "cacti":
            R = ops.cacti_mask_sum(mask)
            x = ops.cacti_adjoint(y / np.where(R == 0, 1.0, R), mask)
            fwd = lambda v: ops.cacti_forward(v, mask)
            adj = lambda r: ops.cacti_adjoint(r, mask)
        else:
            R = np.ones_like(y)
            x = ops.msfa_init(y, wl.C)
            fwd = ops.msfa_forward
            adj = lambda r: ops.msfa_adjoint(r, wl.C)
        y_acc = np.array(y, dtype=np.float64)
        for t in range(T):
            if acc:
                xb, y_acc = ops.gap_acc_update(x, y, y_acc, fwd, adj, R)
            else:
                xb = ops.gap_update(x, y, fwd, adj, R)
            x = _prior(xb, wl, sigmas[t], False)
            if callback:
                callback(t, xb, x)
        return x
    if wl.modality == "mri":
        z = ops.mri_adjoint(y, mask)
        u = np.zeros_like(z)
        for t in range(T):
            x = ops.admm_x_update(y, z, u, mask, wl.rho)
            v = x + u
            z = from_planar(_prior(to_planar(v), wl, sigmas[t], True))
            u = u + x - z
            if callback:
                callback(t, v, z)
        return z
    raise ValueError(wl.modality)


def measure(wl, x_true, mask):
    """y = Phi x_true for the workload's modality (FP64)."""
    if wl.modality == "cacti":
        return ops.cacti_forward(np.asarray(x_true, np.float64), mask)
    if wl.modality == "msfa":
        return ops.msfa_forward(np.asarray(x_true, np.float64))
    if wl.modality == "mri":
        return ops.mri_forward(np.asarray(x_true, np.complex128), mask)
    raise ValueError(wl.modality)
