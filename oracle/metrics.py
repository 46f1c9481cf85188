"""Accuracy metrics (the paper reports PSNR and SSIM, Results section).

PSNR = 10 log10(peak^2 / MSE); peak 1 for CACTI/MSFA (no clipping of the
estimate); for complex MRI data PSNR is taken on the magnitude with
peak = max |x_true|.  Relative L2 = ||a - b|| / ||b|| over all elements.
"""
import numpy as np


def psnr(est, ref, peak=None):
    est = np.asarray(est)
    ref = np.asarray(ref)
    if np.iscomplexobj(ref) or np.iscomplexobj(est):
        est = np.abs(est)
        ref = np.abs(ref)
        if peak is None:
            peak = float(ref.max())
    if peak is None:
        peak = 1.0
    mse = np.mean((est.astype(np.float64) - ref.astype(np.float64)) ** 2)
    return float(10.0 * np.log10(peak * peak / mse)) if mse > 0 else float("inf")


def rel_l2(a, b):
    a = np.asarray(a).astype(np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b).astype(a.dtype)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))
