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


def _gauss11():
    """The 11 x 11 Gaussian window of SSIM (standard deviation 1.5), sum 1."""
    t = np.arange(11) - 5.0
    g = np.exp(-(t * t) / (2.0 * 1.5 * 1.5))
    w = np.outer(g, g)
    return w / w.sum()


def ssim(est, ref, peak=None):
    """Structural similarity (Wang, Bovik, Sheikh, Simoncelli 2004; the
    paper's second metric): on every 11 x 11 window position fully inside
    the image (Gaussian weights, standard deviation 1.5) the local means,
    variances and covariance give
    ((2 mu_a mu_b + C1)(2 s_ab + C2)) / ((mu_a^2 + mu_b^2 + C1)(s_a^2 + s_b^2 + C2)),
    C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L = peak; the mean over positions of
    each 2-D slice ([C][H][W]: every channel) is averaged over slices.
    Complex data: the magnitude, with peak max |ref| (as for PSNR)."""
    est = np.asarray(est)
    ref = np.asarray(ref)
    if np.iscomplexobj(ref) or np.iscomplexobj(est):
        est, ref = np.abs(est), np.abs(ref)
        if peak is None:
            peak = float(ref.max())
    if peak is None:
        peak = 1.0
    a = np.asarray(est, dtype=np.float64)
    b = np.asarray(ref, dtype=np.float64)
    if a.ndim == 2:
        a, b = a[None], b[None]
    C1, C2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    w = _gauss11()
    from numpy.lib.stride_tricks import sliding_window_view
    vals = []
    for sa, sb in zip(a, b):
        A = sliding_window_view(sa, (11, 11))
        B = sliding_window_view(sb, (11, 11))
        ma = np.einsum("ijkl,kl->ij", A, w)
        mb = np.einsum("ijkl,kl->ij", B, w)
        va = np.einsum("ijkl,kl->ij", A * A, w) - ma * ma
        vb = np.einsum("ijkl,kl->ij", B * B, w) - mb * mb
        cab = np.einsum("ijkl,kl->ij", A * B, w) - ma * mb
        m = ((2 * ma * mb + C1) * (2 * cab + C2)) / ((ma * ma + mb * mb + C1) * (va + vb + C2))
        vals.append(m.mean())
    return float(np.mean(vals))
