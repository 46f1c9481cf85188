"""Image-quality figures of a reconstruction (host arrays): PSNR and SSIM,
the paper's two metrics (Results section).  Evaluation only, never part of
the reconstruction.

PSNR = 10 log10(peak^2 / MSE), peak 1 for real images; complex images are
compared on the magnitude with peak max |ref|.
SSIM (Wang et al. 2004): an 11 x 11 Gaussian window (standard deviation
1.5), C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L the same peak, averaged over
the window positions that lie inside the image, per 2-D slice, then over
the slices.  The windowed moments are separable Gaussian filters.
"""
import numpy as np
from scipy import ndimage


def _prep(est, ref):
    est, ref = np.asarray(est), np.asarray(ref)
    peak = 1.0
    if np.iscomplexobj(est) or np.iscomplexobj(ref):
        est, ref = np.abs(est), np.abs(ref)
        peak = float(ref.max())
    return est.astype(np.float64), ref.astype(np.float64), peak


def psnr(est, ref):
    est, ref, peak = _prep(est, ref)
    mse = float(np.mean((est - ref) ** 2))
    return float(10.0 * np.log10(peak * peak / mse)) if mse > 0 else float("inf")


def _gauss(v):
    """Separable 11-tap Gaussian filter (sigma 1.5, normalised) of a 2-D
    slice, kept only where the window lies inside the slice."""
    t = np.arange(-5, 6, dtype=np.float64)
    k = np.exp(-0.5 * (t / 1.5) ** 2)
    k /= k.sum()
    f = ndimage.correlate1d(ndimage.correlate1d(v, k, axis=0, mode="constant"), k, axis=1,
                            mode="constant")
    return f[5:-5, 5:-5]


def ssim(est, ref):
    a, b, peak = _prep(est, ref)
    if a.ndim == 2:
        a, b = a[None], b[None]
    C1, C2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    out = []
    for sa, sb in zip(a, b):
        ma, mb = _gauss(sa), _gauss(sb)
        saa = _gauss(sa * sa) - ma * ma
        sbb = _gauss(sb * sb) - mb * mb
        sab = _gauss(sa * sb) - ma * mb
        num = (2.0 * ma * mb + C1) * (2.0 * sab + C2)
        den = (ma * ma + mb * mb + C1) * (saa + sbb + C2)
        out.append(float(np.mean(num / den)))
    return float(np.mean(out))
