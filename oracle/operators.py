"""Sensing operators Phi, Phi^T and the data-fidelity updates (oracle).

* CACTI (eq. 2): one snapshot y = sum_t A_t * x_t of F mask-coded frames.
* MRI (eq. 3): y = M * F(x), F the orthonormal 2-D DFT, M a k_y-line mask.
* MSFA (eq. 4-5): y = sum_i A_i * x_i with disjoint (orthogonal) masks, so
  Phi Phi^T = I; the 4x4 periodic layout puts band 4*(r%4) + (c%4) at (r, c).
* GAP and ADMM updates (the iterative frameworks named with the low-rank
  objective in the Method section).

All arrays float64 / complex128.
"""
import numpy as np


# ---------------------------------------------------------------- CACTI (eq. 2)
def cacti_forward(x, masks):
    """y[r,c] = sum_t masks[t,r,c] * x[t,r,c]  (eq. 2)."""
    return np.sum(masks.astype(np.float64) * x, axis=0)


def cacti_adjoint(y, masks):
    """Phi^T y: frame t gets masks[t] * y."""
    return masks.astype(np.float64) * y[None]


def cacti_mask_sum(masks):
    """R = sum_t A_t (the diagonal of Phi Phi^T for binary masks)."""
    return np.sum(masks.astype(np.float64), axis=0)


# ---------------------------------------------------------------- MSFA (eq. 4-5)
def msfa_band_map(H, W):
    """Band index of each pixel for the 4x4 periodic filter array."""
    r = np.arange(H)[:, None] % 4
    c = np.arange(W)[None, :] % 4
    return 4 * r + c


def msfa_forward(x):
    """y[r,c] = x[b(r,c), r, c]: each pixel sees exactly one band (eq. 4-5)."""
    B, H, W = x.shape
    b = msfa_band_map(H, W)
    return np.take_along_axis(x, b[None], axis=0)[0]


def msfa_adjoint(y, bands):
    """Phi^T y: band b receives y where b(r,c) = b, zero elsewhere."""
    H, W = y.shape
    b = msfa_band_map(H, W)
    out = np.zeros((bands, H, W))
    for k in range(bands):
        out[k] = np.where(b == k, y, 0.0)
    return out


def msfa_init(y, bands):
    """Replication start: each band's single sample per 4x4 cell fills the cell."""
    H, W = y.shape
    out = np.zeros((bands, H, W))
    for k in range(bands):
        rb, cb = divmod(k, 4)
        cell = y[rb::4, cb::4]
        out[k] = np.repeat(np.repeat(cell, 4, axis=0), 4, axis=1)[:H, :W]
    return out


# ---------------------------------------------------------------- MRI (eq. 3)
def mri_mask2d(line_mask, W):
    """Expand a k_y-line mask ``[H]`` to the full k-space sampling mask."""
    return np.repeat(line_mask.astype(np.float64)[:, None], W, axis=1)


def fft2c(x):
    """Orthonormal 2-D DFT (the library routine)."""
    return np.fft.fft2(x, norm="ortho")


def ifft2c(k):
    """Orthonormal inverse 2-D DFT."""
    return np.fft.ifft2(k, norm="ortho")


def mri_forward(x, line_mask):
    """y = M * F(x)  (eq. 3)."""
    return mri_mask2d(line_mask, x.shape[1]) * fft2c(x)


def mri_adjoint(y, line_mask):
    """Phi^H y = F^H(M * y)."""
    return ifft2c(mri_mask2d(line_mask, y.shape[1]) * y)


# ---------------------------------------------------------------- solvers
def gap_update(x, y, forward, adjoint, R):
    """Generalized alternating projection step:
    x_bar = x + Phi^T((y - Phi x) / R~), R~ = R with zeros replaced by 1."""
    Rt = np.where(R == 0, 1.0, R)
    return x + adjoint((y - forward(x)) / Rt)


def gap_acc_update(x, y, y_acc, forward, adjoint, R):
    """Accelerated GAP step (reading: the measurement replaced by an
    accumulated one): y_acc' = y_acc + (y - Phi x), then
    x_bar = x + Phi^T((y_acc' - Phi x) / R~).  Returns (x_bar, y_acc')."""
    Rt = np.where(R == 0, 1.0, R)
    r = forward(x)
    y_acc = y_acc + (y - r)
    return x + adjoint((y_acc - r) / Rt), y_acc


def admm_x_update(y, z, u, line_mask, rho):
    """Closed-form ADMM data step for eq. 3:
    x = F^H((M*y + rho*F(z - u)) / (M + rho))."""
    M = mri_mask2d(line_mask, y.shape[1])
    return ifft2c((M * y + rho * fft2c(z - u)) / (M + rho))
