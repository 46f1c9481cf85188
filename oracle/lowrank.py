"""Weighted nuclear-norm (WNNM) shrinkage of one patch group (oracle).

The paper solves the low-rank objective (the rank-minimisation equation of
the Method section) with WNNM [Gu et al. 2014].  Reading taken (constants
not printed in the paper): for a group Y (D x K, column j = member patch j),
subtract the row mean mu, take the SVD Yc = U S V^T, estimate the clean
singular values sigma_hat_i = sqrt(max(s_i^2 - K sigma^2, 0)), set weights
tau_i = c sqrt(K) sigma^2 / (sigma_hat_i + eps) and shrink
s'_i = max(s_i - tau_i, 0).  The estimate is written in residual form
X = Y - sum_i (s_i - s'_i) u_i v_i^T, so sigma = 0 returns Y exactly.
The SVD is LAPACK's (numpy.linalg.svd), in FP64.
"""
import numpy as np


def wnnm_weights(s, K, sigma, c, eps):
    """Shrunk singular values s' for singular values ``s`` of a K-member group."""
    s = np.asarray(s, dtype=np.float64)
    shat = np.sqrt(np.maximum(s * s - K * sigma * sigma, 0.0))
    tau = c * np.sqrt(K) * sigma * sigma / (shat + eps)
    return np.maximum(s - tau, 0.0)


def wnnm_group(Y, sigma, c, eps):
    """Shrink one group ``Y`` (D x K).  Returns (X_hat D x K, singular values)."""
    Y = np.asarray(Y, dtype=np.float64)
    D, K = Y.shape
    mu = Y.mean(axis=1, keepdims=True)
    U, s, Vt = np.linalg.svd(Y - mu, full_matrices=False)
    s_new = wnnm_weights(s, K, sigma, c, eps)
    X = Y - (U * (s - s_new)[None, :]) @ Vt
    return X, s


def wnnm_group_complex(Z, sigma, c, eps):
    """Shrink one complex group ``Z`` (d x K complex, column j = member j) by
    the same WNNM rule on the complex SVD Zc = U S V^H (variant for complex
    data; the default stacks [Re; Im] into a real 2d x K group).  Reading:
    the row mean mu is the complex mean, K is the member count and sigma the
    noise level per real component, as in the real form.  LAPACK's complex
    SVD, FP64.  Returns (X_hat d x K complex, singular values)."""
    Z = np.asarray(Z, dtype=np.complex128)
    d, K = Z.shape
    mu = Z.mean(axis=1, keepdims=True)
    U, s, Vh = np.linalg.svd(Z - mu, full_matrices=False)
    s_new = wnnm_weights(s, K, sigma, c, eps)
    X = Z - (U * (s - s_new)[None, :]) @ Vh
    return X, s


def gather_groups(x, patch, idx):
    """Group matrices ``[N][K][D]`` (member-major) from iterate ``x``."""
    from .matching import patch_matrix
    pm = patch_matrix(x, patch)
    return pm[np.asarray(idx)]


def shrink_groups(x, patch, idx, sigma, c, eps, complex_groups=False):
    """WNNM of every group: returns X_hat ``[N][K][D]`` and singular values
    ``[N][min(D,K)]`` (descending).  With ``complex_groups`` the iterate is
    planar complex ``[2][H][W]`` (Re, Im): each member's D = 2 P^2 entries
    [Re; Im] form one complex P^2-vector, the group is shrunk by
    ``wnnm_group_complex`` and written back as [Re; Im]; the singular values
    are then ``[N][min(P^2, K)]``."""
    G = gather_groups(x, patch, idx)
    N, K, D = G.shape
    out = np.empty_like(G)
    if complex_groups:
        d = D // 2
        sv = np.empty((N, min(d, K)))
        for g in range(N):
            X, s = wnnm_group_complex((G[g, :, :d] + 1j * G[g, :, d:]).T, sigma, c, eps)
            out[g, :, :d] = X.T.real
            out[g, :, d:] = X.T.imag
            sv[g] = s
        return out, sv
    sv = np.empty((N, min(D, K)))
    for g in range(N):
        X, s = wnnm_group(G[g].T, sigma, c, eps)
        out[g] = X.T
        sv[g] = s
    return out, sv


def group_weights(sv, K, sigma, c, eps):
    """Per-group aggregation weights (variant; reading: the inverse of the
    shrunk group's rank, 1 / max(r, 1) with r the number of singular values
    WNNM keeps non-zero, so groups the low-rank model describes with fewer
    components weigh more).  ``sv`` ``[N][min(D, K)]``."""
    r = np.sum(wnnm_weights(np.asarray(sv, dtype=np.float64), K, sigma, c, eps) > 0, axis=1)
    return 1.0 / np.maximum(r, 1)
