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


def gather_groups(x, patch, idx):
    """Group matrices ``[N][K][D]`` (member-major) from iterate ``x``."""
    from .matching import patch_matrix
    pm = patch_matrix(x, patch)
    return pm[np.asarray(idx)]


def shrink_groups(x, patch, idx, sigma, c, eps):
    """WNNM of every group: returns X_hat ``[N][K][D]`` and singular values
    ``[N][min(D,K)]`` (descending)."""
    G = gather_groups(x, patch, idx)
    N, K, D = G.shape
    out = np.empty_like(G)
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
