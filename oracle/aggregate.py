"""Aggregation of the shrunk groups back into an image (oracle).

Reading taken: every member estimate is put back at its patch position with
weight 1; each pixel is the mean of all estimates covering it; pixels that no
member covers keep the pre-prior value.
"""
import numpy as np


def aggregate(xbar, patch, idx, Xhat, weights=None):
    """x_out from x_bar ``[C][H][W]``, member positions ``idx [N][K]`` (top-left
    grid indices) and estimates ``Xhat [N][K][D]``.  With ``weights`` ``[N]``
    every estimate of group g weighs weights[g] and a pixel is the weighted
    mean of its covering estimates (the per-group weighting variant)."""
    xbar = np.asarray(xbar, dtype=np.float64)
    C, H, W = xbar.shape
    P = patch
    Wc = W - P + 1
    num = np.zeros((C, H, W))
    cnt = np.zeros((H, W))
    flat_idx = np.asarray(idx).reshape(-1)
    est = np.asarray(Xhat, dtype=np.float64).reshape(flat_idx.shape[0], C, P, P)
    K = np.asarray(idx).shape[1]
    w = np.ones(flat_idx.shape[0]) if weights is None else np.repeat(
        np.asarray(weights, dtype=np.float64), K)
    r0, c0 = np.divmod(flat_idx, Wc)
    for dy in range(P):
        for dx in range(P):
            rr = r0 + dy
            cc = c0 + dx
            np.add.at(cnt, (rr, cc), w)
            for ch in range(C):
                np.add.at(num[ch], (rr, cc), w * est[:, ch, dy, dx])
    out = xbar.copy()
    m = cnt > 0
    out[:, m] = num[:, m] / cnt[m][None]
    return out, cnt


def coverage_count(H, W, patch, idx):
    """Number of member patches covering each pixel (brute force)."""
    P = patch
    Wc = W - P + 1
    cnt = np.zeros((H, W), dtype=np.int64)
    for t in np.asarray(idx).reshape(-1):
        r, c = divmod(int(t), Wc)
        cnt[r:r + P, c:c + P] += 1
    return cnt
