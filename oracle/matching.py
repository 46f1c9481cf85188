"""Global patch matching and top-K grouping (oracle).

Definition followed: the group index set of exemplar i collects the patches
closest to it in squared L2 distance (eq. 1, with the KNN form of block
matching), searched over the whole image (global matching: every valid
stride-1 position of the (H-P+1) x (W-P+1) grid, the heat-map size given after
eq. 8).  Readings: the score is the squared L2 distance on the raw patch
values (the paper's own conventional criterion, made global), groups are the
K nearest patches, and ties are broken by the lowest top-left index.

So for key g the group is the first K entries of all candidates j sorted by
(d(g, j), j) ascending, d(g, j) = sum over (c, dy, dx) of
(x[c, r_g+dy, c_g+dx] - x[c, r_j+dy, c_j+dx])^2.  A patch vector is ordered
d = (c*P + dy)*P + dx.

For speed the oracle shortlists with the FP64 GEMM form
||k||^2 - 2<k, p> + ||p||^2 and a certified FP64 error bound, then recomputes
the direct sum for every shortlisted candidate; the selection is made on the
direct sums only.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

_U64 = 2.0 ** -53


def patch_matrix(x, patch):
    """All stride-1 patches of ``x`` ``[C][H][W]`` as rows ``[N_cand][D]``."""
    x = np.asarray(x, dtype=np.float64)
    C, H, W = x.shape
    P = patch
    win = sliding_window_view(x, (P, P), axis=(1, 2))      # [C][Hc][Wc][P][P]
    Hc, Wc = H - P + 1, W - P + 1
    return np.ascontiguousarray(win.transpose(1, 2, 0, 3, 4).reshape(Hc * Wc, C * P * P))


def direct_distances(x, patch, key, cands):
    """d(key, j) for each j in ``cands`` by the direct sum (FP64)."""
    pm = patch_matrix(x, patch)
    k = pm[key]
    diff = pm[np.asarray(cands)] - k[None, :]
    return np.sum(diff * diff, axis=1)


def topk_exact(x, patch, keys, K, chunk=256, return_boundary=False):
    """Exact K-nearest-patch groups.

    Returns ``idx`` int64 ``[N][K]`` and ``dist`` float64 ``[N][K]`` (sorted by
    (d, j)); with ``return_boundary`` also the direct distance of the (K+1)-th
    candidate in that order (``inf`` if there is none), used to measure how
    close a group boundary is to a tie.
    """
    pm = patch_matrix(x, patch)
    n_cand, D = pm.shape
    keys = np.asarray(keys, dtype=np.int64)
    N = keys.shape[0]
    if not (1 <= K <= n_cand):
        raise ValueError("K out of range")
    pn = np.einsum("ij,ij->i", pm, pm)
    pr = np.sqrt(pn)
    idx = np.empty((N, K), dtype=np.int64)
    dist = np.empty((N, K), dtype=np.float64)
    nxt = np.full(N, np.inf)
    coef = 4.0 * (D + 4) * _U64
    Kx = min(K + 1, n_cand)
    for g0 in range(0, N, chunk):
        ks = pm[keys[g0:g0 + chunk]]
        kn = np.einsum("ij,ij->i", ks, ks)
        dt = kn[:, None] - 2.0 * (ks @ pm.T) + pn[None, :]
        eps = coef * (np.sqrt(kn)[:, None] + pr[None, :]) ** 2
        for a in range(ks.shape[0]):
            up = dt[a] + eps[a]
            T = np.partition(up, Kx - 1)[Kx - 1]
            short = np.nonzero(dt[a] - eps[a] <= T)[0]
            diff = pm[short] - ks[a][None, :]
            d = np.sum(diff * diff, axis=1)
            order = np.lexsort((short, d))
            idx[g0 + a] = short[order[:K]]
            dist[g0 + a] = d[order[:K]]
            if Kx > K:
                nxt[g0 + a] = d[order[K]]
    if return_boundary:
        return idx, dist, nxt
    return idx, dist


def distance_map(x, patch, key):
    """d(key, j) for every candidate j (FP64, ``[Hc*Wc]``) by the direct sum,
    accumulated one patch offset (c, dy, dx) at a time over shifted copies of
    the image: no patch matrix, no GEMM form, memory O(H*W).  Used to check
    single keys of full-size images."""
    x = np.asarray(x, dtype=np.float64)
    C, H, W = x.shape
    P = patch
    Hc, Wc = H - P + 1, W - P + 1
    r, c = divmod(int(key), Wc)
    d = np.zeros((Hc, Wc))
    for ch in range(C):
        for dy in range(P):
            for dx in range(P):
                diff = x[ch, dy:dy + Hc, dx:dx + Wc] - x[ch, r + dy, c + dx]
                d += diff * diff
    return d.reshape(-1)


def topk_one(x, patch, key, K):
    """Exact group of one key from ``distance_map``: (idx [K], dist [K], the
    (K+1)-th distance or inf)."""
    d = distance_map(x, patch, key)
    order = np.lexsort((np.arange(d.size), d))[:K + 1]
    nxt = d[order[K]] if order.size > K else np.inf
    return order[:K], d[order[:K]], nxt


def topk_bruteforce(x, patch, keys, K):
    """Direct-sum reference over every candidate (no shortlist), FP64."""
    pm = patch_matrix(x, patch)
    keys = np.asarray(keys, dtype=np.int64)
    idx = np.empty((keys.shape[0], K), dtype=np.int64)
    dist = np.empty((keys.shape[0], K))
    j = np.arange(pm.shape[0])
    for a, g in enumerate(keys):
        diff = pm - pm[g][None, :]
        d = np.sum(diff * diff, axis=1)
        order = np.lexsort((j, d))[:K]
        idx[a] = order
        dist[a] = d[order]
    return idx, dist


def window_topk(x, patch, keys, K, radius):
    """Block matching in a local window (eq. 1 with KNN grouping, the
    vanilla BM the paper compares against): for the key at (r_g, c_g) the
    candidates are the positions (r, c) of the top-left grid with
    |r - r_g| <= radius and |c - c_g| <= radius; the group is their first K
    by (d, j) ascending, d the direct squared distance (FP64).  Returns
    ``idx`` int64 ``[N][K]`` and ``dist`` ``[N][K]``."""
    x = np.asarray(x, dtype=np.float64)
    C, H, W = x.shape
    P = patch
    Hc, Wc = H - P + 1, W - P + 1
    pm = patch_matrix(x, P)
    keys = np.asarray(keys, dtype=np.int64)
    idx = np.empty((keys.shape[0], K), dtype=np.int64)
    dist = np.empty((keys.shape[0], K))
    for a, g in enumerate(keys):
        rg, cg = divmod(int(g), Wc)
        rr = np.arange(max(rg - radius, 0), min(rg + radius, Hc - 1) + 1)
        cc = np.arange(max(cg - radius, 0), min(cg + radius, Wc - 1) + 1)
        cand = (rr[:, None] * Wc + cc[None, :]).reshape(-1)
        if cand.size < K:
            raise ValueError("window holds fewer than K candidates")
        diff = pm[cand] - pm[g][None, :]
        d = np.sum(diff * diff, axis=1)
        order = np.lexsort((cand, d))[:K]
        idx[a] = cand[order]
        dist[a] = d[order]
    return idx, dist
