"""One GLR prior step (oracle): detect keys, match globally, group top-K,
shrink each group by WNNM, aggregate (Method section, eq. 1, eq. 8 sizes,
the low-rank objective and WNNM)."""
import numpy as np

from .detector import exemplar_keys
from .matching import topk_exact, window_topk
from .lowrank import shrink_groups, group_weights
from .aggregate import aggregate


def prior_step(x, patch, n_keys, K, sigma, c, eps, is_complex=False, keys=None,
               exemplars="corner", step=4, search="global", radius=20, score="l2",
               agg_weights="uniform", inner=1, delta=0.1, lam=0.54, lowrank="stacked"):
    """Apply the prior to iterate ``x`` (planar real ``[C'][H][W]``; complex
    data as ``[2][H][W]`` = (Re, Im)).  ``keys`` may be supplied to bypass the
    detector.  ``exemplars`` ("corner", "uniform", "corner_uniform", with the
    uniform interval ``step``) and ``search`` ("global", or "window" of half
    width ``radius``: the block-matching baselines) select the variant;
    ``score`` "edge" groups by the edge-map heat map of eq. 6-8 instead of
    the squared distance (``dist`` then holds the heat values);
    ``agg_weights`` "rank" weighs each group's estimates by 1 / (its kept
    WNNM rank) in the aggregation (``weights`` then holds them).  ``inner``
    > 1 shrinks the same groups again with WNNM's iterative regularisation
    (``inner_iterations``).  ``lowrank`` "complex" (complex data only)
    shrinks each group as one complex matrix (``wnnm_group_complex``) instead
    of the real-stacked [Re; Im] group.
    Returns a dict with keys, idx, dist, Xhat, sv, weights, x_out, count."""
    x = np.asarray(x, dtype=np.float64)
    if keys is None:
        keys = exemplar_keys(x, patch, n_keys, exemplars, step, is_complex=is_complex)
    if score == "edge":
        from .edges import topk_edge
        idx, dist = topk_edge(x, patch, keys, K, is_complex=is_complex)
    elif search == "global":
        idx, dist = topk_exact(x, patch, keys, K)
    elif search == "window":
        idx, dist = window_topk(x, patch, keys, K, radius)
    else:
        raise ValueError(search)
    if agg_weights not in ("uniform", "rank"):
        raise ValueError(agg_weights)
    if lowrank not in ("stacked", "complex") or (lowrank == "complex" and not is_complex):
        raise ValueError(lowrank)
    cplx = lowrank == "complex"

    def shrink_and_aggregate(y, sig):
        Xh, s = shrink_groups(y, patch, idx, sig, c, eps, complex_groups=cplx)
        w = group_weights(s, K, sig, c, eps) if agg_weights == "rank" else None
        xo, n = aggregate(y, patch, idx, Xh, weights=w)
        return Xh, s, w, xo, n

    Xhat, sv, wts, x_out, cnt = shrink_and_aggregate(x, sigma)
    sigmas = [sigma]
    if inner > 1:
        x_out, sigmas, (Xhat, sv, wts, cnt) = inner_iterations(
            x, x_out, sigma, inner, delta, lam, shrink_and_aggregate)
    return {"keys": keys, "idx": idx, "dist": dist, "Xhat": Xhat, "sv": sv,
            "weights": wts, "x_out": x_out, "count": cnt, "sigmas": sigmas}


def inner_iterations(xbar, x1, sigma, J, delta, lam, step):
    """Iterative regularisation of WNNM [Gu et al. 2014] inside one prior
    step (a variant; the paper runs the low-rank step once per iteration of
    the outer solver).  Reading: the groups of the step's one matching stay
    fixed; with y^(1) = xbar and x^(1) the first shrinkage,
        y^(k) = x^(k-1) + delta (xbar - y^(k-1)),
        sigma_k = lam sqrt(max(sigma^2 - mean((xbar - y^(k))^2), 0)),
        x^(k) = step(y^(k), sigma_k)      (shrink and aggregate),
    for k = 2..J.  ``step(y, sig)`` returns (Xhat, sv, weights, x, count).
    Returns x^(J), the noise levels [sigma_1..sigma_J] and the last step's
    (Xhat, sv, weights, count)."""
    xbar = np.asarray(xbar, dtype=np.float64)
    y_prev, x_prev = xbar, x1
    sigmas = [float(sigma)]
    last = None
    for _ in range(2, J + 1):
        y = x_prev + delta * (xbar - y_prev)
        sk = lam * np.sqrt(max(sigma * sigma - np.mean((xbar - y) ** 2), 0.0))
        Xh, s, w, x_prev, n = step(y, sk)
        last = (Xh, s, w, n)
        sigmas.append(float(sk))
        y_prev = y
    return x_prev, sigmas, last


def to_planar(z):
    """complex ``[H][W]`` -> planar ``[2][H][W]`` (Re, Im)."""
    return np.stack([np.real(z), np.imag(z)]).astype(np.float64)


def from_planar(p):
    """planar ``[2][H][W]`` -> complex ``[H][W]``."""
    return p[0] + 1j * p[1]
