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
               agg_weights="uniform"):
    """Apply the prior to iterate ``x`` (planar real ``[C'][H][W]``; complex
    data as ``[2][H][W]`` = (Re, Im)).  ``keys`` may be supplied to bypass the
    detector.  ``exemplars`` ("corner", "uniform", "corner_uniform", with the
    uniform interval ``step``) and ``search`` ("global", or "window" of half
    width ``radius``: the block-matching baselines) select the variant;
    ``score`` "edge" groups by the edge-map heat map of eq. 6-8 instead of
    the squared distance (``dist`` then holds the heat values);
    ``agg_weights`` "rank" weighs each group's estimates by 1 / (its kept
    WNNM rank) in the aggregation (``weights`` then holds them).
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
    Xhat, sv = shrink_groups(x, patch, idx, sigma, c, eps)
    wts = None
    if agg_weights == "rank":
        wts = group_weights(sv, K, sigma, c, eps)
    elif agg_weights != "uniform":
        raise ValueError(agg_weights)
    x_out, cnt = aggregate(x, patch, idx, Xhat, weights=wts)
    return {"keys": keys, "idx": idx, "dist": dist, "Xhat": Xhat, "sv": sv,
            "weights": wts, "x_out": x_out, "count": cnt}


def to_planar(z):
    """complex ``[H][W]`` -> planar ``[2][H][W]`` (Re, Im)."""
    return np.stack([np.real(z), np.imag(z)]).astype(np.float64)


def from_planar(p):
    """planar ``[2][H][W]`` -> complex ``[H][W]``."""
    return p[0] + 1j * p[1]
