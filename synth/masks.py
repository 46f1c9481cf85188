"""Seeded binary sensing masks (the random part of each forward operator)."""
import numpy as np


def cacti_masks(frames, H, W, seed):
    """Bernoulli(0.5) coded-aperture masks, uint8 ``[frames][H][W]`` in {0,1}."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=(frames, H, W)) < 0.5).astype(np.uint8)


def mri_line_mask(H, seed, fraction=0.25, centre_lines=16):
    """Random Cartesian k-space line mask, uint8 ``[H]``: ``round(fraction*H)``
    phase-encode rows are kept, always including the ``centre_lines`` rows of
    lowest |k_y| in unshifted FFT order (rows 0..c/2-1 and H-c/2..H-1); the
    rest are drawn uniformly without replacement from the remaining rows."""
    rng = np.random.default_rng(seed)
    n_lines = int(round(fraction * H))
    half = min(centre_lines, n_lines) // 2
    centre = list(range(half)) + list(range(H - half, H))
    others = np.array([r for r in range(H) if r not in set(centre)], dtype=np.int64)
    extra = rng.choice(others, size=max(0, n_lines - len(centre)), replace=False)
    m = np.zeros(H, dtype=np.uint8)
    m[centre] = 1
    m[extra] = 1
    return m
