"""Seeded synthetic scenes shaped like the paper's three modalities.

The paper's datasets (CACTI benchmark videos, MRI scans, multispectral cubes)
are not available; these generators stand in for them with the same shapes,
value ranges and structure (piecewise-smooth regions, moving textured objects,
smooth spectra).  All use ``numpy.random.default_rng(seed)``.
"""
import numpy as np
from scipy import ndimage


def _paint_object(img, rr, cc, cy, cx, hy, hx, is_ellipse, base, grat):
    """Paint one textured object (ellipse or rectangle) on ``img`` in place."""
    dy = rr - cy
    dx = cc - cx
    if is_ellipse:
        inside = (dy / hy) ** 2 + (dx / hx) ** 2 <= 1.0
    else:
        inside = (np.abs(dy) <= hy) & (np.abs(dx) <= hx)
    fr, ang, ph = grat
    # grating attached to the object (coordinates relative to its centre)
    u = np.cos(ang) * dx + np.sin(ang) * dy
    tex = base + 0.1 * np.sin(2.0 * np.pi * fr * u + ph)
    img[inside] = tex[inside]


def cacti_video(frames, H, W, seed):
    """Video of ``frames`` frames: smooth background plus six moving textured
    ellipses/rectangles (1-2 px/frame), clipped to [0, 1].  Returns float32
    array ``[frames][H][W]``."""
    rng = np.random.default_rng(seed)
    f1, f2 = rng.uniform(1.0, 4.0, size=2)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    rr, cc = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    background = 0.15 + 0.05 * np.sin(2.0 * np.pi * (f1 * rr + f2 * cc) / H + phi)
    objs = []
    for _ in range(6):
        is_ellipse = bool(rng.uniform() < 0.5)
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        hy = rng.uniform(H / 16.0, H / 5.0)
        hx = rng.uniform(W / 16.0, W / 5.0)
        base = rng.uniform(0.3, 0.9)
        grat = (rng.uniform(0.05, 0.25), rng.uniform(0.0, np.pi), rng.uniform(0.0, 2 * np.pi))
        vy = int(rng.choice([-2, -1, 1, 2]))
        vx = int(rng.choice([-2, -1, 1, 2]))
        objs.append((is_ellipse, cy, cx, hy, hx, base, grat, vy, vx))
    out = np.empty((frames, H, W), dtype=np.float64)
    for t in range(frames):
        img = background.copy()
        for (is_ellipse, cy, cx, hy, hx, base, grat, vy, vx) in objs:
            _paint_object(img, rr, cc, cy + t * vy, cx + t * vx, hy, hx, is_ellipse, base, grat)
        out[t] = img
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def mri_phantom(H, W, seed):
    """Complex piecewise-smooth phantom: ten additive random ellipses
    (magnitude normalised to max 1) times a smooth random phase.  Returns
    complex64 ``[H][W]``."""
    rng = np.random.default_rng(seed)
    rr, cc = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    mag = np.zeros((H, W))
    for _ in range(10):
        rad = 0.8 * np.sqrt(rng.uniform()) * (min(H, W) / 2.0)
        th = rng.uniform(0.0, 2.0 * np.pi)
        cy = H / 2.0 + rad * np.sin(th)
        cx = W / 2.0 + rad * np.cos(th)
        a = rng.uniform(0.05, 0.4) * H
        b = rng.uniform(0.05, 0.4) * W
        ang = rng.uniform(0.0, np.pi)
        amp = rng.uniform(0.1, 0.5)
        dy = rr - cy
        dx = cc - cx
        u = np.cos(ang) * dx + np.sin(ang) * dy
        v = -np.sin(ang) * dx + np.cos(ang) * dy
        mag += amp * (((u / b) ** 2 + (v / a) ** 2) <= 1.0)
    if mag.max() > 0:
        mag /= mag.max()
    phase = np.zeros((H, W))
    for _ in range(3):
        u, v = rng.uniform(0.0, 1.5, size=2)
        beta = rng.uniform(0.0, np.pi / 3.0)
        th = rng.uniform(0.0, 2.0 * np.pi)
        phase += beta * np.cos(2.0 * np.pi * (u * rr + v * cc) / H + th)
    return (mag * np.exp(1j * phase)).astype(np.complex64)


def msfa_cube(bands, H, W, seed, regions=50):
    """Multispectral cube ``[bands][H][W]``: ``regions`` Voronoi cells, each
    with a smooth spectrum (sum of two Gaussians over the band index, max at
    most 0.9), modulated by a 2 % smoothed Gaussian texture, clipped to [0, 1].
    Returns float32."""
    rng = np.random.default_rng(seed)
    seeds = np.stack([rng.uniform(0, H, regions), rng.uniform(0, W, regions)], axis=1)
    b = np.arange(bands, dtype=np.float64)
    spectra = np.zeros((regions, bands))
    for k in range(regions):
        s = np.zeros(bands)
        for _ in range(2):
            cen = rng.uniform(0.0, bands - 1.0)
            wid = rng.uniform(2.0, 6.0)
            amp = rng.uniform(0.2, 0.8)
            s += amp * np.exp(-0.5 * ((b - cen) / wid) ** 2)
        m = s.max()
        if m > 0.9:
            s *= 0.9 / m
        spectra[k] = s
    tex = ndimage.gaussian_filter(rng.standard_normal((H, W)), sigma=1.5, mode="reflect")
    tex *= 0.02 / tex.std()
    label = np.empty((H, W), dtype=np.int64)
    rows = np.arange(H, dtype=np.float64)
    cols = np.arange(W, dtype=np.float64)
    for r0 in range(0, H, 64):
        rr, cc = np.meshgrid(rows[r0:r0 + 64], cols, indexing="ij")
        d2 = (rr[..., None] - seeds[:, 0]) ** 2 + (cc[..., None] - seeds[:, 1]) ** 2
        label[r0:r0 + 64] = np.argmin(d2, axis=-1)
    cube = spectra[label].transpose(2, 0, 1) * (1.0 + tex)[None]
    return np.clip(cube, 0.0, 1.0).astype(np.float32)
