"""Key-patch (exemplar) detection: corner points instead of a uniform grid.

The paper picks exemplar patches centred on corner points of an edge map
(Method section and Fig. 1a) without naming the detector.  The reading taken
here is an integer-exact Harris detector on a quantised detection image:

1. quantise the iterate to u8 (IEEE FP32 steps, emulated with np.float32):
   real data: q_c = clamp(rint(255 * x_c), 0, 255), q = floor((sum_c q_c + C//2) / C);
   complex data: m = re*re + im*im, s = 1/max(m), q = clamp(rint(255*(m*s)), 0, 255);
2. Sobel gradients gx (along columns), gy (along rows), replicate borders;
3. structure tensor: 5x5 binomial [1 4 6 4 1] (x) [1 4 6 4 1] sums of
   gx^2, gy^2, gx*gy, replicate borders;
4. Harris score times 25 (kappa = 1/25): R25 = 25(Sxx Syy - Sxy^2) - (Sxx + Syy)^2;
5. 3x3 non-maximum suppression under the order (R25 desc, pixel index asc),
   neighbours taken inside the image; survivors need R25 > 0;
6. the first N survivors in that order whose centre lies in the key domain
   r in [o, o+H-P], c in [o, o+W-P] (o = (P-1)//2); key = top-left (r-o, c-o);
7. if fewer than N corners exist, a uniform raster fill with step
   s = min{s >= 1 : s*s*N >= N_cand}, skipping chosen positions, then a
   step-1 raster if still short.

Keys are returned as ascending linear indices into the (H-P+1) x (W-P+1)
top-left grid.  Every step after the quantiser is integer arithmetic.
"""
import numpy as np

_F255 = np.float32(255.0)
_W5 = np.array([1, 4, 6, 4, 1], dtype=np.int64)


def quantise_real(x32):
    """u8 detection image of a real ``[C][H][W]`` float32 iterate (step 1)."""
    x32 = np.asarray(x32, dtype=np.float32)
    C = x32.shape[0]
    q = np.clip(np.rint(_F255 * x32), np.float32(0), np.float32(255)).astype(np.int64)
    return (q.sum(axis=0) + C // 2) // C


def quantise_complex(re32, im32):
    """u8 detection image of a complex iterate from its squared magnitude.

    Returns ``None`` when the image is identically zero (no corners)."""
    re32 = np.asarray(re32, dtype=np.float32)
    im32 = np.asarray(im32, dtype=np.float32)
    m = re32 * re32 + im32 * im32
    mx = m.max()
    if not (mx > 0):
        return None
    s = np.float32(1.0) / mx
    return np.clip(np.rint(_F255 * (m * s)), np.float32(0), np.float32(255)).astype(np.int64)


def sobel(q):
    """Integer Sobel gradients with replicate borders: (gx, gy)."""
    H, W = q.shape
    p = np.pad(q, 1, mode="edge")
    def at(dr, dc):
        return p[1 + dr:1 + dr + H, 1 + dc:1 + dc + W]
    gx = (at(-1, 1) + 2 * at(0, 1) + at(1, 1)) - (at(-1, -1) + 2 * at(0, -1) + at(1, -1))
    gy = (at(1, -1) + 2 * at(1, 0) + at(1, 1)) - (at(-1, -1) + 2 * at(-1, 0) + at(-1, 1))
    return gx, gy


def binomial5(img):
    """5x5 binomial window sum with replicate borders (integer)."""
    H, W = img.shape
    p = np.pad(img, 2, mode="edge")
    out = np.zeros((H, W), dtype=np.int64)
    for a in range(5):
        for b in range(5):
            out += _W5[a] * _W5[b] * p[a:a + H, b:b + W]
    return out


def harris_r25(q):
    """R25 = 25*det(S) - tr(S)^2 of the binomial structure tensor (int64)."""
    gx, gy = sobel(q)
    sxx = binomial5(gx * gx)
    syy = binomial5(gy * gy)
    sxy = binomial5(gx * gy)
    return 25 * (sxx * syy - sxy * sxy) - (sxx + syy) ** 2


def nms_survivors(R):
    """Boolean map of 3x3 maxima under (R desc, index asc) with R > 0."""
    H, W = R.shape
    lo = np.iinfo(np.int64).min
    p = np.full((H + 2, W + 2), lo, dtype=np.int64)
    p[1:-1, 1:-1] = R
    keep = R > 0
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if dr == 0 and dc == 0:
                continue
            nb = p[1 + dr:1 + dr + H, 1 + dc:1 + dc + W]
            earlier = dr < 0 or (dr == 0 and dc < 0)
            # an earlier (lower-index) neighbour wins ties
            keep &= (R > nb) if earlier else (R >= nb)
    return keep


def fill_step(n_cand, n_keys):
    """Smallest s >= 1 with s*s*n_keys >= n_cand."""
    s = 1
    while s * s * n_keys < n_cand:
        s += 1
    return s


def detect_keys(x, patch, n_keys, is_complex=False):
    """Key top-left indices (ascending, int64 ``[n_keys]``) for iterate ``x``.

    ``x``: real ``[C][H][W]`` or, with ``is_complex``, planar ``[2][H][W]``
    (Re, Im).  Values are taken as float32 (the detection precision)."""
    x32 = np.asarray(x, dtype=np.float32)
    _, H, W = x32.shape
    P = patch
    Hc, Wc = H - P + 1, W - P + 1
    n_cand = Hc * Wc
    if not (1 <= n_keys <= n_cand):
        raise ValueError("n_keys out of range")
    o = (P - 1) // 2
    q = quantise_complex(x32[0], x32[1]) if is_complex else quantise_real(x32)
    chosen = np.zeros(n_cand, dtype=bool)
    if q is not None:
        R = harris_r25(q)
        surv = nms_survivors(R)
        dom = np.zeros((H, W), dtype=bool)
        dom[o:o + Hc, o:o + Wc] = True
        rr, cc = np.nonzero(surv & dom)           # row-major order = index order
        score = R[rr, cc]
        order = np.lexsort((rr * W + cc, -score))  # (R25 desc, index asc)
        sel = order[:n_keys]
        chosen[(rr[sel] - o) * Wc + (cc[sel] - o)] = True
    need = n_keys - int(chosen.sum())
    if need > 0:
        s = fill_step(n_cand, n_keys)
        for step in (s, 1):
            for gr in range(0, Hc, step):
                for gc in range(0, Wc, step):
                    if need == 0:
                        break
                    t = gr * Wc + gc
                    if not chosen[t]:
                        chosen[t] = True
                        need -= 1
            if need == 0:
                break
    return np.nonzero(chosen)[0].astype(np.int64)


def uniform_keys(Hc, Wc, step):
    """Exemplars of classic block matching: a uniform grid of top-left
    positions (r, c) = (step a, step b) with r < Hc, c < Wc (the paper's
    "traditional uniform selection", Method section), ascending index
    r*Wc + c."""
    rr = np.arange(0, Hc, step, dtype=np.int64)
    cc = np.arange(0, Wc, step, dtype=np.int64)
    return (rr[:, None] * Wc + cc[None, :]).reshape(-1)


def exemplar_keys(x, patch, n_keys, mode, step, is_complex=False):
    """Exemplar keys for one prior step.

    mode "corner": the N corner keys of ``detect_keys``; "uniform": the
    uniform grid of ``step``; "corner_uniform": the corner keys followed by a
    uniform grid whose interval is three times ``step`` (the corner-based
    block matching of the CACTI experiment, Results section, which adds a
    modest number of uniformly selected exemplars at three times the vanilla
    interval).  A grid position that is also a corner is kept twice."""
    _, H, W = np.asarray(x).shape
    Hc, Wc = H - patch + 1, W - patch + 1
    if mode == "corner":
        return detect_keys(x, patch, n_keys, is_complex=is_complex)
    if mode == "uniform":
        return uniform_keys(Hc, Wc, step)
    if mode == "corner_uniform":
        return np.concatenate([detect_keys(x, patch, n_keys, is_complex=is_complex),
                               uniform_keys(Hc, Wc, 3 * step)])
    raise ValueError(mode)
