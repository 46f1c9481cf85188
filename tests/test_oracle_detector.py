"""Pins for the oracle key detector: pure-Python integer brute force and
geometric special cases (corner exemplars, Method section and Fig. 1a)."""
import numpy as np

import synth
from oracle import detector as det


def _clamp(v, lo, hi):
    return lo if v < lo else hi if v > hi else v


def _bf_r25(q):
    """Loop-by-loop Harris R25 with replicate borders (independent of the
    vectorised oracle)."""
    H, W = len(q), len(q[0])
    def Q(r, c):
        return q[_clamp(r, 0, H - 1)][_clamp(c, 0, W - 1)]
    gx = [[0] * W for _ in range(H)]
    gy = [[0] * W for _ in range(H)]
    for r in range(H):
        for c in range(W):
            sx = sy = 0
            for dr, dc, w in [(-1, -1, 1), (0, -1, 2), (1, -1, 1)]:
                sx -= w * Q(r + dr, c + dc)
                sx += w * Q(r + dr, c - dc)
            for dr, dc, w in [(-1, -1, 1), (-1, 0, 2), (-1, 1, 1)]:
                sy -= w * Q(r + dr, c + dc)
                sy += w * Q(r - dr, c + dc)
            gx[r][c] = sx
            gy[r][c] = sy
    w5 = [1, 4, 6, 4, 1]
    R = [[0] * W for _ in range(H)]
    for r in range(H):
        for c in range(W):
            a = b = d = 0
            for i in range(5):
                for j in range(5):
                    rr = _clamp(r + i - 2, 0, H - 1)
                    cc = _clamp(c + j - 2, 0, W - 1)
                    w = w5[i] * w5[j]
                    a += w * gx[rr][cc] * gx[rr][cc]
                    b += w * gy[rr][cc] * gy[rr][cc]
                    d += w * gx[rr][cc] * gy[rr][cc]
            R[r][c] = 25 * (a * b - d * d) - (a + b) ** 2
    return R


def _bf_keys(q, P, N):
    H, W = len(q), len(q[0])
    R = _bf_r25(q)
    o = (P - 1) // 2
    Hc, Wc = H - P + 1, W - P + 1
    surv = []
    for r in range(H):
        for c in range(W):
            if R[r][c] <= 0:
                continue
            ok = True
            for dr in (-1, 0, 1):
                for dc in (-1, 0, 1):
                    rr, cc = r + dr, c + dc
                    if (dr, dc) == (0, 0) or not (0 <= rr < H and 0 <= cc < W):
                        continue
                    # neighbour beats (r,c) if larger score, or equal and lower index
                    if R[rr][cc] > R[r][c] or (R[rr][cc] == R[r][c] and rr * W + cc < r * W + c):
                        ok = False
            if ok and o <= r < o + Hc and o <= c < o + Wc:
                surv.append((-R[r][c], r * W + c, (r - o) * Wc + (c - o)))
    surv.sort()
    chosen = set(t for _, _, t in surv[:N])
    s = 1
    while s * s * N < Hc * Wc:
        s += 1
    for step in (s, 1):
        for gr in range(0, Hc, step):
            for gc in range(0, Wc, step):
                if len(chosen) < N:
                    chosen.add(gr * Wc + gc)
    return sorted(chosen), R


def test_r25_and_keys_match_bruteforce():
    for seed in range(4):
        rng = np.random.default_rng(seed)
        H, W = 11 + seed, 13
        q = rng.integers(0, 256, size=(H, W))
        if seed == 3:
            q = (q > 128).astype(np.int64) * 255  # many exact ties
        keys_bf, R_bf = _bf_keys(q.tolist(), 4, 7)
        np.testing.assert_array_equal(det.harris_r25(q), np.array(R_bf))
        x = (q.astype(np.float32) / np.float32(255))[None]
        keys = det.detect_keys(x, 4, 7)
        assert keys.tolist() == keys_bf


def test_quantiser_real():
    x = np.array([[[-0.3, 0.0, 1.0, 2.0, 0.5]]], dtype=np.float32)
    q = det.quantise_real(x)
    # 255*0.5 = 127.5 exactly in FP32 -> round half to even = 128
    assert q.tolist() == [[0, 0, 255, 255, 128]]
    # channel average with round-half-up integer division
    x2 = np.stack([np.full((1, 3), 1 / 255, np.float32), np.full((1, 3), 2 / 255, np.float32)])
    assert det.quantise_real(x2).tolist() == [[2, 2, 2]]   # (1 + 2 + 1) // 2


def test_constant_image_gives_uniform_fill():
    x = np.full((2, 20, 24), 0.4, dtype=np.float32)
    P, N = 5, 9
    keys = det.detect_keys(x, P, N)
    Hc, Wc = 16, 20
    s = det.fill_step(Hc * Wc, N)
    assert s * s * N >= Hc * Wc and (s - 1) ** 2 * N < Hc * Wc
    grid = [gr * Wc + gc for gr in range(0, Hc, s) for gc in range(0, Wc, s)][:N]
    assert keys.tolist() == sorted(grid)


def test_square_corners():
    H = W = 40
    q = np.zeros((H, W), dtype=np.float32)
    q[10:30, 12:28] = 1.0
    keys = det.detect_keys(q[None], 3, 4)
    o = 1
    Wc = W - 2
    centres = [((k // Wc) + o, (k % Wc) + o) for k in keys]
    corners = [(10, 12), (10, 27), (29, 12), (29, 27)]
    for (cr, cc) in corners:
        assert min(abs(cr - r) + abs(cc - c) for r, c in centres) <= 2


def test_straight_edge_is_not_a_corner():
    H, W = 24, 24
    q = np.zeros((H, W), dtype=np.int64)
    q[:, 12:] = 255
    R = det.harris_r25(q)
    assert (R <= 0).all()


def test_zero_complex_image_has_no_corners():
    z = np.zeros((2, 16, 16), dtype=np.float32)
    assert det.quantise_complex(z[0], z[1]) is None
    keys = det.detect_keys(z, 4, 5, is_complex=True)
    assert len(keys) == 5


def test_keys_on_workload_are_distinct_sorted_in_range():
    wl = synth.WORKLOADS["cacti_128"]
    x = synth.make_instance(wl)["x_true"]
    keys = det.detect_keys(x, wl.patch, wl.n_keys)
    assert len(keys) == wl.n_keys
    assert np.all(np.diff(keys) > 0)
    assert keys[0] >= 0 and keys[-1] < wl.n_cand


def test_quantise_complex_by_hand():
    """Hand-worked values of the complex quantiser q = rint(255 (m / max m)),
    m = re^2 + im^2 (squared magnitude, not magnitude), every FP32 step exact
    here except the one sum that lands on a half-way point.

    Pixel by pixel (max m = 1, so 1/max = 1):
      (1, 0)            m = 1        255 m = 255
      (0.5, b)          m = 0.25 + b^2 rounds to t with 255 t = 126.5 exactly
                        -> round half to even gives 126 (half-up would give 127)
      (0, 0.5)          m = 0.25     63.75    -> 64
      (0.5, 0.5)        m = 0.5      127.5    -> 128 (half to even)
      (0.25, 0.25)      m = 0.125    31.875   -> 32
      (0.75, 0)         m = 0.5625   143.4375 -> 143
      (0, 0), (0, 0)    0
      (0.125, 0)        m = 1/64     3.984375 -> 4
    The magnitude |z| would give 180 for (0.5, 0.5); a missing 1/max scale
    fails on the same image scaled by 2 (max m = 4, same q); floor instead
    of rint gives 63 for (0, 0.5)."""
    from fractions import Fraction
    f32 = np.float32
    b = f32(0.4960629343986511)
    re = np.array([[1, 0.5, 0], [0.5, 0.25, 0.75], [0, 0, 0.125]], dtype=f32)
    im = np.array([[0, b, 0.5], [0.5, 0.25, 0], [0, 0, 0]], dtype=f32)
    t = f32(0.25) + b * b
    assert Fraction(float(f32(255) * t)) == Fraction(253, 2)     # the half-way case
    expect = [[255, 126, 64], [128, 32, 143], [0, 0, 4]]
    assert det.quantise_complex(re, im).tolist() == expect
    # scaling by two multiplies m and max m by four: q is unchanged
    assert det.quantise_complex(2 * re, 2 * im).tolist() == expect
    # a non-power-of-two maximum: s = fl(1/max) is applied as a product
    # (255/9 = 28.33 is far from a rounding boundary: 28)
    re3 = np.array([[3, 1, 0]], dtype=f32)          # m = 9, 1, 0
    im3 = np.zeros_like(re3)
    assert det.quantise_complex(re3, im3).tolist() == [[255, 28, 0]]


def test_uniform_exemplar_grid():
    from oracle import detector as dt
    # rows {0, 3}, columns {0, 3, 6} of a 5 x 7 grid
    np.testing.assert_array_equal(dt.uniform_keys(5, 7, 3), [0, 3, 6, 21, 24, 27])
    np.testing.assert_array_equal(dt.uniform_keys(4, 4, 1), np.arange(16))
    assert dt.uniform_keys(10, 10, 20).tolist() == [0]


def test_corner_uniform_exemplars_concatenate_the_coarse_grid():
    from oracle import detector as dt
    x = synth.workloads.random_image(2, 30, 34, seed=3)
    P, N, s = 5, 12, 2
    k = dt.exemplar_keys(x, P, N, "corner_uniform", s)
    corners = dt.detect_keys(x, P, N)
    grid = dt.uniform_keys(30 - P + 1, 34 - P + 1, 3 * s)
    np.testing.assert_array_equal(k, np.concatenate([corners, grid]))
    np.testing.assert_array_equal(dt.exemplar_keys(x, P, N, "uniform", s),
                                  dt.uniform_keys(26, 30, s))
