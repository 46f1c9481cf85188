"""Pins for the oracle's global matching and top-K grouping: exact rational
brute force, planted duplicates, invariances (eq. 1 / KNN grouping made
global over the stride-1 candidate grid of eq. 8)."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import matching as mt


def _bf_exact(x, P, keys, K):
    """Pure-Python exact arithmetic: d as a Fraction, order (d, j)."""
    C, H, W = x.shape
    Hc, Wc = H - P + 1, W - P + 1
    xf = [[[Fraction(float(x[c, r, q])) for q in range(W)] for r in range(H)] for c in range(C)]
    out = []
    for g in keys:
        gr, gc = divmod(int(g), Wc)
        ds = []
        for j in range(Hc * Wc):
            jr, jc = divmod(j, Wc)
            d = Fraction(0)
            for c in range(C):
                for dy in range(P):
                    for dx in range(P):
                        e = xf[c][gr + dy][gc + dx] - xf[c][jr + dy][jc + dx]
                        d += e * e
            ds.append((d, j))
        ds.sort()
        out.append([j for _, j in ds[:K]])
    return out


@pytest.mark.parametrize("kind", ["uniform", "dup", "smooth"])
def test_topk_equals_exact_rational_bruteforce(kind):
    x = synth.workloads.random_image(2, 12, 12, seed=5, kind=kind)
    P, K = 3, 5
    keys = [0, 17, 45, 99]
    idx, dist = mt.topk_exact(x, P, keys, K)
    assert idx.tolist() == _bf_exact(x, P, keys, K)


def test_planted_duplicates_lowest_index_first():
    x = np.random.default_rng(0).uniform(size=(1, 10, 10)).astype(np.float32)
    P = 3
    Wc = 8
    # copy the patch at top-left (5,5) to (0,0) and (2,6): three identical patches
    src = x[:, 5:8, 5:8].copy()
    x[:, 0:3, 0:3] = src
    x[:, 2:5, 6:9] = src
    key = 5 * Wc + 5
    idx, dist = mt.topk_exact(x, P, [key], 3)
    assert idx[0].tolist() == [0, 2 * Wc + 6, key]
    assert dist[0].tolist() == [0.0, 0.0, 0.0]


def test_self_distance_zero_and_first():
    x = synth.workloads.random_image(3, 20, 18, seed=2, kind="uniform")
    keys = [3, 50, 111]
    idx, dist = mt.topk_exact(x, 4, keys, 6)
    assert (dist[:, 0] == 0).all()
    assert idx[:, 0].tolist() == keys
    assert (np.diff(dist, axis=1) >= 0).all()


def test_constant_shift_and_key_permutation():
    x = synth.workloads.random_image(2, 24, 20, seed=3, kind="smooth")
    keys = np.array([7, 100, 222, 5, 301])
    idx, _ = mt.topk_exact(x, 5, keys, 8)
    # adding a dyadic constant is exact in FP64 for these values
    idx2, _ = mt.topk_exact(x.astype(np.float64) + 0.25, 5, keys, 8)
    np.testing.assert_array_equal(idx, idx2)
    perm = np.array([3, 1, 4, 0, 2])
    idx3, _ = mt.topk_exact(x, 5, keys[perm], 8)
    np.testing.assert_array_equal(idx3, idx[perm])


def test_shortlist_has_no_false_exclusions():
    # the certified shortlist + direct sums equals the direct sum over all candidates
    for seed, kind in [(1, "smooth"), (2, "dup"), (3, "uniform")]:
        x = synth.workloads.random_image(4, 30, 33, seed=seed, kind=kind)
        P, K = 4, 11
        keys = np.arange(0, 27 * 30, 37)
        a, da = mt.topk_exact(x, P, keys, K, chunk=7)
        b, db = mt.topk_bruteforce(x, P, keys, K)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(da, db)


def test_patch_vector_order():
    x = np.arange(2 * 5 * 6, dtype=np.float64).reshape(2, 5, 6)
    pm = mt.patch_matrix(x, 2)
    Wc = 5
    # row for top-left (1, 2): d = (c*P + dy)*P + dx
    row = pm[1 * Wc + 2]
    assert row.tolist() == [x[0, 1, 2], x[0, 1, 3], x[0, 2, 2], x[0, 2, 3],
                            x[1, 1, 2], x[1, 1, 3], x[1, 2, 2], x[1, 2, 3]]


@pytest.mark.parametrize("kind", ["uniform", "dup", "smooth"])
def test_single_key_distance_map_equals_exact_rational_bruteforce(kind):
    # the shifted-image form used for full-size single keys gives the same
    # groups as exact rational arithmetic, and its distances are the direct sums
    x = synth.workloads.random_image(2, 12, 12, seed=11, kind=kind)
    P, K = 3, 6
    keys = [0, 23, 50, 99]
    ref = _bf_exact(x, P, keys, K)
    for a, g in enumerate(keys):
        idx, dist, nxt = mt.topk_one(x, P, g, K)
        assert idx.tolist() == ref[a]
        full = mt.distance_map(x, P, g)
        np.testing.assert_allclose(full, mt.direct_distances(x, P, g, np.arange(full.size)),
                                   rtol=1e-13, atol=1e-300)
        assert nxt >= dist[-1]


def _bf_window_exact(x, P, keys, K, radius):
    """Pure-Python exact arithmetic over the key's window only."""
    C, H, W = x.shape
    Hc, Wc = H - P + 1, W - P + 1
    xf = [[[Fraction(float(x[c, r, q])) for q in range(W)] for r in range(H)] for c in range(C)]
    out = []
    for g in keys:
        gr, gc = divmod(int(g), Wc)
        ds = []
        for jr in range(Hc):
            for jc in range(Wc):
                if abs(jr - gr) > radius or abs(jc - gc) > radius:
                    continue
                d = Fraction(0)
                for c in range(C):
                    for dy in range(P):
                        for dx in range(P):
                            e = xf[c][gr + dy][gc + dx] - xf[c][jr + dy][jc + dx]
                            d += e * e
                ds.append((d, jr * Wc + jc))
        ds.sort()
        out.append([j for _, j in ds[:K]])
    return out


@pytest.mark.parametrize("kind", ["uniform", "dup"])
def test_window_topk_equals_exact_rational_bruteforce(kind):
    x = synth.workloads.random_image(2, 14, 13, seed=6, kind=kind)
    P, K, R = 3, 6, 3
    Wc = 13 - P + 1
    keys = [0, 5, 3 * Wc + 4, 11 * Wc + 10, 7 * Wc]
    idx, dist = mt.window_topk(x.astype(np.float64), P, keys, K, R)
    assert idx.tolist() == _bf_window_exact(x, P, keys, K, R)
    # members lie in the key's window
    for a, g in enumerate(keys):
        gr, gc = divmod(g, Wc)
        rr, cc = np.divmod(idx[a], Wc)
        assert np.all(np.abs(rr - gr) <= R) and np.all(np.abs(cc - gc) <= R)
        assert np.all(np.diff(dist[a]) >= 0)


def test_window_covering_the_grid_is_global_matching():
    x = synth.workloads.random_image(3, 16, 18, seed=7, kind="smooth")
    P, K = 4, 9
    keys = np.array([0, 40, 77, 160, 194])
    a, da = mt.window_topk(x.astype(np.float64), P, keys, K, radius=20)
    b, db = mt.topk_bruteforce(x.astype(np.float64), P, keys, K)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(da, db)


def test_window_too_small_for_k_is_refused():
    x = synth.workloads.random_image(1, 10, 10, seed=8)
    with pytest.raises(ValueError):
        mt.window_topk(x.astype(np.float64), 3, [0], 10, radius=2)   # 3 x 3 corner window
