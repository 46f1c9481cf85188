"""Pins for the oracle's WNNM group shrinkage and aggregation."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import lowrank as lr
from oracle import aggregate as ag
from oracle import prior as pr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rank1_group(D, K, s1, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(D)
    u /= np.linalg.norm(u)
    v = rng.standard_normal(K)
    v -= v.mean()               # v orthogonal to the ones vector: centring keeps it
    v /= np.linalg.norm(v)
    mu = rng.uniform(size=D)
    return mu[:, None] + s1 * np.outer(u, v), mu, u, v


def test_rank1_golden_value():
    g = json.load(open(os.path.join(GOLD, "wnnm_rank1.json")))
    Y, mu, u, v = _rank1_group(9, g["K"], g["s1"], 0)
    X, s = lr.wnnm_group(Y, g["sigma"], g["c"], g["eps"])
    assert abs(s[0] - g["s1"]) < 1e-12 and np.all(s[1:] < 1e-12)
    expect = mu[:, None] + g["s1_shrunk"] * np.outer(u, v)
    np.testing.assert_allclose(X, expect, rtol=0, atol=1e-12)


def test_sigma_zero_is_identity():
    Y = np.random.default_rng(1).uniform(size=(20, 7))
    X, _ = lr.wnnm_group(Y, 0.0, 2.8, 1e-16)
    np.testing.assert_array_equal(X, Y)


def test_huge_sigma_gives_row_mean():
    Y = np.random.default_rng(2).uniform(size=(12, 6))
    X, _ = lr.wnnm_group(Y, 1e3, 2.8, 1e-16)
    np.testing.assert_allclose(X, np.repeat(Y.mean(1, keepdims=True), 6, axis=1), atol=1e-12)


def test_exact_low_rank_recovery_keeps_rank():
    rng = np.random.default_rng(3)
    D, K, r = 30, 16, 3
    Y = rng.standard_normal((D, r)) @ rng.standard_normal((r, K)) * 2 + 0.5
    X, s = lr.wnnm_group(Y, 0.05, 2 * np.sqrt(2), 1e-16)
    Xc = X - X.mean(1, keepdims=True)
    sx = np.linalg.svd(Xc, compute_uv=False)
    assert np.all(sx[r:] < 1e-10 * sx[0])
    # only the threshold moves the retained singular values
    s_new = lr.wnnm_weights(s[:r], K, 0.05, 2 * np.sqrt(2), 1e-16)
    np.testing.assert_allclose(sx[:r], s_new, rtol=1e-10)


def test_shrinkage_bounds_and_denoising():
    rng = np.random.default_rng(4)
    D, K, r, sig = 64, 32, 2, 0.1
    clean = rng.standard_normal((D, r)) @ rng.standard_normal((r, K)) + 0.3
    errs = []
    for t in range(5):
        noisy = clean + sig * rng.standard_normal((D, K))
        X, s = lr.wnnm_group(noisy, sig, 2 * np.sqrt(2), 1e-16)
        sn = lr.wnnm_weights(s, K, sig, 2 * np.sqrt(2), 1e-16)
        assert np.all(sn >= 0) and np.all(sn <= s)
        errs.append((np.linalg.norm(X - clean), np.linalg.norm(noisy - clean)))
    assert all(a < b for a, b in errs)


def test_lapack_svd_invariants():
    Y = np.random.default_rng(5).standard_normal((40, 12))
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    assert np.abs(U.T @ U - np.eye(12)).max() < 1e-12
    assert np.abs(Vt @ Vt.T - np.eye(12)).max() < 1e-12
    assert np.linalg.norm(U * s @ Vt - Y) / np.linalg.norm(Y) < 1e-12


def test_aggregate_identity_shrink_dyadic():
    # sigma = 0 -> every estimate equals its patch; dyadic values make the
    # per-pixel mean exact, so the prior step returns its input bit for bit
    rng = np.random.default_rng(6)
    x = rng.integers(0, 256, size=(2, 20, 22)).astype(np.float64) / 256.0
    out = pr.prior_step(x, 4, 12, 9, 0.0, 2.8, 1e-16)
    np.testing.assert_array_equal(out["x_out"], x)


def test_aggregate_constant_image_and_counts():
    x = np.full((3, 16, 17), 0.375)
    out = pr.prior_step(x, 5, 6, 7, 0.05, 2.8, 1e-16)
    np.testing.assert_allclose(out["x_out"], x, atol=1e-15)
    cnt = ag.coverage_count(16, 17, 5, out["idx"])
    np.testing.assert_array_equal(out["count"], cnt)


def test_aggregate_single_member_by_hand():
    xbar = np.zeros((1, 6, 7))
    P, Wc = 2, 6
    idx = np.array([[1 * Wc + 3]])
    est = np.full((1, 1, 4), 7.0)
    out, cnt = ag.aggregate(xbar, P, idx, est)
    expect = np.zeros((1, 6, 7))
    expect[0, 1:3, 3:5] = 7.0
    np.testing.assert_array_equal(out, expect)
    # two members overlapping one pixel: the mean
    idx = np.array([[0, 1 * Wc + 1]])
    est = np.stack([np.full(4, 2.0), np.full(4, 4.0)])[None]
    out, cnt = ag.aggregate(xbar, P, idx, est)
    assert out[0, 1, 1] == 3.0 and out[0, 0, 0] == 2.0 and out[0, 2, 2] == 4.0
    assert cnt[1, 1] == 2 and cnt[3, 3] == 0


def test_shrink_groups_orientation_closed_form():
    """Group orientation of shrink_groups: members are the columns of the
    D x K group and the mean is taken over members.  The group's members are
    planted as p_j = m + alpha_j u, so Y = m 1^T + u alpha^T has rank 2 and
    only the member-mean removal leaves a rank-1 matrix:
    Y - mean = u (alpha - mean(alpha))^T with singular value
    ||u|| ||alpha - mean(alpha)|| = 1.5 * 2 = 3.  With K = 4, sigma = 0.5,
    c = 2 sqrt(2) the WNNM weight is tau = c sqrt(K) sigma^2 / sqrt(s^2 - K
    sigma^2) = 2 sqrt(2) * 2 * 0.25 / sqrt(8) = 0.5 (the golden rank-1
    value), so s' = 2.5 and the estimate of member j is
    m + mean(alpha) u + (2.5 / 3) (alpha_j - mean(alpha)) u.
    A transposed group (K x D) or a mean over patch elements gives other
    singular values (the second one is not zero) and another estimate."""
    C, P, H, W = 2, 2, 6, 9
    D, K = C * P * P, 4
    Wc = W - P + 1
    rng = np.random.default_rng(21)
    x = rng.uniform(size=(C, H, W))
    m = np.linspace(0.1, 0.8, D)                       # d = (c P + dy) P + dx
    u = np.array([0.75, 0.75, 0.75, 0.75, 0.0, 0.0, 0.0, 0.0])   # ||u|| = 1.5
    alpha = np.array([2.0, 0.0, 2.0, 0.0])             # mean 1, centred norm 2
    tops = [(0, 0), (0, 3), (0, 6), (3, 2)]            # disjoint 2 x 2 patches
    for j, (r, c0) in enumerate(tops):
        for ch in range(C):
            for dy in range(P):
                for dx in range(P):
                    d = (ch * P + dy) * P + dx
                    x[ch, r + dy, c0 + dx] = m[d] + alpha[j] * u[d]
    idx = np.array([[r * Wc + c0 for (r, c0) in tops]])
    Xhat, sv = lr.shrink_groups(x, P, idx, 0.5, 2 * np.sqrt(2), 1e-16)
    assert Xhat.shape == (1, K, D) and sv.shape == (1, K)
    np.testing.assert_allclose(sv[0], [3.0, 0.0, 0.0, 0.0], atol=1e-12)
    for j in range(K):
        expect = m + 1.0 * u + (2.5 / 3.0) * (alpha[j] - 1.0) * u
        np.testing.assert_allclose(Xhat[0, j], expect, atol=1e-12)


def test_gather_groups_loop_by_loop():
    """gather_groups returns member-major [N][K][D] with d = (c P + dy) P + dx,
    compared with an explicit loop over members and patch elements."""
    C, P, H, W = 3, 3, 7, 8
    Wc = W - P + 1
    x = np.random.default_rng(22).uniform(size=(C, H, W))
    idx = np.array([[0, 5, 17], [29, 3, 11]])
    G = lr.gather_groups(x, P, idx)
    for g in range(idx.shape[0]):
        for j in range(idx.shape[1]):
            r, c0 = divmod(int(idx[g, j]), Wc)
            for ch in range(C):
                for dy in range(P):
                    for dx in range(P):
                        assert G[g, j, (ch * P + dy) * P + dx] == x[ch, r + dy, c0 + dx]


def test_weighted_aggregation_by_hand_and_uniform_limit():
    from oracle import aggregate as oag
    # two one-pixel patches (P = 1) on the same pixel: (1 * 2 + 3 / 3) / (1 + 1 / 3)
    xbar = np.zeros((1, 2, 2))
    idx = np.array([[0], [0]])
    Xhat = np.array([[[2.0]], [[3.0]]])
    out, cnt = oag.aggregate(xbar, 1, idx, Xhat, weights=[1.0, 1.0 / 3.0])
    assert out[0, 0, 0] == (2.0 + 1.0) / (1.0 + 1.0 / 3.0)
    assert cnt[0, 0] == 1.0 + 1.0 / 3.0 and out[0, 1, 1] == 0.0
    # equal weights reduce to the uniform mean
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(2, 9, 9))
    idx = rng.integers(0, 49, size=(5, 4))
    Xh = rng.uniform(size=(5, 4, 2 * 9))
    a, _ = oag.aggregate(x, 3, idx, Xh)
    b, _ = oag.aggregate(x, 3, idx, Xh, weights=np.full(5, 0.25))
    np.testing.assert_allclose(a, b, rtol=1e-14)


def test_group_weights_count_the_kept_components():
    from oracle import lowrank as olr
    # K = 4, sigma = 0.5: a singular value is kept iff s - tau > 0; with
    # s^2 = K sigma^2 + shat^2, s = 3 keeps (tau = c sqrt(K) sigma^2 / shat)
    c, eps, K, sig = 2 * np.sqrt(2), 1e-16, 4, 0.5
    sv = np.array([[3.0, 0.2, 0.0, 0.0], [3.0, 2.5, 0.1, 0.0], [0.1, 0.05, 0.0, 0.0]])
    kept = (olr.wnnm_weights(sv, K, sig, c, eps) > 0).sum(axis=1)
    assert kept.tolist() == [1, 2, 0]
    np.testing.assert_array_equal(olr.group_weights(sv, K, sig, c, eps), [1.0, 0.5, 1.0])


def test_inner_iterations_worked_by_hand():
    # the recursion with a stand-in step x = y / 2 (any shrink-and-aggregate
    # map can be passed in): xbar = 1, x1 = 1/2, delta = 0.1, lam = 0.5, sigma = 2
    #   y2 = 0.5 + 0.1 (1 - 1)   = 0.5,   sigma2 = 0.5 sqrt(4 - 0.25)   = 0.5 sqrt(3.75)
    #   x2 = 0.25
    #   y3 = 0.25 + 0.1 (1 - 0.5) = 0.3,  sigma3 = 0.5 sqrt(4 - 0.49)   = 0.5 sqrt(3.51)
    #   x3 = 0.15
    from oracle.prior import inner_iterations
    seen = []

    def step(y, s):
        seen.append((float(y[0]), s))
        return None, None, None, y / 2, None
    x, sig, _ = inner_iterations(np.ones(1), np.full(1, 0.5), 2.0, 3, 0.1, 0.5, step)
    assert abs(x[0] - 0.15) < 1e-15
    np.testing.assert_allclose(sig, [2.0, 0.5 * np.sqrt(3.75), 0.5 * np.sqrt(3.51)], rtol=1e-15)
    np.testing.assert_allclose([v for v, _ in seen], [0.5, 0.3], rtol=1e-15)


def test_inner_iterations_special_cases():
    from oracle import prior as opr
    from synth.workloads import random_image
    C, H, W, P, N, K = 3, 24, 26, 4, 12, 8
    x = random_image(C, H, W, seed=9).astype(np.float64)
    c, eps = 2 * np.sqrt(2), 1e-16
    # sigma = 0: every shrinkage is the identity, so every iteration returns xbar
    r = opr.prior_step(x, P, N, K, 0.0, c, eps, inner=4)
    np.testing.assert_allclose(r["x_out"], x, rtol=0, atol=1e-12)
    assert r["sigmas"] == [0.0, 0.0, 0.0, 0.0]
    # one iteration is the plain step; the second sees a smaller noise level
    one = opr.prior_step(x, P, N, K, 0.05, c, eps)
    two = opr.prior_step(x, P, N, K, 0.05, c, eps, inner=2)
    assert len(one["sigmas"]) == 1 and 0 < two["sigmas"][1] < 0.54 * 0.05
    np.testing.assert_array_equal(one["idx"], two["idx"])
    assert np.abs(two["x_out"] - one["x_out"]).max() > 1e-6
    # delta = 0 and lam chosen so sigma_2 = sigma: the second shrinkage acts on x^(1)
    # (y2 = x1) with the first sigma, i.e. two plain steps on fixed groups
    d = np.mean((x - one["x_out"]) ** 2)
    lam = 0.05 / np.sqrt(0.05 ** 2 - d)
    two0 = opr.prior_step(x, P, N, K, 0.05, c, eps, inner=2, delta=0.0, lam=lam)
    from oracle import aggregate as oag
    Xh, _ = lr.shrink_groups(one["x_out"], P, one["idx"], 0.05, c, eps)
    again, _ = oag.aggregate(one["x_out"], P, one["idx"], Xh)
    np.testing.assert_allclose(two0["sigmas"][1], 0.05, rtol=1e-12)
    np.testing.assert_allclose(two0["x_out"], again, rtol=1e-12, atol=1e-14)


# ---- complex-Hermitian form (complex data shrunk as complex matrices)

def _cgroup(d, K, seed, zero_mean=False):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((d, K)) + 1j * rng.standard_normal((d, K))
    if zero_mean:
        Z -= Z.mean(axis=1, keepdims=True)
    return Z


def test_complex_wnnm_real_group_is_the_real_form():
    # a group with no imaginary part: the complex SVD is the real one, so the
    # complex form equals the (separately pinned) real form
    rng = np.random.default_rng(11)
    Y = rng.uniform(size=(18, 12))
    X, s = lr.wnnm_group_complex(Y.astype(np.complex128), 0.3, 2.8, 1e-16)
    Xr, sr = lr.wnnm_group(Y, 0.3, 2.8, 1e-16)
    np.testing.assert_allclose(X.real, Xr, atol=1e-12)
    assert np.abs(X.imag).max() < 1e-12
    np.testing.assert_allclose(s, sr, rtol=1e-12, atol=1e-12)


def test_complex_wnnm_real_representation():
    # a zero-mean complex group Z = A + iB and its real representation
    # M = [[A, -B], [B, A]]: M's singular values are Z's, each twice, and
    # shrinking M's SVD by the same rule (K = Z's member count) gives the real
    # representation of the complex estimate.  A conjugate or transpose
    # missing anywhere in the complex form breaks this.
    d, K, sigma = 9, 14, 0.4
    Z = _cgroup(d, K, 12, zero_mean=True)
    X, s = lr.wnnm_group_complex(Z, sigma, 2.8, 1e-16)
    A, B = Z.real, Z.imag
    M = np.block([[A, -B], [B, A]])
    U, sm, Vt = np.linalg.svd(M, full_matrices=False)
    np.testing.assert_allclose(sm[0:2 * d:2], s, rtol=1e-12)
    np.testing.assert_allclose(sm[1:2 * d:2], s, rtol=1e-12)
    XM = M - (U * (sm - lr.wnnm_weights(sm, K, sigma, 2.8, 1e-16))[None, :]) @ Vt
    np.testing.assert_allclose(XM, np.block([[X.real, -X.imag], [X.imag, X.real]]), atol=1e-12)


def test_complex_wnnm_phase_equivariance():
    # a global phase e^{i theta} rotates the complex estimate by the same
    # phase and leaves the singular values
    d, K, sigma, th = 16, 10, 0.5, 0.7
    Z = _cgroup(d, K, 13)
    X, s = lr.wnnm_group_complex(Z, sigma, 2.8, 1e-16)
    Xp, sp = lr.wnnm_group_complex(Z * np.exp(1j * th), sigma, 2.8, 1e-16)
    np.testing.assert_allclose(Xp, X * np.exp(1j * th), atol=1e-12)
    np.testing.assert_allclose(sp, s, rtol=1e-12, atol=1e-12)


def test_complex_wnnm_rank_one_closed_form():
    # mu 1^T + s1 u v^H with unit u, v and v orthogonal to the ones vector:
    # one singular value s1, and the estimate keeps mu and scales the rank-one
    # term to the shrunk value
    rng = np.random.default_rng(14)
    d, K, s1, sigma = 8, 12, 5.0, 0.3
    u = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    u /= np.linalg.norm(u)
    v = rng.standard_normal(K) + 1j * rng.standard_normal(K)
    v -= v.mean()
    v /= np.linalg.norm(v)
    mu = rng.uniform(size=d) + 1j * rng.uniform(size=d)
    Z = mu[:, None] + s1 * np.outer(u, v.conj())
    X, s = lr.wnnm_group_complex(Z, sigma, 2.8, 1e-16)
    assert abs(s[0] - s1) < 1e-12 and np.all(s[1:] < 1e-12)
    shat = np.sqrt(s1 * s1 - K * sigma * sigma)
    s1n = s1 - 2.8 * np.sqrt(K) * sigma * sigma / (shat + 1e-16)
    np.testing.assert_allclose(X, mu[:, None] + s1n * np.outer(u, v.conj()), atol=1e-12)
    X0, _ = lr.wnnm_group_complex(Z, 0.0, 2.8, 1e-16)
    np.testing.assert_array_equal(X0, Z)
    # the real-stacked group [Re; Im] of the same data has rank two: the two
    # forms differ
    _, s2 = lr.wnnm_group(np.vstack([Z.real, Z.imag]), sigma, 2.8, 1e-16)
    assert s2[1] > 1e-3 * s2[0]


def test_shrink_groups_complex_packing():
    # a planar complex image with a zero imaginary plane: the complex groups
    # are the real groups of the real plane, written back as [Re; 0]; and on
    # a general image the [Re; Im] halves are Re and Im of the complex group
    # estimate of the gathered complex patches
    rng = np.random.default_rng(15)
    P, K = 3, 7
    re = rng.uniform(size=(1, 14, 13))
    x = np.concatenate([re, np.zeros_like(re)])
    idx = rng.choice(12 * 11, size=(5, K), replace=False).reshape(5, K)
    Xc, svc = lr.shrink_groups(x, P, idx, 0.2, 2.8, 1e-16, complex_groups=True)
    Xr, svr = lr.shrink_groups(re, P, idx, 0.2, 2.8, 1e-16)
    np.testing.assert_allclose(Xc[:, :, :P * P], Xr, atol=1e-12)
    assert np.abs(Xc[:, :, P * P:]).max() < 1e-12
    np.testing.assert_allclose(svc, svr[:, :min(P * P, K)], rtol=1e-10, atol=1e-12)
    x = rng.uniform(size=(2, 14, 13))
    Xc, svc = lr.shrink_groups(x, P, idx, 0.2, 2.8, 1e-16, complex_groups=True)
    assert svc.shape == (5, min(P * P, K))
    g = 3
    Zg = np.array([[x[0, t // 13 + dy, t % 13 + dx] + 1j * x[1, t // 13 + dy, t % 13 + dx]
                    for dy in range(P) for dx in range(P)] for t in
                   [(i // 11) * 13 + i % 11 for i in idx[g]]]).T
    Xg, sg = lr.wnnm_group_complex(Zg, 0.2, 2.8, 1e-16)
    np.testing.assert_allclose(Xc[g, :, :P * P], Xg.T.real, atol=1e-12)
    np.testing.assert_allclose(Xc[g, :, P * P:], Xg.T.imag, atol=1e-12)
    np.testing.assert_allclose(svc[g], sg, rtol=1e-12)
    with pytest.raises(ValueError):
        pr.prior_step(x, P, 5, K, 0.2, 2.8, 1e-16, lowrank="complex")
