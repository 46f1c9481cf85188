"""Pins for the oracle's sensing operators (eq. 2-5) and data steps."""
import numpy as np
import pytest

import synth
from oracle import operators as ops


def _rng(s):
    return np.random.default_rng(s)


def test_cacti_adjointness():
    r = _rng(1)
    F, H, W = 5, 9, 7
    m = synth.cacti_masks(F, H, W, 3)
    x = r.standard_normal((F, H, W))
    y = r.standard_normal((H, W))
    lhs = np.vdot(ops.cacti_forward(x, m), y)
    rhs = np.vdot(x, ops.cacti_adjoint(y, m))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_cacti_phi_phit_is_mask_sum():
    # for binary masks Phi Phi^T = diag(sum_t A_t^2) = diag(R)
    F, H, W = 8, 6, 5
    m = synth.cacti_masks(F, H, W, 4)
    y = _rng(2).integers(-50, 50, size=(H, W)).astype(np.float64)  # exact sums
    R = m.astype(np.int64).sum(0)
    np.testing.assert_array_equal(ops.cacti_forward(ops.cacti_adjoint(y, m), m), R * y)
    np.testing.assert_array_equal(ops.cacti_mask_sum(m), R)


def test_cacti_forward_bruteforce():
    F, H, W = 3, 4, 5
    m = synth.cacti_masks(F, H, W, 5)
    x = _rng(3).standard_normal((F, H, W))
    y = ops.cacti_forward(x, m)
    for r in range(H):
        for c in range(W):
            s = 0.0
            for t in range(F):
                if m[t, r, c]:
                    s += x[t, r, c]
            assert abs(y[r, c] - s) <= 1e-14


def test_msfa_orthogonal_masks_give_identity():
    # eq. 5: A_i (.) A_j = 0 for i != j, each pixel in exactly one band
    H, W = 8, 12
    b = ops.msfa_band_map(H, W)
    for i in range(16):
        for j in range(16):
            if i != j:
                assert not np.any((b == i) & (b == j))
    assert set(np.unique(b)) == set(range(16))
    y = _rng(6).standard_normal((H, W))
    np.testing.assert_array_equal(ops.msfa_forward(ops.msfa_adjoint(y, 16)), y)


def test_msfa_adjointness_and_init():
    r = _rng(7)
    x = r.standard_normal((16, 8, 8))
    y = r.standard_normal((8, 8))
    lhs = np.vdot(ops.msfa_forward(x), y)
    rhs = np.vdot(x, ops.msfa_adjoint(y, 16))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    x0 = ops.msfa_init(ops.msfa_forward(x), 16)
    # the replicated start is consistent with the measurement
    np.testing.assert_array_equal(ops.msfa_forward(x0), ops.msfa_forward(x))
    # band 5 = (row 1, col 1) of each cell
    assert x0[5, 4, 6] == x[5, 5, 5]


def _dft_matrix(n):
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def test_fft2c_matches_explicit_dft():
    r = _rng(8)
    H, W = 8, 16
    x = r.standard_normal((H, W)) + 1j * r.standard_normal((H, W))
    ref = _dft_matrix(H) @ x @ _dft_matrix(W).T
    np.testing.assert_allclose(ops.fft2c(x), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ops.ifft2c(ref), x, rtol=0, atol=1e-12)
    # Parseval for the orthonormal transform
    assert abs(np.linalg.norm(ops.fft2c(x)) - np.linalg.norm(x)) < 1e-12


def test_mri_adjointness_and_mask():
    r = _rng(9)
    H, W = 16, 8
    m = synth.mri_line_mask(H, 11)
    assert m.sum() == 4 and m[:2].all() and m[-2:].all()
    x = r.standard_normal((H, W)) + 1j * r.standard_normal((H, W))
    y = r.standard_normal((H, W)) + 1j * r.standard_normal((H, W))
    lhs = np.vdot(y, ops.mri_forward(x, m))
    rhs = np.vdot(ops.mri_adjoint(y, m), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_mri_line_mask_geometry():
    m = synth.mri_line_mask(256, 1001)
    assert m.sum() == 64
    assert m[:8].all() and m[-8:].all()


def test_gap_is_consistent_where_R_positive():
    r = _rng(10)
    F, H, W = 8, 10, 10
    m = synth.cacti_masks(F, H, W, 12)
    x = r.uniform(size=(F, H, W))
    y = ops.cacti_forward(r.uniform(size=(F, H, W)), m)
    R = ops.cacti_mask_sum(m)
    xb = ops.gap_update(x, y, lambda v: ops.cacti_forward(v, m),
                        lambda q: ops.cacti_adjoint(q, m), R)
    yb = ops.cacti_forward(xb, m)
    np.testing.assert_allclose(yb[R > 0], y[R > 0], rtol=0, atol=1e-12)
    # pixels with no open mask receive no update
    np.testing.assert_array_equal(xb[:, R == 0], x[:, R == 0])


def test_admm_x_update_solves_its_subproblem():
    # x = argmin ||M F x - y||^2 + rho ||x - (z - u)||^2  <=>  gradient zero
    r = _rng(13)
    H, W = 16, 16
    m = synth.mri_line_mask(H, 14)
    y = ops.mri_forward(r.standard_normal((H, W)) + 1j * r.standard_normal((H, W)), m)
    z = r.standard_normal((H, W)) + 1j * r.standard_normal((H, W))
    u = r.standard_normal((H, W)) + 1j * r.standard_normal((H, W))
    rho = 0.7
    x = ops.admm_x_update(y, z, u, m, rho)
    M = ops.mri_mask2d(m, W)
    grad = ops.ifft2c(M * (M * ops.fft2c(x) - y)) + rho * (x - (z - u))
    assert np.abs(grad).max() < 1e-12


def test_accelerated_gap_makes_a_linear_shrink_consistent():
    # with the prior x -> x / 2 the accelerated iteration's fixed point has
    # Phi x = y (the accumulated residual undoes the shrink); plain GAP keeps
    # a residual of the order of the shrink
    import synth
    F, H, W = 4, 12, 10
    m = synth.cacti_masks(F, H, W, 3)
    rng = np.random.default_rng(4)
    y = ops.cacti_forward(rng.uniform(size=(F, H, W)), m)
    R = ops.cacti_mask_sum(m)
    fwd = lambda v: ops.cacti_forward(v, m)
    adj = lambda r: ops.cacti_adjoint(r, m)
    x = ops.cacti_adjoint(y / np.where(R == 0, 1.0, R), m)
    xa, ya = x.copy(), y.copy()
    for _ in range(400):
        xb, ya = ops.gap_acc_update(xa, y, ya, fwd, adj, R)
        xa = 0.5 * xb
        x = 0.5 * ops.gap_update(x, y, fwd, adj, R)
    ok = R > 0
    assert np.abs(fwd(xa) - y)[ok].max() <= 1e-9 * np.abs(y).max()
    assert np.abs(fwd(x) - y)[ok].max() >= 0.1 * np.abs(y)[ok].min()


def test_accelerated_gap_step_by_hand():
    # one pixel, two frames, both masks open: Phi x = x0 + x1, R = 2
    m = np.ones((2, 1, 1), np.uint8)
    x = np.array([[[0.25]], [[0.5]]])
    y = np.array([[1.5]])
    y_acc = np.array([[1.5]])
    xb, ya = ops.gap_acc_update(x, y, y_acc, lambda v: ops.cacti_forward(v, m),
                                lambda r: ops.cacti_adjoint(r, m), ops.cacti_mask_sum(m))
    # y_acc' = 1.5 + (1.5 - 0.75) = 2.25; update (2.25 - 0.75) / 2 = 0.75 per frame
    assert ya[0, 0] == 2.25
    np.testing.assert_array_equal(xb[:, 0, 0], [1.0, 1.25])
