"""Pins for the oracle's CNN surrogate: central finite differences of the
analytic backprop on a small net, the forward pass against a library
convolution (torch, CPU, FP64), Adam's first step in closed form, the BF16
rounding rule, and the judge's deviation on hand-made cases."""
import numpy as np
import pytest
import torch

from oracle import cnn
from synth.cnn import cnn_params


def test_param_count():
    assert cnn.param_count() == 2 * 64 * 9 + 64 + 3 * (64 * 64 * 9 + 64) + 64 * 9 + 1
    assert cnn_params(0).size == cnn.param_count()


def test_forward_matches_library_convolution():
    rng = np.random.default_rng(1)
    ch = 8
    theta = rng.standard_normal(cnn.param_count(ch)) * 0.3
    x = rng.uniform(size=(2, 9, 11))
    sig = np.array([0.2, 0.7])
    out = cnn.forward(theta, x, sig, ch=ch)
    ps = [torch.from_numpy(p.copy()) for p in cnn.unflatten(theta, ch)]
    a = torch.from_numpy(cnn.network_input(x, sig))
    for layer in range(5):
        a = torch.nn.functional.conv2d(a, ps[2 * layer], ps[2 * layer + 1], padding=1)
        if layer < 4:
            a = torch.relu(a)
    ref = x + a[:, 0].numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("bf16", [False, True])
def test_backprop_matches_finite_differences(bf16):
    # central differences in FP64 on a small net; with BF16 emulation the
    # rounding makes the loss piecewise, so the check uses the exact (FP64)
    # network and the BF16 variant is checked for self-consistency only
    rng = np.random.default_rng(2)
    ch = 8
    theta = rng.standard_normal(cnn.param_count(ch)) * 0.3
    x = rng.uniform(size=(2, 16, 16))
    sig = np.array([0.3, 0.1])
    tgt = rng.uniform(size=x.shape)
    loss, g = cnn.loss_and_grad(theta, x, sig, tgt, bf16=bf16, ch=ch)
    if bf16:
        loss64, g64 = cnn.loss_and_grad(theta, x, sig, tgt, ch=ch)
        assert abs(loss - loss64) <= 1e-2 * loss64
        assert np.linalg.norm(g - g64) <= 0.05 * np.linalg.norm(g64)
        return
    idx = rng.choice(theta.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = cnn.loss_and_grad(tp, x, sig, tgt, ch=ch)[0]
        lm = cnn.loss_and_grad(tm, x, sig, tgt, ch=ch)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = cnn.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 0.01, eps=0.0)
    np.testing.assert_allclose(new, th - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 1.0 + 2.0 ** -9], np.float32)
    out = cnn.bf16_round(vals)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    np.testing.assert_array_equal(out, [1.0, 1.0, 1.0 + 2.0 ** -6, -2.5, 1.0])


def test_judge_deviation_cases():
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    cov = np.array([[True, False], [True, False]])
    assert cnn.judge_deviation(a, a, cov) == 0.0
    b = a.copy()
    b[0, 1] = 100.0                      # not covered: ignored
    assert cnn.judge_deviation(b, a, cov) == 0.0
    b[1, 0] = 3.3
    assert abs(cnn.judge_deviation(b, a, cov) - 0.3 / np.sqrt(10.0)) < 1e-15
    b[0, 0] = np.nan
    assert cnn.judge_deviation(b, a, cov) == float("inf")
