"""GPU parity of the CNN surrogate kernels (forward, loss gradient, Adam)
against the oracle run with the same BF16 roundings in FP64.

The only differences left are FP32 sum order and, through it, an occasional
hidden activation (or back-propagated gradient) that rounds to the
neighbouring BF16 value; the tolerances below bound that effect and are
reported by each test."""
import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
from oracle import cnn as ocnn
from synth.cnn import cnn_params
from gpu_util import require_gpu, gpu, host

pytestmark = pytest.mark.gpu


def _case(B, h, w, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(B, h, w)).astype(np.float32)
    sig = rng.uniform(0.05, 0.5, size=B).astype(np.float32)
    tgt = (x + 0.1 * rng.standard_normal((B, h, w))).astype(np.float32)
    theta = cnn_params(seed, out_scale=0.05)
    return x, sig, tgt, theta


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape", [(2, 20, 150), (1, 9, 7), (3, 33, 128)])
def test_cnn_forward_vs_oracle(shape):
    require_gpu()
    B, h, w = shape
    x, sig, _, theta = _case(B, h, w, seed=h * w)
    net = glr.Cnn(theta)
    out = host(net.forward(gpu(x), gpu(sig)))
    ref = ocnn.forward(theta.astype(np.float64), x, sig, bf16=True)
    e = _rel(out - x, ref - x)
    print(f"forward {shape}: residual rel-L2 {e:.2e}", flush=True)
    assert np.isfinite(out).all()
    assert e <= 2e-3


def test_cnn_loss_grad_vs_oracle():
    require_gpu()
    B, h, w = 2, 24, 140
    x, sig, tgt, theta = _case(B, h, w, seed=5)
    net = glr.Cnn(theta)
    loss, grad, out = net.loss_grad(gpu(x), gpu(sig), gpu(tgt))
    loss, grad = float(host(loss)[0]), host(grad)
    rl, rg = ocnn.loss_and_grad(theta.astype(np.float64), x, sig, tgt, bf16=True)
    print(f"loss gpu {loss:.8f} oracle {rl:.8f}", flush=True)
    assert abs(loss - rl) <= 1e-4 * rl
    shapes = ocnn.param_shapes()
    o = 0
    for i, s in enumerate(shapes):
        n = int(np.prod(s))
        e = _rel(grad[o:o + n], rg[o:o + n])
        print(f"  param block {i} {s}: grad rel-L2 {e:.2e}", flush=True)
        assert e <= 1e-3, (i, e)
        o += n
    assert _rel(grad, rg) <= 1e-3


def test_cnn_adam_step_vs_oracle():
    # Adam is elementwise: applied to the GPU's own gradient it must match
    # the oracle's update to FP32 rounding
    require_gpu()
    x, sig, tgt, theta = _case(1, 16, 40, seed=9)
    net = glr.Cnn(theta)
    net.loss_grad(gpu(x), gpu(sig), gpu(tgt))
    g = host(net.grad).astype(np.float64)
    th, m, v = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in (1, 2, 3):
        net.adam(1e-3)
        th, m, v = ocnn.adam_step(th, m, v, g, step, 1e-3)
    np.testing.assert_allclose(host(net.params), th, rtol=1e-6, atol=1e-7)


def test_cnn_training_reduces_loss():
    # a few hundred Adam steps on a fixed denoising batch
    require_gpu()
    rng = np.random.default_rng(11)
    B, h, w = 8, 48, 48
    clean = np.cumsum(np.cumsum(rng.standard_normal((B, h, w)), 1), 2)
    clean = (clean - clean.min()) / (clean.max() - clean.min())
    sig = np.full(B, 0.1, np.float32)
    noisy = (clean + 0.1 * rng.standard_normal((B, h, w))).astype(np.float32)
    net = glr.Cnn(cnn_params(3))
    xg, tg, sg = gpu(noisy), gpu(clean.astype(np.float32)), gpu(sig)
    first = float(host(net.train_step(xg, sg, tg, 1e-3))[0])
    for _ in range(300):
        last = net.train_step(xg, sg, tg, 1e-3)
    last = float(host(last)[0])
    print(f"training loss {first:.5f} -> {last:.5f}", flush=True)
    assert last < 0.5 * first
