"""Smallest checks of the library on the GPU: it loads, plans, forward op."""
import numpy as np
import pytest
import torch

import paper_2301_03047_amd as glr
import synth
from oracle import operators as ops
from gpu_util import require_gpu, gpu, host

pytestmark = pytest.mark.gpu


def test_cacti_forward_adjoint():
    require_gpu()
    F, H, W = 8, 33, 47
    m = synth.cacti_masks(F, H, W, 1)
    x = np.random.default_rng(0).uniform(size=(F, H, W)).astype(np.float32)
    plan = glr.Plan("cacti", H, W, F, 4, 8, 4, mask=gpu(m))
    y = host(plan.forward(gpu(x)))
    ref = ops.cacti_forward(x.astype(np.float64), m)
    assert np.abs(y - ref).max() <= 1e-6 * np.abs(ref).max()
    yy = np.random.default_rng(1).uniform(size=(H, W)).astype(np.float32)
    xa = host(plan.adjoint(gpu(yy)))
    np.testing.assert_array_equal(xa, ops.cacti_adjoint(yy.astype(np.float64), m).astype(np.float32))
