"""Seeded initial parameters of the residual CNN surrogate (flat FP32, in the
order W1, b1, ..., W5, b5 with W_l [co][ci][3][3]): He-normal hidden layers,
a small output layer, zero biases."""
import numpy as np


def cnn_params(seed, ch=64, out_scale=1e-3):
    rng = np.random.default_rng(seed)
    shapes = [(2, ch), (ch, ch), (ch, ch), (ch, ch), (ch, 1)]
    parts = []
    for i, (ci, co) in enumerate(shapes):
        std = out_scale if i == len(shapes) - 1 else np.sqrt(2.0 / (ci * 9))
        parts.append((rng.standard_normal((co, ci, 3, 3)) * std).ravel())
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
