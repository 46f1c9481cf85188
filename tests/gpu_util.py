"""Helpers for the GPU parity tests (imported by test modules, not collected)."""
import numpy as np
import torch

import paper_2301_03047_amd as glr
from oracle import matching as om

WNNM_C = float(np.float32(2.0 * np.sqrt(2.0)))   # the FP32 value the library uses
WNNM_EPS = float(np.float32(1e-16))


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def planar(z):
    """complex [H][W] -> float64 planar [2][H][W] (exact)."""
    return np.stack([np.real(z), np.imag(z)]).astype(np.float64)


def ones_mask(C, H, W):
    return torch.ones((C, H, W), dtype=torch.uint8, device="cuda")


def check_groups(x64, P, keys, idx_gpu, idx_ref, rtol=1e-9):
    """Groups must be identical, except rows where the oracle's own direct
    distances show the differing members tie within ``rtol`` (relative to the
    row's largest distance): such rows count as numerical ties, the GPU's
    members must still be distinct and its distance profile must match.
    Returns the number of tie rows."""
    idx_gpu = np.asarray(idx_gpu)
    idx_ref = np.asarray(idx_ref)
    assert idx_gpu.shape == idx_ref.shape
    ties = 0
    bad = np.nonzero((idx_gpu != idx_ref).any(axis=1))[0]
    if len(bad) == 0:
        return 0
    pm = om.patch_matrix(x64, P)
    for a in bad:
        k = pm[keys[a]]
        dg = np.sum((pm[idx_gpu[a]] - k) ** 2, axis=1)
        dr = np.sum((pm[idx_ref[a]] - k) ** 2, axis=1)
        assert len(set(idx_gpu[a].tolist())) == idx_gpu.shape[1], f"row {a}: duplicate members"
        scale = max(float(dr.max()), 1e-300)
        diff = np.abs(np.sort(dg) - np.sort(dr)).max()
        assert diff <= rtol * scale, (
            f"row {a}: groups differ beyond a numerical tie (max |dd| {diff:.3e}, "
            f"scale {scale:.3e})\n gpu {idx_gpu[a].tolist()}\n ref {idx_ref[a].tolist()}")
        # order by distance must also hold for the GPU row
        assert np.all(np.diff(dg) >= -rtol * scale), f"row {a}: GPU row not sorted by distance"
        ties += 1
    return ties
