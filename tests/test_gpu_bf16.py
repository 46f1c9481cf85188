"""BF16 form of the matcher (mean-centred key and candidate patches on BF16
MFMA, FP32 accumulation, its own certified bound).  The margin set is
rescored with the same FP64 arithmetic as the FP32 form, so the bar
is unchanged: groups identical to the oracle's exact top-K, distances within
1e-6 relative, and identical (bitwise) to the FP32 form's output."""
import numpy as np
import pytest

import paper_2301_03047_amd as glr
import synth
from synth.workloads import random_image
from oracle import matching as om, operators as ops, detector as odet
from gpu_util import require_gpu, gpu, host, ones_mask, check_groups

pytestmark = pytest.mark.gpu


def _plan(C, H, W, P, N, K, **kw):
    return glr.Plan("cacti", H, W, C, P, N, K, mask=ones_mask(C, H, W), **kw)


BF16_CASES = [
    # C, H, W, P, N, K, kind     (ragged tiles, odd and even P, P = 1, P = 16)
    (2, 12, 12, 3, 5, 5, "uniform"),
    (2, 21, 150, 3, 17, 5, "smooth"),
    (8, 40, 41, 6, 130, 32, "smooth"),
    (3, 37, 29, 7, 50, 64, "uniform"),
    (1, 64, 300, 5, 257, 45, "smooth"),
    (2, 30, 30, 1, 40, 9, "uniform"),
    (1, 40, 40, 16, 20, 8, "smooth"),
    (4, 24, 24, 4, 30, 11, "dup"),
    (24, 48, 160, 8, 150, 64, "smooth"),
    (40, 36, 44, 4, 30, 16, "smooth"),
]


@pytest.mark.parametrize("case", BF16_CASES, ids=lambda c: "x".join(map(str, c[:6])) + c[6])
def test_bf16_match_topk_vs_oracle(case):
    require_gpu()
    C, H, W, P, N, K, kind = case
    print("bf16 case", case, flush=True)
    x = random_image(C, H, W, seed=H * W + P, kind=kind)
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.sort(np.random.default_rng(7).choice(n_cand, size=N, replace=False))
    plan = _plan(C, H, W, P, N, K, precision="bf16")
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    idx, dist = host(idx), host(dist)
    ref_idx, ref_dist = om.topk_exact(x.astype(np.float64), P, keys, K)
    ties = check_groups(x.astype(np.float64), P, keys, idx, ref_idx)
    assert ties == 0, f"{ties} numerical-tie rows"
    np.testing.assert_allclose(dist, ref_dist, rtol=1e-6, atol=1e-30)


@pytest.mark.parametrize("offset", [0.0, 40.0])
def test_bf16_equals_fp32_form(offset):
    # a large common offset is where centring matters: without it the BF16
    # rounding of the raw values would swamp every distance
    require_gpu()
    C, H, W, P, N, K = 8, 96, 128, 6, 300, 32
    x = (random_image(C, H, W, seed=21, kind="smooth") + np.float32(offset)).astype(np.float32)
    keys = np.arange(0, N * 29, 29).astype(np.int32)
    a = _plan(C, H, W, P, N, K, precision="fp32")
    b = _plan(C, H, W, P, N, K, precision="bf16")
    ia, da = a.match_topk(gpu(x), gpu(keys))
    ib, db = b.match_topk(gpu(x), gpu(keys))
    np.testing.assert_array_equal(host(ia), host(ib))
    np.testing.assert_array_equal(host(da), host(db))
    sa, sb = a.read_stats(), b.read_stats()
    print("margins fp32", sa["margin_sum"] / N, "bf16", sb["margin_sum"] / N, flush=True)
    ref, _ = om.topk_exact(x.astype(np.float64), P, keys, K)
    assert check_groups(x.astype(np.float64), P, keys, host(ib), ref) == 0


def test_bf16_small_chunks_and_splits():
    require_gpu()
    C, H, W, P, N, K = 3, 64, 200, 5, 300, 20
    x = random_image(C, H, W, seed=3, kind="smooth")
    keys = np.arange(0, N * 37, 37)
    plan = _plan(C, H, W, P, N, K, dist_chunk_mb=1, precision="bf16")
    idx, _ = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    ref, _ = om.topk_exact(x.astype(np.float64), P, keys, K)
    assert check_groups(x.astype(np.float64), P, keys, host(idx), ref) == 0


@pytest.mark.parametrize("H,W", [(40, 50), (200, 200)])
def test_bf16_constant_image_exact_path(H, W):
    # every centred patch is zero, so every d~ and every bound is exactly 0:
    # all candidates tie, the range lists overflow and the keys are
    # re-matched in FP32, where the margin set is re-derived from the
    # distance row (40 x 50) or, above 32768 candidates, the exact full-row
    # path runs (200 x 200); lowest positions win
    require_gpu()
    C, P, N, K = 2, 4, 6, 10
    x = np.full((C, H, W), 0.3, dtype=np.float32)
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.linspace(0, n_cand - 1, N).astype(np.int64)
    plan = _plan(C, H, W, P, N, K, precision="bf16")
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    np.testing.assert_array_equal(host(idx), np.tile(np.arange(K), (N, 1)))
    assert np.all(host(dist) == 0)
    st = plan.read_stats()
    assert st["rematch_keys"] == N
    if n_cand <= 32768:
        assert st["regather_keys"] == N and st["overflow_keys"] == 0
    else:
        assert st["overflow_keys"] == N


def _gap_iterate(wl):
    inst = synth.make_instance(wl)
    m = inst["mask"]
    y = ops.cacti_forward(inst["x_true"].astype(np.float64), m)
    R = ops.cacti_mask_sum(m)
    x0 = ops.cacti_adjoint(y / np.where(R == 0, 1, R), m)
    xb = ops.gap_update(x0, y, lambda v: ops.cacti_forward(v, m),
                        lambda r: ops.cacti_adjoint(r, m), R)
    return xb.astype(np.float32), m


def test_bf16_cacti_1024_full_size_sampled_keys():
    # the 1024 x 1024 x 24-frame workload at its real size, in the launch
    # configuration of the timed run: all 16384 keys against all 1017^2
    # candidates; sampled keys checked one by one against the oracle's
    # direct-sum distance map; the whole prior step must equal the FP32
    # form's bitwise (same groups => same low-rank step and aggregation)
    require_gpu()
    wl = synth.WORKLOADS["cacti_1024"]
    x, m = _gap_iterate(wl)
    print("cacti_1024 instance ready", flush=True)
    mg = gpu(m)
    pb = glr.Plan("cacti", wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, mask=mg, precision="bf16")
    xg = gpu(x)
    keys = host(pb.detect_keys(xg))
    idx, dist = pb.match_topk(xg, gpu(keys))
    idx, dist = host(idx), host(dist)
    st = pb.read_stats()
    print("bf16 margins mean", st["margin_sum"] / wl.n_keys, "max", st["margin_max"],
          "overflow", st["overflow_keys"], flush=True)
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(17)
    for a in sorted(rng.choice(wl.n_keys, size=4, replace=False).tolist()):
        ref_idx, ref_d, nxt = om.topk_one(x64, wl.patch, int(keys[a]), wl.k)
        if not np.array_equal(idx[a], ref_idx):
            # only a numerical tie at the group boundary may differ
            dmap = om.distance_map(x64, wl.patch, int(keys[a]))
            scale = float(ref_d.max())
            assert np.abs(np.sort(dmap[idx[a]]) - ref_d).max() <= 1e-9 * scale, a
        np.testing.assert_allclose(dist[a], ref_d, rtol=1e-6, atol=1e-30)
        print("key", a, "ok", flush=True)
    sigma = float(synth.sigma_schedule(wl)[0])
    out_b = host(pb.prior_step(xg, sigma))
    del pb
    pf = glr.Plan("cacti", wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, mask=mg, precision="fp32")
    out_f = host(pf.prior_step(xg, sigma))
    np.testing.assert_array_equal(out_b, out_f)
    assert np.isfinite(out_b).all()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_large_margin_path_periodic_image(precision):
    # a texture of period 4 makes every patch recur ~1500 times at distance 0:
    # the margin sets exceed the wave buffer and take the global-memory path
    # (radix selection on (distance, low part, position)); ties resolve to the
    # lowest positions, exactly as the oracle orders them
    require_gpu()
    C, H, W, P, N, K = 2, 128, 192, 4, 20, 32
    tile = np.random.default_rng(4).uniform(size=(C, 4, 4)).astype(np.float32)
    x = np.tile(tile, (1, H // 4, W // 4))
    n_cand = (H - P + 1) * (W - P + 1)
    keys = np.sort(np.random.default_rng(8).choice(n_cand, size=N, replace=False))
    plan = _plan(C, H, W, P, N, K, precision=precision)
    idx, dist = plan.match_topk(gpu(x), gpu(keys.astype(np.int32)))
    st = plan.read_stats()
    print("margin max", st["margin_max"], "overflow", st["overflow_keys"],
          "rematch", st["rematch_keys"], flush=True)
    ref_idx, ref_dist = om.topk_exact(x.astype(np.float64), P, keys, K)
    np.testing.assert_array_equal(host(idx), ref_idx)
    np.testing.assert_array_equal(host(dist), 0.0)
    assert st["margin_max"] > 1024 and st["overflow_keys"] == 0
