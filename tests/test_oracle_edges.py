"""Pins for the oracle's edge-map matching score (eq. 6-8): hand-worked
edge maps of a step and a ramp, the heat map against explicit correlation
loops, self-correlation, and the tie rule."""
import numpy as np

import synth
from oracle import edges as oe


def test_step_edge_maps_by_hand():
    # a rising step between columns 4 and 5 of a 9 x 10 image: gx = 4 * 255 at
    # columns 4 and 5 (replicate borders), th = ceil(1020 / 10) = 102
    x = np.zeros((1, 9, 10), dtype=np.float32)
    x[0, :, 5:] = 1.0
    E = oe.edge_maps(x)
    assert E.shape == (4, 9, 10)
    want = np.zeros((9, 10), dtype=np.int64)
    want[:, 4:6] = 1
    np.testing.assert_array_equal(E[0], want)      # h+
    assert E[1].sum() == 0 and E[2].sum() == 0 and E[3].sum() == 0
    # the falling step gives the h- map
    Ef = oe.edge_maps(1.0 - x)
    np.testing.assert_array_equal(Ef[1], want)
    assert Ef[0].sum() == 0


def test_vertical_ramp_is_a_rising_v_edge():
    # values growing down the rows: gy > 0 everywhere inside (v+), gx = 0
    x = (np.arange(12, dtype=np.float32)[:, None] / 11.0 * np.ones((1, 12, 8), np.float32))
    E = oe.edge_maps(x)
    assert E[2].sum() > 0 and E[3].sum() == 0 and E[0].sum() == 0 and E[1].sum() == 0


def test_threshold_is_a_tenth_of_the_largest_gradient():
    # quantised rows 0 | 26 (col 3) | 255 (col 10) | 232 (col 15) | 208 (col 17):
    # the largest |gx| is 4 * 229 = 916, th = ceil(91.6) = 92; the step of 26
    # (gx = 104) is a rising edge, the fall of 23 (-gx = 92) is not, the fall
    # of 24 (-gx = 96) is
    q = np.zeros(20)
    q[3:] = 26
    q[10:] = 255
    q[15:] = 232
    q[17:] = 208
    x = np.tile((q / 255.0).astype(np.float32), (1, 7, 1))
    E = oe.edge_maps(x)
    assert np.nonzero(E[0].any(axis=0))[0].tolist() == [2, 3, 9, 10]
    assert np.nonzero(E[1].any(axis=0))[0].tolist() == [16, 17]


def test_heat_map_equals_explicit_correlation():
    x = synth.workloads.random_image(2, 11, 12, seed=4, kind="smooth")
    P = 3
    E = oe.edge_maps(x)
    M, H, W = E.shape
    Hc, Wc = H - P + 1, W - P + 1
    keys = [0, 7, 33, 60, Hc * Wc - 1]
    Hm = oe.heat_map_rows(E, P, keys)
    for a, g in enumerate(keys):
        gr, gc = divmod(g, Wc)
        for j in range(Hc * Wc):
            jr, jc = divmod(j, Wc)
            s = 0
            for m in range(M):
                for dy in range(P):
                    for dx in range(P):
                        s += int(E[m, gr + dy, gc + dx]) * int(E[m, jr + dy, jc + dx])
            assert Hm[a, j] == s
        # self-correlation: the number of edge pixels in the key's patch
        assert Hm[a, g] == int(E[:, gr:gr + P, gc:gc + P].sum())


def test_edge_groups_order_and_ties():
    # a flat image has no edges: every heat value is 0 and the groups are the
    # lowest positions
    x = np.full((2, 12, 12), 0.3, np.float32)
    idx, val = oe.topk_edge(x, 3, [0, 50, 99], 5)
    np.testing.assert_array_equal(idx, np.tile(np.arange(5), (3, 1)))
    assert np.all(val == 0)
    # otherwise values are non-increasing along each group, ties by position
    x = synth.workloads.random_image(3, 20, 22, seed=6, kind="smooth")
    idx, val = oe.topk_edge(x, 4, [5, 77, 200], 12)
    for a in range(3):
        assert np.all(np.diff(val[a]) <= 0)
        for q in range(11):
            if val[a, q] == val[a, q + 1]:
                assert idx[a, q] < idx[a, q + 1]
