"""The paper's own matching score: correlation of binary edge maps (oracle).

Method section, eq. 6-8.  The image is reduced to binary maps of its
horizontal and vertical Sobel gradients; each exemplar's edge patches are the
kernels of a cross-correlation ("Conv2d") with those maps, and the four heat
maps are summed; a larger value means a more similar patch.

Readings taken (the paper prints no constants):
- edge maps are taken per real channel of the quantised image the detector
  uses (q_c = clamp(rint(255 x_c)) in IEEE FP32 for real data; for complex
  data the single quantised squared-magnitude image), with the detector's
  integer Sobel (replicate borders): gx along columns (horizontal, nabla_h),
  gy along rows (nabla_v);
- eq. 6 as printed gives identical "+" and "-" maps (abs(-g) = abs(g)); the
  reading is rising and falling edges: E_h^+ = [gx > th], E_h^- = [-gx > th],
  E_v^+ = [gy > th], E_v^- = [-gy > th] (eq. 7's T);
- th = ceil(max over channels and pixels of max(|gx|, |gy|) / 10), an
  integer, per prior step (th = 0 on a flat image, which has no edges);
- the heat value of key g and candidate j is
  H = sum over the 4 maps, channels and patch offsets of E[key] E[cand],
  an integer; the group is the K candidates of largest H, the lowest
  position winning ties.
"""
import numpy as np

from .detector import quantise_real, quantise_complex, sobel, _F255


def quantised_channels(x, is_complex=False):
    """u8 channel images [C][H][W] of a real iterate (before the detector's
    channel average), or the single detection image of a complex one
    ([1][H][W]; None when it is identically zero)."""
    x32 = np.asarray(x, dtype=np.float32)
    if is_complex:
        q = quantise_complex(x32[0], x32[1])
        return None if q is None else q[None]
    return np.clip(np.rint(_F255 * x32), np.float32(0), np.float32(255)).astype(np.int64)


def edge_maps(x, is_complex=False):
    """The binary maps of eq. 6-7 as an int64 stack [4 C][H][W], ordered
    (h+, h-, v+, v-) per channel: map 4c + m."""
    q = quantised_channels(x, is_complex)
    _, H, W = np.asarray(x).shape
    if q is None:
        return np.zeros((4, H, W), dtype=np.int64)
    grads = [sobel(qc) for qc in q]
    gmax = max(int(max(np.abs(gx).max(), np.abs(gy).max())) for gx, gy in grads)
    th = (gmax + 9) // 10
    out = []
    for gx, gy in grads:
        out += [gx > th, -gx > th, gy > th, -gy > th]
    return np.stack(out).astype(np.int64)


def heat_map_rows(E, patch, keys):
    """Heat values [N][N_cand] of eq. 8: H[g][j] = <e_g, e_j> over the edge
    patch vectors of the stacked maps (exact integers)."""
    from .matching import patch_matrix
    pm = patch_matrix(E.astype(np.float64), patch)          # 0/1 rows: exact dot products
    return pm[np.asarray(keys)] @ pm.T


def topk_edge(x, patch, keys, K, is_complex=False):
    """Groups by the edge heat map: the K candidates of largest H, lowest
    position first among equal values.  Returns (idx int64 [N][K], H [N][K])."""
    E = edge_maps(x, is_complex)
    Hm = heat_map_rows(E, patch, keys)
    n = Hm.shape[1]
    j = np.arange(n)
    idx = np.empty((len(keys), K), dtype=np.int64)
    val = np.empty((len(keys), K))
    for a in range(len(keys)):
        order = np.lexsort((j, -Hm[a]))[:K]
        idx[a] = order
        val[a] = Hm[a][order]
    return idx, val
