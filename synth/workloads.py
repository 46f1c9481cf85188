"""Workload definitions (shapes, counts, seeds, frozen constants).

Each entry mirrors one synthetic stand-in for the paper's experiments:
compressive temporal imaging (CACTI, eq. 2), single-coil MRI (eq. 3) and
multispectral filter-array demosaicing (eq. 4-5).  The constants the paper
leaves open (noise schedule, WNNM constant, ADMM penalty) are frozen here and
read identically by the oracle and by the HIP path.
"""
from dataclasses import dataclass, replace
import numpy as np

from .scenes import cacti_video, mri_phantom, msfa_cube
from .masks import cacti_masks, mri_line_mask


@dataclass(frozen=True)
class Workload:
    name: str
    modality: str          # "cacti" | "mri" | "msfa"
    H: int
    W: int
    C: int                 # frames (cacti), bands (msfa), 1 (mri, complex)
    patch: int             # patch side P
    n_keys: int            # number of key (exemplar) patches N
    k: int                 # group size K
    iters: int             # outer iterations T
    sigma0: float          # noise level at the first iteration
    sigma1: float          # noise level at the last iteration
    wnnm_c: float = 2.0 * np.sqrt(2.0)
    wnnm_eps: float = 1e-16
    rho: float = 1.0       # ADMM penalty (mri)
    precision: str = "fp32"
    seed: int = 0          # scene seed; the mask seed is seed + 1
    # exemplar selection ("corner", "uniform", "corner_uniform"; uniform grid
    # interval, three times it for corner_uniform) and search region
    # ("global", or a local "window" of half width `window`)
    exemplars: str = "corner"
    uniform_step: int = 4
    search: str = "global"
    window: int = 20
    gap_acc: bool = False  # accelerated GAP (measurement residual accumulated)
    score: str = "l2"      # matching score: "l2" distance or the "edge"-map correlation
    agg_weights: str = "uniform"   # aggregation: "uniform", or "rank" (1 / kept rank per group)
    # inner WNNM iterations per prior step (iterative regularisation step
    # delta, noise re-estimate factor lambda)
    wnnm_iters: int = 1
    wnnm_delta: float = 0.1
    wnnm_lambda: float = 0.54
    # complex data: groups shrunk as real-stacked [Re; Im] ("stacked") or as
    # complex matrices ("complex")
    lowrank: str = "stacked"

    @property
    def real_channels(self):
        return 2 if self.modality == "mri" else self.C

    @property
    def n_cand(self):
        return (self.H - self.patch + 1) * (self.W - self.patch + 1)

    @property
    def dim(self):
        return self.real_channels * self.patch * self.patch

    @property
    def keys_total(self):
        """Exemplars per prior step: n_keys corners, the uniform grid, or both."""
        Hc, Wc = self.H - self.patch + 1, self.W - self.patch + 1

        def grid(s):
            return (-(-Hc // s)) * (-(-Wc // s))
        if self.exemplars == "uniform":
            return grid(self.uniform_step)
        if self.exemplars == "corner_uniform":
            return self.n_keys + grid(3 * self.uniform_step)
        return self.n_keys


# Noise schedules: the first level is of the order of the initial estimate's
# artefacts (mask modulation for CACTI, mosaic replication for MSFA, k-space
# undersampling for MRI), decaying geometrically to the last.
WORKLOADS = {
    "cacti_128": Workload("cacti_128", "cacti", 128, 128, 8, 6, 128, 32, 5, 1.0, 0.05, seed=0),
    "mri_256": Workload("mri_256", "mri", 256, 256, 1, 6, 1024, 45, 30, 0.05, 0.01, seed=1000),
    "msfa_512": Workload("msfa_512", "msfa", 512, 512, 16, 6, 4096, 64, 40, 0.5, 0.05, seed=2000),
    # evaluation instances of the CNN surrogate: the 128 x 128 CACTI generator
    # at 512 x 512 (keys scaled with the area), 20 iterations
    "cacti_512": Workload("cacti_512", "cacti", 512, 512, 8, 6, 2048, 32, 20, 1.0, 0.05,
                          seed=4200),
    "cacti_1024": Workload("cacti_1024", "cacti", 1024, 1024, 24, 8, 16384, 64, 50, 1.0, 0.05,
                           precision="bf16", seed=3000),
    # the paper's CACTI shape (8 frames of 256 x 256) for the matching
    # ablation: global matching from corner exemplars against block matching
    # in a 41 x 41 window from a uniform grid (interval 4), from corners, and
    # from corners plus a grid of three times the interval
    "cacti_256": Workload("cacti_256", "cacti", 256, 256, 8, 6, 512, 32, 20, 1.0, 0.05,
                          seed=5000),
}


ABLATION = {
    "gm_corner": dict(exemplars="corner", search="global"),
    "gm_corner_edge": dict(exemplars="corner", search="global", score="edge"),
    "bm_uniform": dict(exemplars="uniform", search="window"),
    "bm_corner": dict(exemplars="corner", search="window"),
    "bm_corner_uniform": dict(exemplars="corner_uniform", search="window"),
}


def small(wl, **kw):
    """A copy of ``wl`` with some fields replaced (for reduced test shapes)."""
    return replace(wl, **kw)


def sigma_schedule(wl):
    """Geometric decay sigma0 -> sigma1 over ``iters`` iterations (float32)."""
    T = wl.iters
    if T == 1:
        return np.array([wl.sigma0], dtype=np.float32)
    t = np.arange(T, dtype=np.float64) / (T - 1)
    return (wl.sigma0 * (wl.sigma1 / wl.sigma0) ** t).astype(np.float32)


def make_instance(wl):
    """Ground truth and masks for ``wl``.

    Returns a dict with ``x_true`` (float32 ``[C][H][W]``, or complex64
    ``[H][W]`` for mri) and ``mask`` (uint8: cacti ``[C][H][W]``, mri ``[H]``
    line mask, msfa ``None`` - its filter pattern is fixed by the operator).
    """
    if wl.modality == "cacti":
        x = cacti_video(wl.C, wl.H, wl.W, wl.seed)
        m = cacti_masks(wl.C, wl.H, wl.W, wl.seed + 1)
    elif wl.modality == "mri":
        x = mri_phantom(wl.H, wl.W, wl.seed)
        m = mri_line_mask(wl.H, wl.seed + 1)
    elif wl.modality == "msfa":
        x = msfa_cube(wl.C, wl.H, wl.W, wl.seed)
        m = None
    else:
        raise ValueError(wl.modality)
    return {"x_true": np.ascontiguousarray(x), "mask": m}


def random_image(C, H, W, seed, kind="smooth"):
    """A generic seeded test image ``[C][H][W]`` float32 in [0, 1].

    ``kind``: "uniform" (i.i.d. U[0,1]), "smooth" (smoothed noise with a few
    edges), "dup" (tiles repeated so exact duplicate patches exist)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(size=(C, H, W)).astype(np.float32)
    if kind == "dup":
        th, tw = max(2, H // 3), max(2, W // 3)
        tile = rng.uniform(size=(C, th, tw))
        reps = (1, -(-H // th), -(-W // tw))
        return np.tile(tile, reps)[:, :H, :W].astype(np.float32)
    from scipy import ndimage
    z = ndimage.gaussian_filter(rng.standard_normal((C, H, W)), sigma=(0, 1.5, 1.5))
    z = (z - z.min()) / max(z.max() - z.min(), 1e-12)
    step = (np.arange(W)[None, None, :] > W // 2) * 0.3
    return np.clip(0.6 * z + step, 0.0, 1.0).astype(np.float32)
