"""The certified error bounds of the matcher's distances, checked on the CPU.

The top-K pass keeps every candidate whose distance d~ (computed by the
matcher in FP32 or BF16 arithmetic) could be within its error bound eps of
the K-th smallest; groups are exact only if |d~ - d| <= eps always holds.
These tests emulate the kernels' arithmetic step by step in numpy float32
(sequential sums, one of the orders the bound allows; BF16 rounding by this
file's own round-to-nearest-even) and compare |d~ - d| with eps against the
exact distance (rational arithmetic), on worst-case and random inputs:

- BF16 form (one mean per patch): a = fl(k - mu_k), pbar = fl(p - mu_p),
  e_a = a - bf16(a), e_p = pbar - bf16(pbar) (exact residuals),
  S = sum bf16(a) bf16(pbar), d~ = ((|a|^2 + |pbar|^2) - 2 S + (D dmu) dmu)
  + 2 dmu (sum a - sum pbar), eps = c2 R^2 + c1 (|a| |e_p| + |e_a| (|pbar|
  + |e_p|)) with R = |a| + |pbar| + sqrt(D) |dmu|, c1 = 2 (1 + 2^-8),
  c2 = (3 D + 26) u.  The residual term is a direct Cauchy-Schwarz bound of
  <a, pbar> - <bf16(a), bf16(pbar)> = <a, e_p> + <e_a, bf16(pbar)>, with no
  slack beyond the FP32 roundings of its norms: the worst case attains it,
  and |d~ - d| <= eps is the test; the FP32 sums' term c2 R^2 keeps a
  factor two.
- FP32 form (every channel centred on its own mean): d~ = fma(-2, S,
  |a~|^2 + |p~|^2) + sum_c (fl(P mu_kc) - fl(P mu_pc))^2, eps =
  y (c2 y + w) + w^2 with y = |a~| + |p~| + sqrt(max(d~, 0)) + w,
  w = 8.02 P u (h_k + h_p), c2 = 2.02 (D + C + 4) u.
"""
import math
from fractions import Fraction

import numpy as np

f32 = np.float32
U = 2.0 ** -24


def _up(v):
    """The float32 at or above v (the library rounds its coefficients up)."""
    return np.nextafter(f32(v), f32(np.inf), dtype=f32)


def bf16(x):
    """Round float32 values to BF16 (8 significant bits), nearest even, via
    float64 scaling (independent of any bit trick)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    e = np.floor(np.log2(np.abs(x[nz])))
    q = np.exp2(e - 7)
    out[nz] = np.rint(x[nz] / q) * q
    return out.astype(f32)


def fma(a, b, c):
    """float32 fma: the product is exact in float64, then one rounding of the
    sum in float64 and one to float32 (a double rounding that only moves a
    tie, far below the bound's slack)."""
    return (np.float64(1.0) * np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(f32)


def seq_sum(terms):
    """Sequential float32 sum over the first axis."""
    acc = np.zeros(terms.shape[1:], dtype=f32)
    for t in terms:
        acc = f32(acc + t)
    return acc


def seq_fma_sq(vals):
    """Sequential float32 sum of squares with fused multiply-add (one rounding
    per step, emulated in float64 where a*a + acc is exact)."""
    acc = np.zeros(vals.shape[1:], dtype=f32)
    for v in vals:
        acc = (v.astype(np.float64) * v.astype(np.float64) + acc.astype(np.float64)).astype(f32)
    return acc


def exact_d(k, p):
    """Exact squared distance of float32 patches as a float (rational sum)."""
    s = Fraction(0)
    for a, b in zip(k.tolist(), p.tolist()):
        t = Fraction(a) - Fraction(b)
        s += t * t
    return float(s)


def bf16_form(k, P, key_residual=True):
    """d~ and eps of the BF16 form for key k [D] and candidates P [n][D]
    (key_residual=False drops the key's residual term, a plausible mistake
    the worst case must expose)."""
    D = k.shape[0]
    k = k.astype(f32)
    P = P.astype(f32)
    mu_k = f32(seq_sum(k[:, None])[0] / f32(D))
    a = f32(k - mu_k)
    an = seq_fma_sq(a[:, None])[0]
    sa = seq_sum(a[:, None])[0]
    kr = f32(np.sqrt(an))
    mu_p = f32(seq_sum(P.T) / f32(D))
    pb = f32(P - mu_p[:, None])
    pn = seq_fma_sq(pb.T)
    sp = seq_sum(pb.T)
    pr = f32(np.sqrt(pn))
    # BF16 products are exact in FP32; FP32 accumulation
    S = seq_sum((bf16(a)[None, :].astype(np.float64) * bf16(pb).astype(np.float64))
                .astype(f32).T)
    dmu = f32(mu_k - mu_p)
    base = f32(f32(an + pn) - f32(f32(2) * S))
    dt = f32(f32(base + f32(f32(f32(D) * dmu) * dmu)) + f32(f32(f32(2) * dmu) * f32(sa - sp)))
    # residual norms of the BF16 operands, summed as the metadata kernels do
    ek = f32(np.sqrt(seq_fma_sq(f32(a - bf16(a))[:, None])[0]))
    ep = f32(np.sqrt(seq_fma_sq(f32(pb - bf16(pb)).T)))
    if not key_residual:
        ek = f32(0)
    c1 = _up(2.0 * (1.0 + 2.0 ** -8))
    c2 = _up((3.0 * D + 26.0) * U)
    cz = _up(math.sqrt(D))
    # the kernel's order: R = fma(cz, |dmu|, kr + pr),
    # eps = fma(c2 R, R, c1 fma(ek, pr + ep, kr ep))
    R = fma(cz, np.abs(f32(mu_k - mu_p)), f32(kr + pr))
    res = fma(ek, f32(pr + ep), f32(kr * ep))
    eps = fma(f32(c2 * R), R, f32(c1 * res))
    return dt, eps


def fp32_form(k, P, C, psz):
    """d~ and eps of the channel-centred FP32 form (C channels of psz^2)."""
    n = psz * psz
    D = C * n
    k = k.astype(f32).reshape(C, n)
    P = P.astype(f32).reshape(-1, C, n)
    # key: channel means from FP64 sums, correctly rounded
    mu_k = (k.astype(np.float64).sum(1) / n).astype(f32)
    a = f32(k - mu_k[:, None]).reshape(D)
    an = seq_fma_sq(a[:, None])[0]
    hk = f32(0)
    for c in range(C):
        ma = f32(np.abs(k[c].astype(np.float64)).sum() / n)
        hk = f32(np.float64(ma) * ma + np.float64(hk))
    h_k = f32(np.sqrt(hk))
    kr = f32(np.sqrt(an))
    kc = f32(f32(psz) * mu_k)
    mu_p = (P.astype(np.float64).sum(2) / n).astype(f32)             # [n][C]
    pt = f32(P - mu_p[:, :, None]).reshape(-1, D)
    pn = seq_fma_sq(pt.T)
    hp = np.zeros(P.shape[0], dtype=f32)
    for c in range(C):
        ma = (np.abs(P[:, c].astype(np.float64)).sum(1) / n).astype(f32)
        hp = (ma.astype(np.float64) * ma + hp.astype(np.float64)).astype(f32)
    h_p = f32(np.sqrt(hp))
    pr = f32(np.sqrt(pn))
    pcs = f32(f32(psz) * mu_p)
    # FP32 products rounded, FP32 accumulation
    S = seq_sum(f32(a[None, :] * pt).T)
    v = (np.float64(-2.0) * S + f32(an + pn)).astype(f32)               # fma(-2, S, .)
    for c in range(C):
        d = f32(kc[c] - pcs[:, c])
        v = (d.astype(np.float64) * d + v.astype(np.float64)).astype(f32)
    coef2 = _up(2.02 * (D + C + 4.0) * U)
    cz = _up(8.02 * psz * U)
    w = f32(cz * f32(h_k + h_p))
    y = f32(f32(f32(kr + pr) + f32(np.sqrt(np.maximum(v, f32(2.0 ** -126))))) + w)
    inner = (coef2.astype(np.float64) * y + w).astype(f32)
    eps = (y.astype(np.float64) * inner + f32(w * w)).astype(f32)
    return v, eps


def _ratio(dt, eps, k, P):
    """max |d~ - d| / eps over the candidates (a zero eps needs d~ == d)."""
    r = 0.0
    for j in range(P.shape[0]):
        d = exact_d(k, P[j])
        if float(eps[j]) == 0.0:
            assert float(dt[j]) == d
            continue
        r = max(r, abs(float(dt[j]) - d) / float(eps[j]))
    return r


def test_bf16_worst_case_small_d():
    # a = pbar = +-v with v just below a BF16 half-way point, signs aligned:
    # both operands lose ~2^-8 relative in the same direction, the residuals
    # are parallel to the operands, the exact distance is 0 and the error
    # sits at the Cauchy-Schwarz bound
    v = f32(1.0 + 2.0 ** -8 - 2.0 ** -20)
    assert bf16(np.array([v]))[0] == f32(1.0)
    for D in (2, 4, 8, 16, 1536):
        k = np.array([v, -v] * (D // 2), dtype=f32)
        P = np.stack([k, 4 * k, k / 8])
        dt, eps = bf16_form(k, P[:1])
        r = _ratio(dt, eps, k, P[:1])
        assert 0.9 < r <= 1.0, (D, r)           # tight: the bound is attained
        dt, eps = bf16_form(k, P)
        assert _ratio(dt, eps, k, P) <= 1.0


def test_bf16_bound_without_the_key_residual_fails():
    # the same worst case exceeds a bound that keeps only |a| |e_p|
    v = f32(1.0 + 2.0 ** -8 - 2.0 ** -20)
    D = 8
    k = np.array([v, -v] * (D // 2), dtype=f32)
    dt, eps = bf16_form(k, k[None], key_residual=False)
    assert abs(float(dt[0])) > float(eps[0])


def test_bf16_random_patches():
    rng = np.random.default_rng(7)
    for D, n in ((2, 64), (18, 64), (288, 48), (1536, 24)):
        for scale, level in ((1.0, 0.0), (0.05, 0.5), (1.0, 1000.0), (0.01, 1000.0)):
            k = f32(level + scale * rng.uniform(size=D))
            near = f32(k[None] + scale * 1e-3 * rng.standard_normal((n // 2, D)))
            far = f32(level + scale * rng.uniform(size=(n - n // 2, D)))
            P = np.concatenate([near, far])
            dt, eps = bf16_form(k, P)
            r = _ratio(dt, eps, k, P)
            assert r <= 1.0, (D, scale, level, r)
            # with many elements random rounding errors do not align (at
            # D = 2 a centred patch is +-v, its residual parallel to it)
            if D >= 288:
                assert r <= 0.5, (D, scale, level, r)


def test_bf16_residual_bound_is_tighter_than_the_worst_case_rounding():
    # on random centred patches the residual norms are ~2^-9.7 of the
    # operand norms (RMS relative error of BF16 rounding), so the BF16 term
    # is several times below the worst-case 4 (2 b + b^2) |a| |pbar|, b = 2^-8
    rng = np.random.default_rng(11)
    D = 1536
    k = f32(0.3 + 0.05 * rng.standard_normal(D))
    P = f32(0.3 + 0.05 * rng.standard_normal((16, D)))
    a = f32(k - f32(k.mean()))
    pb = f32(P - P.mean(1, keepdims=True).astype(f32))
    ra = np.linalg.norm(a - bf16(a)) / np.linalg.norm(a)
    rp = np.linalg.norm(pb - bf16(pb), axis=1) / np.linalg.norm(pb, axis=1)
    new = 2 * (1 + 2.0 ** -8) * (rp + ra * (1 + rp))
    old = 4 * (2 * 2.0 ** -8 + 2.0 ** -16)
    assert np.all(new < old / 4), (new.max(), old)


def test_fp32_channel_centred_random_and_offsets():
    rng = np.random.default_rng(8)
    cases = [(2, 6, 1.0, 0.0, 0.01), (16, 6, 1.0, 0.5, 0.02), (24, 8, 1.0, 1000.0, 0.01),
             (64, 1, 1.0, 0.0, 1.0), (4, 3, 1.0, 0.0, 1.0)]
    for C, psz, _, level, tex in cases:
        n = psz * psz
        levels = level + rng.uniform(size=C) if level else 10.0 ** rng.uniform(-3, 3, size=C)
        k = f32(np.repeat(levels, n) * (1 + tex * rng.standard_normal(C * n)))
        near = f32(k[None] * (1 + 1e-4 * rng.standard_normal((16, C * n))))
        far = f32(np.repeat(levels, n)[None] * (1 + tex * rng.standard_normal((16, C * n))))
        P = np.concatenate([k[None], near, far])
        dt, eps = fp32_form(k, P, C, psz)
        assert _ratio(dt, eps, k, P) <= 0.5, (C, psz, level)


def test_fp32_half_way_subtractions():
    # values one half-ulp off the channel mean's grid, signs aligned: the
    # centring subtractions all round the same way
    C, psz = 8, 4
    n = psz * psz
    base = f32(3.0)
    ulp = np.spacing(base)
    k = np.full(C * n, base, dtype=f32)
    k[::2] = f32(base + 0.5 * ulp * 3)
    k[1::2] = f32(base - 0.5 * ulp * 3)
    P = np.stack([k, f32(k + ulp), f32(k * 1.0001), np.roll(k, 1)])
    dt, eps = fp32_form(k, P, C, psz)
    assert _ratio(dt, eps, k, P) <= 0.5
