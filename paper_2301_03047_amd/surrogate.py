"""Training data and training loop for the CNN surrogate.

The network learns the GLR prior step itself: each training pair is a
pre-prior slice and the GLR step's output on it, at that iteration's noise
level, captured from plain GLR runs (every step runs in the library's
kernels; this module only indexes device tensors).
"""
import numpy as np
import torch

from .glr import Plan, Cnn

MRI = 1


def glr_pairs(plan: Plan, y, iters=None):
    """Run the plain GLR loop of ``plan`` on measurement ``y`` and return, per
    iteration, (pre-prior slices [S][H][W], post-prior slices, sigma_t):
    S = C frames/bands, or the real and imaginary planes for MRI."""
    T = plan.iters if iters is None else iters
    H, W = plan.H, plan.W
    state = plan.new_state()
    plan.reconstruct(y, 0, 0, state=state)              # initial estimate only
    out = []
    for t in range(T):
        pre = plan.pre_prior(y, state)                  # what iteration t's prior receives
        plan.reconstruct(y, t, t + 1, state=state)
        if plan.modality == MRI:
            z = state[: 3 * H * W * 8].view(torch.complex64)[H * W:2 * H * W].view(H, W)
            pre = torch.stack([pre.real, pre.imag]).contiguous()
            post = torch.stack([z.real, z.imag]).contiguous()
        else:
            post = state[: plan.C * H * W * 4].view(torch.float32).view(plan.C, H, W).clone()
        out.append((pre, post, float(plan._sigma[t])))
    return out


def random_crops(pairs, n, size, seed):
    """n random size x size crops of random slices of random iterations:
    (x [n][size][size], target, sigma [n]) on the pairs' device."""
    rng = np.random.default_rng(seed)
    xs, ts, ss = [], [], []
    for _ in range(n):
        pre, post, sig = pairs[rng.integers(len(pairs))]
        s = int(rng.integers(pre.shape[0]))
        r = int(rng.integers(pre.shape[1] - size + 1))
        c = int(rng.integers(pre.shape[2] - size + 1))
        xs.append(pre[s, r:r + size, c:c + size])
        ts.append(post[s, r:r + size, c:c + size])
        ss.append(sig)
    dev = pairs[0][0].device
    return (torch.stack(xs).contiguous(), torch.stack(ts).contiguous(),
            torch.tensor(ss, dtype=torch.float32, device=dev))


def train(cnn: Cnn, data, steps, batch, lr, seed=0, log_every=0):
    """Adam on random mini-batches of ``data`` = (x, target, sigma); returns
    the per-step losses (host floats, read once at the end)."""
    x, tgt, sig = data
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for i in range(steps):
        sel = torch.randint(0, x.shape[0], (batch,), generator=g).to(x.device)
        loss = cnn.train_step(x[sel].contiguous(), sig[sel].contiguous(),
                              tgt[sel].contiguous(), lr)
        losses.append(loss)
        if log_every and (i + 1) % log_every == 0:
            print(f"  step {i + 1}: loss {float(loss):.3e}", flush=True)
    return [float(v) for v in torch.cat(losses).cpu()]


def eval_loss(cnn: Cnn, data, batch=64):
    """Mean loss of the surrogate estimate over ``data`` (no update)."""
    x, tgt, sig = data
    tot, n = 0.0, 0
    for i in range(0, x.shape[0], batch):
        out = cnn.forward(x[i:i + batch].contiguous(), sig[i:i + batch].contiguous())
        tot += float(((out - tgt[i:i + batch]) ** 2).sum())
        n += out.numel()
    return tot / n


def psnr(est, ref):
    """PSNR in dB: peak 1 for real images; for complex images on the
    magnitude with peak max |ref| (host arrays)."""
    est, ref = np.asarray(est), np.asarray(ref)
    peak = 1.0
    if np.iscomplexobj(est) or np.iscomplexobj(ref):
        est, ref = np.abs(est), np.abs(ref)
        peak = float(ref.max())
    mse = float(np.mean((est.astype(np.float64) - ref.astype(np.float64)) ** 2))
    return float(10.0 * np.log10(peak * peak / mse)) if mse > 0 else float("inf")
