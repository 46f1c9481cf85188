"""Evaluation of the CNN surrogate form: train the network on (pre-prior,
GLR output) crops captured from one plain run of the 256 x 256 MRI problem
and one of the 1024 x 1024 x 24 CACTI problem, then reconstruct a batch of
16 MRI (256 x 256) and 16 CACTI (512 x 512 x 8) held-out instances three
ways: plain GLR, surrogate with the GLR judge, surrogate only.  Prints
progress lines and returns a dict of wall times and PSNRs.
"""
import time

import numpy as np
import torch

from .glr import Plan, Cnn
from . import surrogate as sg


def _instance(synth, name, seed):
    wl = synth.workloads.small(synth.WORKLOADS[name], seed=seed)
    inst = synth.make_instance(wl)
    m = torch.from_numpy(inst["mask"]).cuda() if inst["mask"] is not None else None
    sig = synth.sigma_schedule(wl)

    def mk(**kw):
        return Plan(wl.modality, wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, iters=wl.iters,
                    sigma=sig, mask=m, precision=wl.precision, **kw)
    plan = mk()
    y = plan.forward(torch.from_numpy(inst["x_true"]).cuda())
    return wl, inst, y, mk, plan


def run(train_steps=3000, n_crops=20000, crop=128, n_eval=16, delta_max=0.02, log=print):
    import synth
    from synth.cnn import cnn_params
    t0 = time.time()
    pairs = []
    for name, seed in (("mri_256", 1000), ("cacti_1024", 3000)):
        _, _, y, _, plan = _instance(synth, name, seed)
        pairs += sg.glr_pairs(plan, y)
        del plan
        log(f"captured GLR pairs from {name}: {len(pairs)} iterations so far "
            f"({time.time() - t0:.0f} s)")
    crops = sg.random_crops(pairs, n_crops, crop, seed=4000)
    del pairs
    n_val = n_crops // 10
    val = tuple(c[:n_val] for c in crops)
    train = tuple(c[n_val:] for c in crops)
    net = Cnn(cnn_params(4000))
    l0 = sg.eval_loss(net, val)
    torch.cuda.synchronize()
    t1 = time.time()
    sg.train(net, train, train_steps, 32, 1e-3, seed=4000)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    l1 = sg.eval_loss(net, val)
    ident = float(((val[0] - val[1]) ** 2).mean())
    log(f"trained {train_steps} steps in {t_train:.1f} s: validation loss {l0:.3e} -> {l1:.3e} "
        f"(identity {ident:.3e})")
    variants = {"plain": {}, "surrogate+judge": {"cnn": net, "judge_delta_max": delta_max},
                "surrogate-only": {"cnn": net, "judge_delta_max": float("inf")}}
    res = {v: {"seconds": 0.0, "psnr": [], "surrogate_steps": 0, "fallbacks": 0}
           for v in variants}
    for name, seed0 in (("mri_256", 4100), ("cacti_512", 4200)):
        for i in range(n_eval):
            wl, inst, y, mk, _ = _instance(synth, name, seed0 + i)
            for v, kw in variants.items():
                p = mk(**kw)
                if i == 0:
                    p.reconstruct(y)                      # warm-up per shape
                    p.read_stats(reset=True)
                torch.cuda.synchronize()
                t = time.perf_counter()
                out, _ = p.reconstruct(y)
                torch.cuda.synchronize()
                r = res[v]
                r["seconds"] += time.perf_counter() - t
                r["psnr"].append(sg.psnr(out.cpu().numpy(), inst["x_true"]))
                st = p.read_stats()
                r["surrogate_steps"] += st["surrogate_steps"]
                r["fallbacks"] += st["fallback_steps"]
        log(f"evaluated {n_eval} {name} instances ({time.time() - t0:.0f} s)")
    out = {"train_steps": train_steps, "train_seconds": round(t_train, 2),
           "val_loss": {"untrained": l0, "trained": l1, "identity": ident},
           "judge_delta_max": delta_max, "variants": {}}
    for v, r in res.items():
        ps = np.array(r["psnr"])
        out["variants"][v] = {"seconds": round(r["seconds"], 3),
                              "psnr_mri_db": round(float(ps[:n_eval].mean()), 3),
                              "psnr_cacti_db": round(float(ps[n_eval:].mean()), 3),
                              "surrogate_steps": r["surrogate_steps"],
                              "fallbacks": r["fallbacks"]}
    base = out["variants"]["plain"]["seconds"]
    for v in out["variants"].values():
        v["speedup_vs_plain"] = round(base / v["seconds"], 3)
    return out
