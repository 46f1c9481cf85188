#!/usr/bin/env python3
"""Benchmark of the GLR reconstruction hot path on one MI355X.

A step is one outer iteration of the data-fidelity loop: the data step plus
the whole GLR prior step (key detection, global matching, top-K grouping,
WNNM shrinkage, aggregation).  The default workload is the synthetic
single-coil MRI problem (256 x 256 complex64, 6 x 6 patches, 1024 keys,
K = 45, 30 ADMM iterations); ``--workload`` selects another one (the
1024 x 1024 x 24-frame CACTI problem with ``--precision bf16`` is the
precision form at scale).  Inputs are resident in HBM before the timed
region starts.

Prints one JSON line.  ``value`` is timed on a plan without per-stage
events; a second plan with them repeats the same number of iterations from
the same state, and ``roofline`` covers the dominant kernel of that pass
(largest share), with its average launch duration taken from the HIP events
the library records on the launch stream.  ``cpu_baseline`` is the FP64 CPU
oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GLR iterations/sec + matching TFLOP/s (% MFMA peak) at fixed PSNR vs oracle"
WORKLOAD = "mri_256"

# MI355X published peaks
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60, help="timed GLR iterations")
    ap.add_argument("--warmup", type=int, default=30, help="untimed GLR iterations first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the full-length reconstruction that reports PSNR")
    ap.add_argument("--cpu-iters", type=int, default=16, help="oracle iterations in the CPU sample")
    ap.add_argument("--workload", default=WORKLOAD, choices=["mri_256", "cacti_1024", "msfa_512",
                                                              "cacti_128", "surrogate"])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16"],
                    help="matcher precision (default: the workload's own)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (a known-size "
                         "kernel that scales the HBM byte counters of a profiler run)")
    return ap.parse_args()


KERNEL_SOURCES = {
    "k_wnnm": "paper_2301_03047_amd/csrc/lowrank.hip",
    "k_match_f32": "paper_2301_03047_amd/csrc/match.hip",
    "k_match_f32_slab": "paper_2301_03047_amd/csrc/match.hip",
    "k_match_bf16": "paper_2301_03047_amd/csrc/match.hip",
    "k_topk_partial": "paper_2301_03047_amd/csrc/topk.hip",
}
CONFIG_TEXT = {
    "mri_256": {"image": "256x256 complex64", "solver": "ADMM",
                "mask": "25% random Cartesian lines, 16 centre lines kept"},
    "cacti_1024": {"image": "1024x1024, 24 frames per snapshot", "solver": "GAP",
                   "mask": "Bernoulli(0.5) binary coded apertures"},
    "msfa_512": {"image": "512x512x16 bands", "solver": "GAP", "mask": "4x4 periodic MSFA"},
    "cacti_128": {"image": "128x128, 8 frames per snapshot", "solver": "GAP",
                  "mask": "Bernoulli(0.5) binary coded apertures"},
}


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"{workload}_traffic.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of ``kernel`` from the committed profiler counters
    (FETCH_SIZE + WRITE_SIZE, scaled by a known-size copy), or None when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(traffic_file(workload)))["kernels"][kernel]
        src = os.path.join(ROOT, KERNEL_SOURCES[kernel])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
            return None
        return int(rec["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2301_03047_amd as glr
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wname = args.workload
    if wname == "surrogate":
        from paper_2301_03047_amd import eval_surrogate
        res = eval_surrogate.run(log=lambda m: print(m, file=sys.stderr, flush=True))
        v = res["variants"]
        print(json.dumps({
            "metric": "CNN-surrogate form: wall time and PSNR on 16 MRI 256^2 + 16 CACTI "
                      "512^2x8 instances", "value": v["surrogate+judge"]["speedup_vs_plain"],
            "unit": "x speed-up of surrogate+judge over plain GLR", "n_gpus": 1,
            "higher_is_better": True, "dtype": "bf16+f32", "data": "synthetic",
            "config": {"workload": "surrogate", "train": "20000 128^2 crops of GLR runs of "
                       "mri_256 and cacti_1024"}, "surrogate": res}), flush=True)
        return
    wl = synth.WORKLOADS[wname]
    prec = args.precision or wl.precision
    inst = synth.make_instance(wl)
    sig = synth.sigma_schedule(wl)
    T = wl.iters
    mask = torch.from_numpy(inst["mask"]).cuda() if inst["mask"] is not None else None
    x_true = torch.from_numpy(inst["x_true"]).cuda()
    def make_plan(timing):
        return glr.Plan(wl.modality, wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, iters=T,
                        sigma=sig, mask=mask, timing=timing, precision=prec)

    # `value` comes from a plan without per-stage events; a second plan with
    # them repeats the same number of iterations (continuing from the same
    # state) for the stage split and the roofline of the dominant kernel
    plan = make_plan(False)
    y = plan.forward(x_true)                       # measurement synthesised on the GPU
    state = plan.new_state()
    out = torch.empty_like(x_true)

    def run(p, n, t0):
        t = t0
        for _ in range(n):
            p.reconstruct(y, t, t + 1, state=state, out=out)
            t = (t + 1) % T
        return t

    t = run(plan, args.warmup, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t = run(plan, args.steps, t)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    value = 1000.0 / ms_per_step
    plan_t = make_plan(True)
    plan_t.read_stats(reset=True)                  # stage timers cover the second pass only
    run(plan_t, args.steps, t)
    torch.cuda.synchronize()
    st = plan_t.read_stats(reset=True)
    del plan_t

    stages = {k[3:]: st[k] / args.steps for k in
              ("ms_detect", "ms_norms", "ms_match", "ms_topk", "ms_select", "ms_lowrank",
               "ms_aggregate", "ms_data")}
    match_ms = st["ms_match"] / max(st["match_launches"], 1)
    flop_per_launch = 2.0 * wl.n_keys * wl.n_cand * wl.dim / max(st["match_launches"] / args.steps, 1)
    match_tflops = flop_per_launch / (match_ms * 1e-3) / 1e12
    dominant = max(stages, key=stages.get)

    # roofline of the dominant kernel
    # the FP32 form runs its small-patch variant when a key tile's padded
    # slab (Cp P P2 <= 72 values per key, Cp <= 4) fits in LDS
    P, P2 = wl.patch, wl.patch + (wl.patch & 1)
    Cp = wl.dim // (P * P)
    small = Cp * P * P2 <= 72 and Cp <= 4
    match_kernel = "k_match_bf16" if prec == "bf16" else (
        "k_match_f32_slab" if small else "k_match_f32")
    match_peak = PEAK_BF16_MFMA_TFLOPS if prec == "bf16" else PEAK_FP32_MFMA_TFLOPS
    if dominant == "match":
        roof = {"kernel": match_kernel, "bound": "mfma", "achieved": round(match_tflops, 3),
                "peak": match_peak, "unit": "TFLOP/s",
                "frac": round(match_tflops / match_peak, 4),
                "traffic": measured_traffic(match_kernel, wname)}
    elif dominant == "lowrank":
        # WNNM per group: streamed Householder QR (2 D K^2), Jacobi sweeps on the
        # K x K factor (6 K flop per pair per sweep for the three dots plus 12 K
        # for the two rotations), W = V diag V^T (2 K^3) and the residual Y_c W
        # (2 D K^2, FP64); counted at the measured sweep count
        K, D = wl.k, wl.dim
        sweeps = max(st["jacobi_sweeps_max"], 1)
        flop = wl.n_keys * (2 * D * K * K + sweeps * (K * (K - 1) / 2) * 18 * K + 2 * K ** 3 + 2 * D * K * K)
        ach = flop / (stages["lowrank"] * 1e-3) / 1e12
        roof = {"kernel": "k_wnnm", "bound": "alu", "achieved": round(ach, 4),
                "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_VALU_TFLOPS, 5),
                "traffic": measured_traffic("k_wnnm", wname),
                "note": "upper-bound flop count at the worst group's sweep count"}
    elif dominant == "topk":
        gbs = 4.0 * wl.n_keys * wl.n_cand / (stages["topk"] * 1e-3) / 1e9
        roof = {"kernel": "k_topk_partial", "bound": "hbm", "achieved": round(gbs, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("k_topk_partial", wname)}
    else:
        roof = {"kernel": dominant, "bound": "latency", "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None}

    # quality: a fresh full reconstruction, and the first iterations vs the oracle
    from paper_2301_03047_amd.surrogate import psnr
    xt = inst["x_true"]
    psnr_full = None
    if not args.no_quality:
        fresh, _ = plan.reconstruct(y, 0, T)
        psnr_full = psnr(fresh.cpu().numpy(), xt)

    cpu = None
    psnr_cmp = None
    if not args.no_cpu_baseline and wname == "mri_256":
        from threadpoolctl import threadpool_info
        from oracle import reconstruct as orc, metrics as om_metrics
        n_it = args.cpu_iters
        y64 = y.cpu().numpy().astype(np.complex128)
        wl_cpu = synth.workloads.small(wl, wnnm_c=float(np.float32(wl.wnnm_c)))
        n_cmp = min(5, n_it)                         # tight comparison point
        early = {}

        def keep(t, _v, z):
            if t + 1 == n_cmp:
                early["z"] = z.copy()

        t0 = time.perf_counter()
        ref = orc.reconstruct(wl_cpu, y64, inst["mask"], sig.astype(np.float64), iters=n_it,
                              callback=keep)
        dt = time.perf_counter() - t0
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        cpu = {"value": round(n_it / dt, 4), "unit": "iterations/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {n_it} of {T} ADMM iterations of {wname} (same input), "
                         f"{dt:.1f} s on {os.cpu_count()} host CPUs"}
        # the first n_cmp iterations agree to FP32 rounding; later ones drift
        # apart once a rounding difference flips a discrete choice (a key or
        # a group member), which the per-iteration parity tests allow for
        psnr_cmp = {}
        for name, n, r in (("first", n_cmp, early["z"]), ("sample", n_it, ref)):
            g, _ = plan.reconstruct(y, 0, n)
            g = g.cpu().numpy()
            pg, pr = om_metrics.psnr(g, xt), om_metrics.psnr(r, xt)
            psnr_cmp[name] = {"iters": n, "gpu_db": round(pg, 4), "oracle_db": round(pr, 4),
                              "delta_db": round(pg - pr, 5),
                              "rel_l2_vs_oracle": float(f"{om_metrics.rel_l2(g, r):.3e}")}

    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32" if prec == "bf16" else "f32",
        "data": "synthetic",
        "config": dict({"workload": wname, "patch": wl.patch, "keys": wl.n_keys, "K": wl.k,
                        "iters": T, "matcher": prec}, **CONFIG_TEXT[wname]),
        "roofline": roof,
        "cpu_baseline": cpu,
        "matching_tflops": round(match_tflops, 3),
        "matching_frac_mfma_peak": round(match_tflops / match_peak, 4),
        "stages_ms_per_step": {k: round(v, 4) for k, v in stages.items()},
        "psnr_full_db": None if psnr_full is None else round(psnr_full, 4),
        "psnr_vs_oracle": psnr_cmp,
        "margin_mean": round(st["margin_sum"] / max(wl.n_keys * args.steps, 1), 2),
        "margin_max": st["margin_max"], "overflow_keys": st["overflow_keys"],
        "jacobi_sweeps_max": st["jacobi_sweeps_max"],
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
