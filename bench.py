"""Benchmark: seconds per nuSHT synthesis + adjoint at lmax = 4095 on one MI355X.

Workload (the configuration the headline metric is quoted on): lmax = mmax = 4095, a batch
of 4 independent coefficient sets, N = 33,550,336 = (lmax+1)(2 lmax+1) uniform random points
(cos theta ~ U[-1,1], phi ~ U[0, 2 pi)), seeded synthetic inputs.  One step = one synthesis
(type 2) of the 4 maps plus one adjoint (type 1) of 4 maps, inputs resident in HBM.  The
headline line times the mixed-precision path at eps = 1e-5; the FP64 path at eps = 1e-12 is
timed beside it and their ratio is reported.  Planning (point binning, tables, FFT plans) is
excluded, as in the paper (Sec. III).

Prints ONE JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def legendre_flops(g, nmaps):
    """Algorithmic flops of one Legendre launch: per (l, m, ring pair) one recurrence step
    (3 flops: a multiply and an FMA) and one complex-by-real FMA per map (4 flops)."""
    pairs = (g["nrings"] + 1) // 2
    return float(g["nalm"]) * pairs * (3 + 4 * nmaps)


def point_bytes(g, nmaps, elem):
    """Algorithmic HBM bytes of one interpolation / spreading pass: FP64 theta, phi read once,
    the B point values, and the touched half of the fine grid (rows theta in [0, pi] + w)."""
    n = g["npts"]
    touched = (g["n1"] // 2 + g["width"]) * g["n2"]
    return 16.0 * n + 8.0 * nmaps * n + float(elem) * nmaps * touched


def run_precision(P, torch, cfg, eps, dtype, steps, warmup, alm, d):
    th = torch.from_numpy(cfg["theta"]).cuda()
    ph = torch.from_numpy(cfg["phi"]).cuda()
    t0 = time.perf_counter()
    plan = P.Plan(cfg["lmax"], cfg["mmax"], th, ph, eps, dtype=dtype, timing=True)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    del th, ph
    B = alm.shape[0]
    fmap = torch.empty((B, plan.npts), dtype=torch.float64, device="cuda")
    calm = torch.empty((B, plan.nalm), dtype=torch.complex128, device="cuda")

    def step():
        plan.synthesis(alm, out=fmap)
        plan.adjoint(d, out=calm)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    # per-stage device times from the library's own HIP events on the call stream
    syn, adj = {}, {}
    for _ in range(max(3, min(steps, 5))):
        plan.synthesis(alm, out=fmap)
        for k, v in plan.stage_times().items():
            syn.setdefault(k, []).append(v)
        plan.adjoint(d, out=calm)
        for k, v in plan.stage_times().items():
            adj.setdefault(k, []).append(v)
    syn = {k: float(np.mean(v)) for k, v in syn.items() if np.mean(v) > 0}
    adj = {k: float(np.mean(v)) for k, v in adj.items() if np.mean(v) > 0}
    plan.synthesis(alm, out=fmap)
    f = fmap.cpu().numpy()
    plan.adjoint(d, out=calm)
    c = calm.cpu().numpy()
    return dict(plan=plan, plan_s=plan_s, sec=sec, syn=syn, adj=adj, f=f, c=c)


def cpu_baseline(cfg, alm_np, d_np, nsample, nmaps):
    """The oracle (plain C direct sums) on a bounded sample of the same workload, scaled
    linearly in the number of points to one full step (synthesis + adjoint of all maps)."""
    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    idx = np.random.default_rng(7).choice(cfg["theta"].size, nsample, replace=False)
    th, ph = cfg["theta"][idx], cfg["phi"][idx]
    t0 = time.perf_counter()
    fs = oracle.synthesis(cfg["lmax"], cfg["mmax"], th, ph, alm_np[:1], nthreads=threads)
    t1 = time.perf_counter()
    oracle.adjoint(cfg["lmax"], cfg["mmax"], th, ph, d_np[:1, idx], nthreads=threads)
    t2 = time.perf_counter()
    scale = cfg["theta"].size / nsample * nmaps
    return dict(value=(t2 - t0) * scale, syn=(t1 - t0) * scale, adj=(t2 - t1) * scale,
                threads=threads, idx=idx, f_sample=fs, sample_s=t2 - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c3", "c1"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2406_14542_amd as P
    from paper_2406_14542_amd import inputs

    P.lib()
    log("generating inputs")
    if args.workload == "c3":
        cfg = inputs.config_c3()
        eps_mixed, eps_ref = cfg["eps"], cfg["eps_ref"]
    else:
        cfg = inputs.config_c1()
        eps_mixed, eps_ref = 1e-5, 1e-12
    alm_np, d_np = cfg["alm"], cfg["d"]
    B = alm_np.shape[0]
    alm = torch.from_numpy(alm_np).cuda()
    d = torch.from_numpy(d_np).cuda()
    log(f"workload {cfg['name']}: lmax={cfg['lmax']} B={B} N={cfg['theta'].size}")

    log("mixed precision")
    mx = run_precision(P, torch, cfg, eps_mixed, "mixed", args.steps, args.warmup, alm, d)
    g = mx["plan"].geometry
    log(f"mixed: {mx['sec'] * 1e3:.2f} ms/step; stages syn {mx['syn']} adj {mx['adj']}")
    fp = None
    if not args.no_fp64:
        mx["plan"].close()
        log("fp64")
        fp = run_precision(P, torch, cfg, eps_ref, "f64", args.steps, args.warmup, alm, d)
        log(f"fp64: {fp['sec'] * 1e3:.2f} ms/step; stages syn {fp['syn']} adj {fp['adj']}")

    # roofline of the dominant kernel of the headline (mixed) step
    cands = []
    for direction, st in (("synthesis", mx["syn"]), ("adjoint", mx["adj"])):
        if "legendre" in st:
            fl = legendre_flops(g, B)
            cands.append(dict(kernel=f"legendre_{direction}", ms=st["legendre"], bound="alu",
                              work=fl, achieved=fl / (st["legendre"] * 1e-3) / 1e12,
                              peak=FP64_PEAK_TFLOPS, unit="TFLOP/s"))
        if "points" in st:
            by = point_bytes(g, B, 4)
            name = "interp" if direction == "synthesis" else "spread"
            cands.append(dict(kernel=name, ms=st["points"], bound="hbm", work=by,
                              achieved=by / (st["points"] * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                              unit="GB/s"))
    dom = max(cands, key=lambda c: c["ms"])
    roofline = {"bound": dom["bound"], "achieved": round(dom["achieved"], 3),
                "peak": dom["peak"], "unit": dom["unit"],
                "frac": round(dom["achieved"] / dom["peak"], 4), "traffic": None,
                "kernel": dom["kernel"], "ms_per_launch": round(dom["ms"], 4),
                "algorithmic_work_per_launch": dom["work"]}
    others = {c["kernel"]: {"ms": round(c["ms"], 4), "achieved": round(c["achieved"], 3),
                            "unit": c["unit"], "frac": round(c["achieved"] / c["peak"], 4)}
              for c in cands}

    # accuracy: mixed vs FP64 path, and both vs the oracle on a sample of points
    acc = {}
    cpu = None
    if fp is not None:
        acc["mixed_vs_fp64_synthesis_rel_l2"] = float(
            np.linalg.norm(mx["f"] - fp["f"]) / np.linalg.norm(fp["f"]))
        _, ms_ = inputs.ell_of_index(cfg["lmax"], cfg["mmax"])
        w = np.where(ms_ == 0, 1.0, 2.0)
        acc["mixed_vs_fp64_adjoint_rel_l2"] = float(np.sqrt(
            np.sum(w * np.abs(mx["c"] - fp["c"]) ** 2) / np.sum(w * np.abs(fp["c"]) ** 2)))
    if not args.no_cpu_baseline:
        log(f"cpu baseline on {args.cpu_sample} points")
        cpu = cpu_baseline(cfg, alm_np, d_np, args.cpu_sample, B)
        idx = cpu["idx"]
        ref = cpu["f_sample"][0]
        acc["mixed_vs_oracle_sample_rel_l2"] = float(
            np.linalg.norm(mx["f"][0, idx] - ref) / np.linalg.norm(ref))
        if fp is not None:
            acc["fp64_vs_oracle_sample_rel_l2"] = float(
                np.linalg.norm(fp["f"][0, idx] - ref) / np.linalg.norm(ref))
        log(f"cpu: {cpu['sample_s']:.1f} s on the sample -> {cpu['value']:.1f} s/step")

    out = {
        "metric": "nuSHT synthesis+adjoint seconds at lmax=4095 (mixed eps=1e-5; FP64 eps=1e-12 "
                  "beside it)",
        "value": round(mx["sec"], 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["sec"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: lmax=mmax={cfg['lmax']}, {B} maps, "
                               f"N={cfg['theta'].size} uniform points, synthesis+adjoint",
                   "eps": eps_mixed, "precision": "mixed (FP64 Legendre/coords, FP32 nuFFT+FFT)",
                   "nmaps": B, "npts": int(cfg["theta"].size), "lmax": cfg["lmax"],
                   "dfs_mode": "fused", "sigma": g["sigma"], "width": g["width"],
                   "fine_grid": [g["n1"], g["n2"]]},
        "mixed": {"s_per_step": mx["sec"], "synthesis_stages_ms": mx["syn"],
                  "adjoint_stages_ms": mx["adj"], "plan_s": mx["plan_s"]},
        "roofline": roofline,
        "roofline_kernels": others,
        "accuracy": acc,
    }
    if fp is not None:
        out["fp64"] = {"s_per_step": fp["sec"], "eps": eps_ref, "synthesis_stages_ms": fp["syn"],
                       "adjoint_stages_ms": fp["adj"], "plan_s": fp["plan_s"],
                       "width": fp["plan"].geometry["width"]}
        out["speedup_mixed_over_fp64"] = round(fp["sec"] / mx["sec"], 3)
    if cpu is not None:
        out["cpu_baseline"] = {"value": round(cpu["value"], 3), "unit": "s", "cores": cpu["threads"],
                               "kind": "oracle",
                               "sample": f"FP64 direct-sum synthesis+adjoint of 1 map on "
                                         f"{args.cpu_sample} of the {cfg['theta'].size} points, "
                                         f"scaled by N/{args.cpu_sample} x {B} maps"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
