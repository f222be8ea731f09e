"""Benchmark: seconds per nuSHT synthesis + adjoint at lmax = 4095 on one MI355X.

Workload (the configuration the headline metric is quoted on): lmax = mmax = 4095, a batch
of 4 independent coefficient sets, N = 33,550,336 = (lmax+1)(2 lmax+1) uniform random points
(cos theta ~ U[-1,1], phi ~ U[0, 2 pi)), seeded synthetic inputs.  One step = one synthesis
(type 2) of the 4 maps plus one adjoint (type 1) of 4 maps, inputs resident in HBM.  The
headline line times the mixed-precision path at eps = 1e-5; the FP64 path at eps = 1e-12 is
timed beside it and their ratio is reported.  Planning (point binning, tables, FFT plans) is
excluded, as in the paper (Sec. III).

Prints ONE JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
`--cg` runs the learned-preconditioner leg instead (CGLS iterations, learned weights vs
plain; see run_cg).
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
    """Algorithmic flops of one Legendre launch: per (l, m, ring pair) one step of the
    three-term recurrence lam_l = A x lam_{l-1} - B lam_{l-2} (a multiply and an FMA, 3 flops)
    and, per map, one complex-by-real FMA into the parity accumulator (4 flops):
    nalm x ceil(N_r / 2) x (3 + 4 B)."""
    pairs = (g["nrings"] + 1) // 2
    return float(g["nalm"]) * pairs * (3 + 4 * nmaps)


def point_bytes(g, nmaps, elem):
    """Algorithmic HBM bytes of one interpolation / spreading pass: FP64 theta, phi read once
    (16 N), the B point values in the kernel's precision (s B N) and the touched half of the
    fine grid (rows theta in [0, pi] plus w) once (s B (n1/2 + w) n2), s = 4 or 8."""
    n = g["npts"]
    touched = (g["n1"] // 2 + g["width"]) * g["n2"]
    return 16.0 * n + float(elem) * nmaps * n + float(elem) * nmaps * touched


def step_stats(times):
    """median of all timed steps, and mean +- 1 sigma over the first five (Sec. IV reports
    the mean of 5 runs with one standard deviation)"""
    t = np.asarray(times)
    five = t[:5]
    return {"median_s": float(np.median(t)), "mean5_s": float(five.mean()),
            "std5_s": float(five.std(ddof=1)) if five.size > 1 else 0.0}


def run_precision(P, torch, cfg, eps, dtype, steps, warmup, alm, d, sigma=0.0):
    th = torch.from_numpy(cfg["theta"]).cuda()
    ph = torch.from_numpy(cfg["phi"]).cuda()
    t0 = time.perf_counter()
    plan = P.Plan(cfg["lmax"], cfg["mmax"], th, ph, eps, dtype=dtype, timing=True, sigma=sigma)
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
    plan.stage_reset()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        # the library enqueues on torch's current stream, so these events bracket the step
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    per_step = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    plan.status()
    # per-stage device times over exactly the timed calls, from the HIP events the library
    # records around each stage on the stream the stage's kernels run on
    syn = {k: v[0] for k, v in plan.stage_stats("synthesis").items() if v[0] > 0}
    adj = {k: v[0] for k, v in plan.stage_stats("adjoint").items() if v[0] > 0}
    plan.synthesis(alm, out=fmap)
    f = fmap.cpu().numpy()
    plan.adjoint(d, out=calm)
    c = calm.cpu().numpy()
    return dict(plan=plan, plan_s=plan_s, sec=sec, syn=syn, adj=adj, f=f, c=c,
                stats=step_stats(per_step))


def host_cpu():
    """model name and logical core count of the host"""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg, alm_np, d_np, nsample, nmaps, nsample1):
    """The oracle (plain C direct sums) on a bounded sample of the same workload, scaled
    linearly in the number of points to one full step (synthesis + adjoint of all maps), on
    all the threads the host gives this process and on one thread (smaller sample)."""
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
    i1 = idx[:nsample1]
    t3 = time.perf_counter()
    oracle.synthesis(cfg["lmax"], cfg["mmax"], cfg["theta"][i1], cfg["phi"][i1], alm_np[:1],
                     nthreads=1)
    oracle.adjoint(cfg["lmax"], cfg["mmax"], cfg["theta"][i1], cfg["phi"][i1], d_np[:1, i1],
                   nthreads=1)
    t4 = time.perf_counter()
    return dict(value=(t2 - t0) * scale, syn=(t1 - t0) * scale, adj=(t2 - t1) * scale,
                threads=threads, idx=idx, f_sample=fs, sample_s=t2 - t0,
                one_core=(t4 - t3) * cfg["theta"].size / nsample1 * nmaps,
                one_core_sample_s=t4 - t3)


def golden_adjoint_error(c, lmax, path):
    """relative error of the adjoint of all maps on the stored whole m-columns of the oracle
    (written by tests/golden/make_large_oracle_values.py), in the <.,.>_m norm"""
    if not os.path.exists(path):
        return None
    z = np.load(path)
    ms, ref = [int(m) for m in z["ms"]], z["cols"]
    got = np.zeros_like(ref)
    for k, m in enumerate(ms):
        i0 = m * (2 * lmax + 1 - m) // 2
        got[:, k, m:] = c[:, i0 + m:i0 + lmax + 1]
    w = np.where(np.asarray(ms) == 0, 1.0, 2.0)[None, :, None]
    return float(np.sqrt(np.sum(w * np.abs(got - ref) ** 2) / np.sum(w * np.abs(ref) ** 2)))


def run_cg(args):
    """Learned-preconditioner leg (`--cg`): CGLS iterations to ||S a - d|| / ||d|| <= tol on
    holey point sets (lmax = mmax, N = 1.5 (lmax+1)^2 points with density
    (1 + 0.8 cos^2 theta) and 20 Gaussian holes of 5 degrees, d = S a_true).

    `--cg-phase train`: the network is trained on the GPU by the library's kernels on the
    seeded sets 1000 .. 1000 + cg-train - 1, streamed: every new set is planned, its target a*
    is the method's own plain CGLS solve (at most `--cg-target-iters` iterations), and it joins
    a replay buffer of the last `--cg-buffer` sets; after each new set `--cg-steps-per-set`
    Adam steps run on `--cg-batch` sets drawn from the buffer.  The parameters and Adam state
    are saved to `--cg-save`.
    `--cg-phase eval`: the network loaded from `--cg-load` is evaluated on the held-out sets
    1160 .. 1160 + cg-test - 1: plain CGLS from zero, CGLS on W^(1/2) S from S^H W d with the
    network's weights, and the same with the analytic weights (4 pi / N) / rho^ (the coarse
    density map at the point), each to `--cg-maxiter` iterations.  Prints ONE JSON line."""
    import torch
    import paper_2406_14542_amd as P
    from paper_2406_14542_amd import inputs
    from paper_2406_14542_amd.learned import LearnedWeights

    P.lib()
    L = args.cg_lmax
    tol = args.cg_tol
    marks = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8]

    def first_below(hist, t):
        idx = np.nonzero(hist <= t)[0]
        return int(idx[0]) if idx.size else None

    def make(seed):
        cfg = inputs.config_c5(seed, lmax=L)
        th = torch.from_numpy(cfg["theta"]).cuda()
        ph = torch.from_numpy(cfg["phi"]).cuda()
        pl = P.Plan(L, L, th, ph, args.cg_eps)
        d = pl.synthesis(torch.from_numpy(cfg["alm"]).cuda())
        return dict(plan=pl, theta=th, phi=ph, d=d, seed=seed)

    workload = (f"holey point sets: lmax=mmax={L}, N={int(1.5 * (L + 1) ** 2)}, 20 holes of "
                f"5 deg, density 1 + 0.8 cos^2 theta")
    if args.cg_phase == "train":
        lw = LearnedWeights(64, 128, seed=args.cg_seed)
        rng = np.random.default_rng(args.cg_seed)
        buf = []
        losses = []
        t0 = time.perf_counter()
        for s in range(args.cg_train):
            ex = make(1000 + s)
            ex["features"] = lw.features(ex["theta"], ex["phi"])
            a, it, rr, st = ex["plan"].solve(ex["d"], tol=tol, maxiter=args.cg_target_iters,
                                             check=False)
            ex["astar"] = a
            buf.append(ex)
            if len(buf) > args.cg_buffer:
                old = buf.pop(0)
                old["plan"].close()
            for _ in range(args.cg_steps_per_set):
                pick = rng.choice(len(buf), size=min(args.cg_batch, len(buf)), replace=False)
                h = lw.train([buf[k] for k in pick], steps=1, lr=args.cg_lr)
                losses.append(h[-1] / len(pick))
            torch.cuda.synchronize()
            log(f"train set {1000 + s}: target after {it} iterations (residual {rr:.2e}); "
                f"loss {losses[-1]:.4f} ({time.perf_counter() - t0:.0f} s)")
        lw.save(args.cg_save)
        out = {"metric": "learned-weight training (CGLS preconditioner)", "phase": "train",
               "value": float(np.mean(losses[-20:])), "unit": "loss", "n_gpus": 1,
               "higher_is_better": False, "data": "synthetic",
               "config": {"workload": workload, "train_seeds": [1000, 1000 + args.cg_train - 1],
                          "target_iters": args.cg_target_iters, "buffer": args.cg_buffer,
                          "batch": args.cg_batch, "steps_per_set": args.cg_steps_per_set,
                          "lr": args.cg_lr, "eps": args.cg_eps, "density_map": [64, 128]},
               "loss_first": losses[:10], "loss_last": losses[-10:],
               "adam_steps": len(losses), "train_s": round(time.perf_counter() - t0, 1)}
        print(json.dumps(out), flush=True)
        return

    lw = LearnedWeights.load(args.cg_load)
    rows = []
    for s in range(args.cg_test):
        ex = make(1160 + s)
        pl, d = ex["plan"], ex["d"]
        res = {"seed": 1160 + s}
        feats = lw.features(ex["theta"], ex["phi"])
        scale = LearnedWeights.scale(pl.npts)
        for kind in ("plain", "learned", "analytic"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if kind == "plain":
                _, it, rr, st, h = pl.solve(d, tol=tol, maxiter=args.cg_maxiter, check=False,
                                            history=True)
            else:
                if kind == "learned":
                    w = lw.weights(features=feats)
                else:
                    # 1 / rho^ at the point (feature 0 is log rho^, bilinear in the map)
                    w = (torch.exp(-feats[:, 0]) * scale).contiguous()
                x0 = pl.weighted_adjoint(d, w)
                _, it, rr, st, h = pl.solve(d, x0=x0, weights=w, tol=tol,
                                            maxiter=args.cg_maxiter, check=False, history=True)
            torch.cuda.synchronize()
            res[kind] = {"iters": it, "relres": rr, "s": round(time.perf_counter() - t1, 3),
                         "iters_to": {f"{m:g}": first_below(h, m) for m in marks}}
        rows.append(res)
        if args.cg_rows:
            with open(args.cg_rows, "a") as fh:
                fh.write(json.dumps(res) + "\n")
        log(f"held-out {1160 + s}: " + ", ".join(
            f"{k} {res[k]['iters']} it ({res[k]['relres']:.2e}), to 1e-4 in "
            f"{res[k]['iters_to']['0.0001']}" for k in ("plain", "learned", "analytic")))
        pl.close()

    def stat(kind, m):
        v = [r[kind]["iters_to"][f"{m:g}"] for r in rows]
        got = [x for x in v if x is not None]
        return {"reached": len(got), "of": len(v),
                "mean": float(np.mean(got)) if got else None,
                "median": float(np.median(got)) if got else None}

    table = {kind: {f"{m:g}": stat(kind, m) for m in marks}
             for kind in ("plain", "learned", "analytic")}
    out = {"metric": f"CGLS iterations to relative residual thresholds at lmax={L} "
                     "(learned weights vs plain vs analytic 1/rho)",
           "phase": "eval",
           "value": table["learned"]["0.0001"]["mean"], "unit": "iterations to 1e-4 (mean)",
           "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
           "dtype": "f64 transforms, f32 network", "data": "synthetic",
           "config": {"workload": workload, "tol": tol, "maxiter": args.cg_maxiter,
                      "test_seeds": [1160, 1160 + args.cg_test - 1], "eps": args.cg_eps},
           "thresholds": table,
           "residual_after_maxiter_mean": {k: float(np.mean([r[k]["relres"] for r in rows]))
                                           for k in ("plain", "learned", "analytic")},
           "wall_s_mean": {k: float(np.mean([r[k]["s"] for r in rows]))
                           for k in ("plain", "learned", "analytic")},
           "held_out": rows}
    print(json.dumps(out), flush=True)


def run_pointing(args):
    """Lensing-pointing leg (`--pointing`, App. C, Fig. C1): for each lmax, a regular grid of
    (lmax + 1) rings x (2 lmax + 1) pixels (ring centres, pixel 0 at phi = 0) and a potential
    Phi_lm with C_l ~ l^-4 scaled to 2.5' rms deflection.  Times, after one warm-up call, the
    whole pointing (derivative synthesis for Eq. C2, then Eq. C1 per point) and the Eq. (C1)
    kernel on its own (nusht_deflect on the resulting alpha), FP64 plans at `--pointing-eps`.
    Prints ONE JSON line."""
    import torch
    import paper_2406_14542_amd as P
    from paper_2406_14542_amd import inputs

    P.lib()
    rows = []
    for L in [int(x) for x in args.pointing_lmax.split(",") if x]:
        rings, pix = L + 1, 2 * L + 1
        th1 = (np.arange(rings) + 0.5) * np.pi / rings
        ph1 = 2.0 * np.pi * np.arange(pix) / pix
        T, Ph = np.meshgrid(th1, ph1, indexing="ij")
        th = torch.from_numpy(np.ascontiguousarray(T.ravel())).cuda()
        ph = torch.from_numpy(np.ascontiguousarray(Ph.ravel())).cuda()
        dlm = torch.from_numpy(inputs.potential_alm(np.random.default_rng(105), L, L, 2.5)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl = P.Plan(L, L, th, ph, args.pointing_eps)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        n = pl.npts
        pl.pointing(dlm)
        _, dth, dph = pl.synthesis_deriv(dlm)
        s = torch.sin(th)
        ath = dth[0].contiguous()
        aph = torch.where(s != 0, dph[0] / s, torch.zeros_like(s)).contiguous()
        t2, p2 = P.deflect(th, ph, ath, aph)
        torch.cuda.synchronize()
        times, ktimes = [], []
        for _ in range(max(args.steps, 1)):
            t0 = time.perf_counter()
            pl.pointing(dlm)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(max(args.steps, 1)):
            ev0.record()
            t2, p2 = P.deflect(th, ph, ath, aph)
            ev1.record()
            torch.cuda.synchronize()
            ktimes.append(ev0.elapsed_time(ev1) * 1e-3)
        pl.status()
        t = float(np.median(times))
        k = float(np.median(ktimes))
        rows.append({"lmax": L, "npts": n, "plan_s": round(plan_s, 3),
                     "pointing_ms": round(1e3 * t, 3), "pointing_gpts_s": round(n / t / 1e9, 3),
                     "c1_kernel_ms": round(1e3 * k, 4),
                     "c1_kernel_gbs": round(48.0 * n / k / 1e9, 1)})
        log(f"pointing lmax {L}: N = {n}, {1e3 * t:.2f} ms ({n / t / 1e9:.2f} Gpts/s); "
            f"Eq. C1 kernel alone {1e3 * k:.3f} ms")
        pl.close()
        del th, ph, dlm, dth, dph, ath, aph, t2, p2, s
        torch.cuda.empty_cache()
    out = {"metric": "lensing pointing time (Eq. C2 + C1) per call", "value": rows[-1]["pointing_ms"],
           "unit": "ms", "n_gpus": 1, "steps": max(args.steps, 1), "higher_is_better": False,
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "regular grids of (lmax+1) x (2 lmax+1) points, potential "
                                  "C_l ~ l^-4 at 2.5 arcmin rms deflection",
                      "eps": args.pointing_eps},
           "c1_kernel_bytes_per_point": 48, "rows": rows}
    print(json.dumps(out), flush=True)


def spin_legendre_flops(g, nfields):
    """Algorithmic flops of one spin-weighted Legendre launch (synthesis or adjoint): per
    (l, m, ring pair) one step of the two Wigner-d recurrences (an FMA for the x-dependent
    factor, a multiply and an FMA for the step: 5 flops each), the two combinations W+- (an
    FMA each, 4 flops) and, per field, 8 real multiply-adds (16 flops: the synthesis' four
    complex-by-real accumulations; the adjoint's four products with the ring data and their
    sums over rings): nalm x ceil(N_r / 2) x (14 + 16 F)."""
    pairs = (g["nrings"] + 1) // 2
    return float(g["nalm"]) * pairs * (14 + 16 * nfields)


def spin_leg(spin, F, dtypes, steps, warmup):
    """The spin-weighted step on the headline workload's points: lmax = 4095, the 33,550,336
    uniform C3 points (the nmaps = 1 draw), F spin-`spin` fields (two real maps each; F = 2
    gives the same four real maps as the spin-0 step), one step = one synthesis_spin + one
    adjoint_spin, for each (dtype, eps) in dtypes.  Accuracy: the dot test
    <d, S a> = <S^H d, a>_m per dtype and, for spin 2 with two fields, the synthesis against the
    oracle's direct sums stored by tests/golden/make_large_oracle_values.py (48 points)."""
    import torch
    import paper_2406_14542_amd as P
    from paper_2406_14542_amd import inputs

    P.lib()
    cfg = inputs.config_c3(nmaps=1)
    L = cfg["lmax"]
    rng = np.random.default_rng(106)
    a_np = inputs.spin_alm(rng, L, L, spin, F)
    d_np = rng.standard_normal((F, 2, cfg["theta"].size))
    a = torch.from_numpy(a_np).cuda()
    d = torch.from_numpy(d_np).cuda()
    _, ms = inputs.ell_of_index(L, L)
    w = torch.from_numpy(np.where(ms == 0, 1.0, 2.0)).cuda()
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "c3_spin2_sample_synthesis.npz")
    if spin == 2 and F == 2 and os.path.exists(gpath):
        with np.load(gpath) as z:
            golden = (z["idx"], z["f"])
    res = {}
    maps = {}
    for dtype, eps in dtypes:
        th = torch.from_numpy(cfg["theta"]).cuda()
        ph = torch.from_numpy(cfg["phi"]).cuda()
        pl = P.Plan(L, L, th, ph, eps, dtype=dtype, timing=True)
        del th, ph
        f = torch.empty((F, 2, pl.npts), dtype=torch.float64, device="cuda")
        c = torch.empty((F, 2, pl.nalm), dtype=torch.complex128, device="cuda")

        def step():
            pl.synthesis_spin(spin, a, out=f)
            pl.adjoint_spin(spin, d, out=c)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        pl.stage_reset()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for e0, e1 in evs:
            e0.record()
            step()
            e1.record()
        torch.cuda.synchronize()
        pl.status()
        per = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
        syn = {k: v[0] for k, v in pl.stage_stats("synthesis_spin").items() if v[0] > 0}
        adj = {k: v[0] for k, v in pl.stage_stats("adjoint_spin").items() if v[0] > 0}
        g = pl.geometry
        fl = spin_legendre_flops(g, F)
        lhs = float(torch.sum(d * f))
        rhs = float(torch.sum(w * (torch.conj(c) * a).real))
        maps[dtype] = f.cpu().numpy()
        st = step_stats(per)
        res[dtype] = {"ms_per_step": round(1e3 * st["median_s"], 3), **st, "eps": eps,
                      "width": g["width"], "synthesis_stages_ms": syn, "adjoint_stages_ms": adj,
                      "roofline_kernels": {
                          "spin_legendre_synthesis": {
                              "ms": round(syn["legendre"], 4),
                              "achieved": round(fl / (syn["legendre"] * 1e-3) / 1e12, 3),
                              "unit": "TFLOP/s",
                              "frac": round(fl / (syn["legendre"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)},
                          "spin_legendre_adjoint": {
                              "ms": round(adj["legendre"], 4),
                              "achieved": round(fl / (adj["legendre"] * 1e-3) / 1e12, 3),
                              "unit": "TFLOP/s",
                              "frac": round(fl / (adj["legendre"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}},
                      "dot_test_rel": abs(lhs - rhs) / abs(lhs),
                      "legendre_flops_per_launch": fl}
        if golden is not None:
            idx, ref = golden
            res[dtype]["synthesis_vs_oracle_sample_rel_l2"] = float(
                np.linalg.norm(maps[dtype][:, :, idx] - ref) / np.linalg.norm(ref))
        log(f"spin {spin} {dtype}: {res[dtype]['ms_per_step']:.2f} ms/step; syn {syn} adj {adj}")
        pl.close()
        del f, c
        torch.cuda.empty_cache()
    return res, maps, cfg


def run_spin(args):
    """Spin-weighted leg (`--spin S`, the spin-n extension of Sec. V): spin_leg for mixed
    precision at eps = 1e-5 and FP64 at 1e-12, plus the mixed synthesis against the FP64 one.
    Prints ONE JSON line."""
    spin, F = args.spin, args.spin_fields
    res, maps, cfg = spin_leg(spin, F, (("mixed", 1e-5), ("f64", 1e-12)), args.steps,
                              args.warmup)
    L = cfg["lmax"]
    acc = {"mixed_vs_fp64_synthesis_rel_l2": float(
        np.linalg.norm(maps["mixed"] - maps["f64"]) / np.linalg.norm(maps["f64"]))}
    for dt in ("mixed", "f64"):
        if "synthesis_vs_oracle_sample_rel_l2" in res[dt]:
            acc[f"{dt}_vs_oracle_sample_rel_l2"] = res[dt]["synthesis_vs_oracle_sample_rel_l2"]
    out = {"metric": f"spin-{spin} nuSHT synthesis+adjoint seconds at lmax={L} "
                     f"({F} fields = {2 * F} real maps)",
           "value": res["mixed"]["median_s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["mixed"]["ms_per_step"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"c3 points (N={cfg['theta'].size} uniform), lmax=mmax={L}, "
                                  f"spin {spin}, {F} fields", "spin": spin, "nfields": F},
           "mixed": res["mixed"], "fp64": res["f64"], "accuracy": acc,
           "legendre_flops_per_launch": res["mixed"]["legendre_flops_per_launch"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c3", "c1"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=768)
    ap.add_argument("--cpu-sample1", type=int, default=32)
    ap.add_argument("--sigma125-steps", type=int, default=5,
                    help="timed steps of the mixed plan at sigma = 1.25 (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cg", action="store_true",
                    help="run the learned-preconditioner CGLS leg instead of the transform step")
    ap.add_argument("--cg-lmax", type=int, default=2047)
    ap.add_argument("--cg-phase", choices=["train", "eval"], default="eval")
    ap.add_argument("--cg-tol", type=float, default=1e-8)
    ap.add_argument("--cg-eps", type=float, default=1e-12)
    ap.add_argument("--cg-maxiter", type=int, default=1500)
    ap.add_argument("--cg-target-iters", type=int, default=600)
    ap.add_argument("--cg-train", type=int, default=160)
    ap.add_argument("--cg-test", type=int, default=40)
    ap.add_argument("--cg-buffer", type=int, default=16)
    ap.add_argument("--cg-batch", type=int, default=4)
    ap.add_argument("--cg-steps-per-set", type=int, default=1)
    ap.add_argument("--cg-lr", type=float, default=1e-3)
    ap.add_argument("--cg-seed", type=int, default=7)
    ap.add_argument("--cg-save", default="c5_network.npz")
    ap.add_argument("--cg-load", default="c5_network.npz")
    ap.add_argument("--cg-rows", default="",
                    help="eval: also append each held-out row to this JSON-lines file as it ends")
    ap.add_argument("--pointing", action="store_true",
                    help="run the lensing-pointing leg (Eq. C2 + C1) instead of the transform step")
    ap.add_argument("--pointing-lmax", default="1023,2047,4095")
    ap.add_argument("--pointing-eps", type=float, default=1e-12)
    ap.add_argument("--spin", type=int, default=0,
                    help="run the spin-weighted leg with this spin instead of the transform step")
    ap.add_argument("--spin-fields", type=int, default=2)
    ap.add_argument("--no-spin", action="store_true",
                    help="leave out the spin-2 entry of the default line")
    ap.add_argument("--spin-steps", type=int, default=5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one elementwise device copy of BYTES bytes (the reference "
                         "kernel that scales HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.pointing:
        run_pointing(args)
        return
    if args.spin:
        run_spin(args)
        return
    if args.cg:
        run_cg(args)
        return

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

    # the paper's upsampling sigma = 1.25 beside sigma = 2 (mixed, same eps; fewer steps)
    s125 = None
    if args.sigma125_steps > 0:
        if fp is not None:
            fp["plan"].close()
        else:
            mx["plan"].close()
        log("mixed, sigma = 1.25")
        s125 = run_precision(P, torch, cfg, eps_mixed, "mixed", args.sigma125_steps, 2, alm, d,
                             sigma=1.25)
        log(f"sigma 1.25: {s125['sec'] * 1e3:.2f} ms/step; stages syn {s125['syn']} "
            f"adj {s125['adj']}")

    def kernels(run, elem, geo):
        """per-kernel roofline figures of one precision's step: the Legendre launches against
        the FP64 peak, the point stages (a7 interpolation, b1 spreading) against HBM"""
        cands = []
        for direction, st in (("synthesis", run["syn"]), ("adjoint", run["adj"])):
            if "legendre" in st:
                fl = legendre_flops(geo, B)
                cands.append(dict(kernel=f"legendre_{direction}", ms=st["legendre"],
                                  bound="alu", work=fl,
                                  achieved=fl / (st["legendre"] * 1e-3) / 1e12,
                                  peak=FP64_PEAK_TFLOPS, unit="TFLOP/s"))
            if "points" in st:
                by = point_bytes(geo, B, elem)
                ms = st["points"]
                name = "interp" if direction == "synthesis" else "spread"
                cands.append(dict(kernel=name, ms=ms, bound="hbm", work=by,
                                  achieved=by / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                                  unit="GB/s"))
        return cands

    def roofline_of(cands, traffic_key):
        dom = max(cands, key=lambda c: c["ms"])
        # measured HBM bytes per launch of that kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE
        # runs scaled by a copy kernel), when they are on record for the kernel as it stands
        traffic = None
        tfile = os.path.join(ROOT, "profiles", "c3_traffic.json")
        if args.workload == "c3" and os.path.exists(tfile):
            rec = json.load(open(tfile)).get(traffic_key, {}).get(dom["kernel"])
            if rec:
                traffic = round(rec["hbm_bytes"], -6)
        return {"bound": dom["bound"], "achieved": round(dom["achieved"], 3),
                "peak": dom["peak"], "unit": dom["unit"],
                "frac": round(dom["achieved"] / dom["peak"], 4), "traffic": traffic,
                "kernel": dom["kernel"], "ms_per_launch": round(dom["ms"], 4),
                "algorithmic_work_per_launch": dom["work"]}

    cands = kernels(mx, 4, g)
    roofline = roofline_of(cands, "kernels")
    others = {c["kernel"]: {"ms": round(c["ms"], 4), "achieved": round(c["achieved"], 3),
                            "unit": c["unit"], "frac": round(c["achieved"] / c["peak"], 4)}
              for c in cands}
    fp_roofline = fp_others = None
    if fp is not None:
        fcands = kernels(fp, 8, fp["plan"].geometry)
        fp_roofline = roofline_of(fcands, "kernels_fp64")
        fp_others = {c["kernel"]: {"ms": round(c["ms"], 4), "achieved": round(c["achieved"], 3),
                                   "unit": c["unit"], "frac": round(c["achieved"] / c["peak"], 4)}
                     for c in fcands}

    # accuracy: mixed vs FP64 path, both vs the oracle on a sample of points (synthesis) and on
    # whole m-columns over all points (adjoint, stored oracle values)
    acc = {}
    cpu = None
    golden = os.path.join(ROOT, "tests", "golden", "c3_adjoint_columns.npz")
    if args.workload == "c3":
        acc["mixed_adjoint_vs_oracle_columns_rel"] = golden_adjoint_error(mx["c"], cfg["lmax"],
                                                                          golden)
        if fp is not None:
            acc["fp64_adjoint_vs_oracle_columns_rel"] = golden_adjoint_error(
                fp["c"], cfg["lmax"], golden)
    if fp is not None:
        acc["mixed_vs_fp64_synthesis_rel_l2"] = float(
            np.linalg.norm(mx["f"] - fp["f"]) / np.linalg.norm(fp["f"]))
        _, ms_ = inputs.ell_of_index(cfg["lmax"], cfg["mmax"])
        w = np.where(ms_ == 0, 1.0, 2.0)
        acc["mixed_vs_fp64_adjoint_rel_l2"] = float(np.sqrt(
            np.sum(w * np.abs(mx["c"] - fp["c"]) ** 2) / np.sum(w * np.abs(fp["c"]) ** 2)))
    if not args.no_cpu_baseline:
        log(f"cpu baseline on {args.cpu_sample} points ({args.cpu_sample1} on one core)")
        cpu = cpu_baseline(cfg, alm_np, d_np, args.cpu_sample, B, args.cpu_sample1)
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
        "mixed": {"s_per_step": mx["sec"], **mx["stats"], "synthesis_stages_ms": mx["syn"],
                  "adjoint_stages_ms": mx["adj"], "plan_s": mx["plan_s"]},
        "roofline": roofline,
        "roofline_kernels": others,
        "accuracy": acc,
    }
    if fp is not None:
        out["fp64"] = {"s_per_step": fp["sec"], **fp["stats"], "eps": eps_ref,
                       "synthesis_stages_ms": fp["syn"], "adjoint_stages_ms": fp["adj"],
                       "plan_s": fp["plan_s"], "width": fp["plan"].geometry["width"],
                       "roofline": fp_roofline, "roofline_kernels": fp_others}
        out["speedup_mixed_over_fp64"] = round(fp["sec"] / mx["sec"], 3)
    if s125 is not None:
        g125 = s125["plan"].geometry
        e125 = {}
        if fp is not None:
            e125["synthesis_vs_fp64_rel_l2"] = float(
                np.linalg.norm(s125["f"] - fp["f"]) / np.linalg.norm(fp["f"]))
        if args.workload == "c3":
            e125["adjoint_vs_oracle_columns_rel"] = golden_adjoint_error(
                s125["c"], cfg["lmax"], os.path.join(ROOT, "tests", "golden",
                                                     "c3_adjoint_columns.npz"))
        out["mixed_sigma_1_25"] = {"s_per_step": s125["sec"], **s125["stats"],
                                   "steps": args.sigma125_steps, "width": g125["width"],
                                   "fine_grid": [g125["n1"], g125["n2"]],
                                   "synthesis_stages_ms": s125["syn"],
                                   "adjoint_stages_ms": s125["adj"], "accuracy": e125}
    if not args.no_spin:
        # the spin-weighted extension on the same points: two spin-2 fields, mixed precision
        for obj in (mx, fp, s125):
            if obj is not None:
                obj["plan"].close()
        torch.cuda.empty_cache()
        log("spin 2, mixed")
        sres, _, _ = spin_leg(2, 2, (("mixed", 1e-5),), args.spin_steps, 2)
        out["spin2_mixed"] = {"workload": "the C3 points (nmaps = 1 draw), two spin-2 fields",
                              "steps": args.spin_steps, **sres["mixed"]}
    if cpu is not None:
        model, ncpu = host_cpu()
        out["cpu_baseline"] = {"value": round(cpu["value"], 3), "unit": "s", "cores": cpu["threads"],
                               "kind": "oracle",
                               "sample": f"FP64 direct-sum synthesis+adjoint of 1 map on "
                                         f"{args.cpu_sample} of the {cfg['theta'].size} points, "
                                         f"scaled by N/{args.cpu_sample} x {B} maps "
                                         f"(extrapolated O(N lmax^2) direct sum)",
                               "host_cpu": model, "host_logical_cpus": ncpu,
                               "sample_s": round(cpu["sample_s"], 3),
                               "one_core_value": round(cpu["one_core"], 3),
                               "one_core_sample": f"{args.cpu_sample1} points, 1 thread, "
                                                  f"{cpu['one_core_sample_s']:.2f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
