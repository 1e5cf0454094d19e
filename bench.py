#!/usr/bin/env python3
"""Throughput of the LETKF local analysis on one MI355X.

One step = one whole analysis (observation binning, transpose, forecast
observations, localized Gram, eigensolve + transform + update, transpose
back) of a synthetic D2Q9 ensemble already resident in HBM.  Prints one JSON
line: grid-point analyses/s, per-phase GPU times from HIP events recorded on
the analysis stream, the roofline position of the dominant kernel and the
CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2308_03310_amd import synth  # noqa: E402

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0
# dense MFMA peaks of the Gram contraction by precision form
PEAK_GRAM_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def local_counts_regular(wl) -> np.ndarray:
    """Observation points within the inclusive radius 2L of every grid point of a
    regular stride mask, by enumerating lattice offsets: [ny, nx] counts."""
    s, Lr = wl.stride, wl.L
    R = int(math.floor(2 * Lr))
    per = np.zeros((s, s), dtype=np.int64)
    for ry in range(s):
        for rx in range(s):
            n = 0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if dx * dx + dy * dy <= 4 * Lr * Lr and (rx + dx) % s == 0 and (ry + dy) % s == 0:
                        n += 1
            per[ry, rx] = n
    yy, xx = np.meshgrid(np.arange(wl.ny) % s, np.arange(wl.nx) % s, indexing="ij")
    return per[yy, xx]


def algorithmic_flops(wl):
    """Per-analysis algorithmic flop counts of the two dominant kernels.

    gram: SYRK of the local perturbations, p k (k+1), plus the right-hand side 2 p k,
          with p = scalar local observations of the point;
    evd:  symmetric eigendecomposition 9 k^3 (Golub & Van Loan's count for the
          symmetric QR algorithm with eigenvectors), plus V^T b and V z (4 k^2),
          dX V and (dX V D) V^T for the nine components (36 k^2).
    """
    k = wl.k
    p = local_counts_regular(wl).astype(np.float64) * len(wl.kinds)
    gram = float(np.sum(p * (k * (k + 1) + 2 * k)))
    evd = float(wl.nx * wl.ny * (9 * k ** 3 + 40 * k ** 2))
    return {"gram": gram, "evd_update": evd}


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}@{workload}")
    except Exception:
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec.get("sha256"):
        return None
    return rec.get("bytes_per_launch")


def timed_analyses(L, torch, wl, p, precision, steps, warmup, xb=None):
    """Whole analyses of one problem at one precision form: returns (analyses/s,
    ms per analysis, per-phase ms per analysis, launches per phase, the
    analysis ensemble on the device)."""
    dev = torch.device("cuda:0")
    if xb is None:
        xb = torch.from_numpy(p.xb).to(dev)
    xa = torch.empty_like(xb)
    obs = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                (p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                                        precision=precision)], flags=L.LETKF_FLAG_PHASE_TIMING)
    try:
        io = [L.make_io(0, xb, xa, obs)]
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            L.letkf_analyze(plan, io, stream)
        torch.cuda.synchronize()
        L.letkf_phase_times(plan)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            L.letkf_analyze(plan, io, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        calls, phase_ms, launches = L.letkf_phase_times(plan)
        st = L.letkf_status(plan, sync=True)
        if st != L.LETKF_OK:
            raise SystemExit(f"{wl.name} precision {precision}: {L.letkf_strerror(st)}")
        per_call = {k: v / max(calls, 1) for k, v in phase_ms.items()}
    finally:
        L.letkf_plan_destroy(plan)
    return wl.nx * wl.ny / (ms / 1e3), ms, per_call, launches, xa


def precision_form(L, torch, steps: int):
    """The precision form on the 1024 x 1024, k = 64 workload: FP64 baseline,
    FP32 and BF16 Gram/update contractions (FP64 eigensolve and eigenvalue
    scaling in all three).  Errors are taken against the FP64 path over the
    whole field (the FP64 path itself is held to the oracle by the tests)."""
    wl = synth.WORKLOADS["grid1024_k64"]
    p = synth.make_problem(wl)
    xb = torch.from_numpy(p.xb).to(torch.device("cuda:0"))
    gram_flops = algorithmic_flops(wl)["gram"]
    res = {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "k": wl.k, "steps": steps,
           "errors": "relative L2 over every entry of the analysis ensemble, against the "
                     "FP64 path"}
    base = ref = None
    for name, prec in (("fp64", L.LETKF_PREC_FP64), ("fp32", L.LETKF_PREC_FP32),
                       ("bf16", L.LETKF_PREC_BF16)):
        rate, ms, ph, launches, xa = timed_analyses(L, torch, wl, p, prec, steps, 1, xb)
        gram_tf = gram_flops / (ph["gram"] / 1e3) / 1e12
        r = {"value": round(rate, 1), "unit": "grid-point analyses/s", "ms_per_analysis": round(ms, 3),
             "gram_ms": round(ph["gram"], 4), "evd_update_ms": round(ph["evd_update"], 3),
             "gram_tflops": round(gram_tf, 3),
             "gram_frac_of_mfma_peak": round(gram_tf / PEAK_GRAM_TFLOPS[name], 4),
             "gram_peak_tflops": PEAK_GRAM_TFLOPS[name]}
        if base is None:
            base, ref = r, xa
        else:
            r["rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(xa - ref) /
                                        torch.linalg.vector_norm(ref))
            r["increment_rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(xa - ref) /
                                                  torch.linalg.vector_norm(ref - xb))
            r["speedup_vs_fp64"] = round(rate / base["value"], 3)
            r["gram_speedup_vs_fp64"] = round(base["gram_ms"] / r["gram_ms"], 3)
            del xa
        res[name] = r
    del ref, xb
    torch.cuda.empty_cache()
    return res


def batching_form(L, torch, n: int, grids, precision: str):
    """The batching form: n independent problems drawn by the mixed-batch
    recipe (lattice sizes from grids, k from {16, 32, 64}, random masks with
    clustered gaps), in the given precision form, timed as one batched call
    with the default launch settings, after letkf_tune, and as one call per
    problem."""
    dev = torch.device("cuda:0")
    prec = {"fp64": L.LETKF_PREC_FP64, "fp32": L.LETKF_PREC_FP32, "bf16": L.LETKF_PREC_BF16}[precision]
    wls = synth.batching_workloads(n, seed=3, grids=grids)
    probs, ios, keep = [], [], []
    n_obs = []
    for i, wl in enumerate(wls):
        if i % 16 == 0:
            print(f"batching form: generating problem {i} of {n}", file=sys.stderr, flush=True)
        p = synth.make_problem(wl)
        obs = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                    (p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var))
        xb = torch.from_numpy(p.xb).to(dev)
        xa = torch.empty_like(xb)
        keep.append((xb, xa, obs))
        probs.append(L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                                    precision=prec))
        ios.append(L.make_io(i, xb, xa, obs))
        n_obs.append(len(p.obs_ix))
        del p
    points = sum(w.nx * w.ny for w in wls)
    plan = L.letkf_plan(probs)
    stream = torch.cuda.current_stream()

    def timed(calls, reps=3):
        for c in calls:                                   # warm-up
            L.letkf_analyze(plan, c, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            for c in calls:
                L.letkf_analyze(plan, c, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    try:
        ms_default = timed([ios])
        ms_single = timed([[io] for io in ios])
        tune = L.letkf_tune(plan, ios, stream)
        ms_tuned = timed([ios])
        st = L.letkf_status(plan, sync=True)
        if st != L.LETKF_OK:
            raise SystemExit(f"batching form: {L.letkf_strerror(st)}")
    finally:
        L.letkf_plan_destroy(plan)
        del keep
        torch.cuda.empty_cache()
    rate = lambda ms: round(points / (ms / 1e3), 1)
    return {"problems": n, "grids": list(grids), "precision": precision, "grid_points": points,
            "obs_per_problem": [min(n_obs), max(n_obs)],
            "batched_default": {"ms": round(ms_default, 3), "value": rate(ms_default)},
            "batched_tuned": {"ms": round(ms_tuned, 3), "value": rate(ms_tuned), "setting": tune},
            "one_call_per_problem": {"ms": round(ms_single, 3), "value": rate(ms_single)},
            "unit": "grid-point analyses/s"}


def cpu_baseline(wl, p, seconds: float):
    """The oracle, as it is, on a bounded sample of the workload's grid points."""
    from threadpoolctl import threadpool_limits
    from oracle import letkf_oracle as orc
    pts = synth.sample_points(wl.nx, wl.ny, wl.nx * wl.ny, seed=3)
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        an = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                          wl.infl)
        for q in pts:
            an.point(int(q) % wl.nx, int(q) // wl.nx)
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "grid-point analyses/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} seeded random grid points of {wl.name} (forecast observations of "
                      f"all {len(p.obs_ix)} observations included), {dt:.1f} s, 1 BLAS thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid256_k32", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests of the serving run (0 to skip)")
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB before the "
                         "timed loop (the known-size reference for HBM byte counters)")
    ap.add_argument("--batching-problems", type=int, default=64,
                    help="problems of the mixed-batch measurement (0 to skip)")
    ap.add_argument("--batching-grids", default="64,128,256",
                    help="lattice edges the mixed batch draws from")
    ap.add_argument("--batching-precision", default="fp32", choices=("fp64", "fp32", "bf16"),
                    help="precision form of the mixed batch (its recipe names the FP32 path)")
    ap.add_argument("--precision-steps", type=int, default=2,
                    help="timed analyses per precision form on the 1024^2, k = 64 workload "
                         "(0 to skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the analysis is measured on one MI355X; see DESIGN.md for how it shards)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_03310_amd import letkf as L

    wl = synth.WORKLOADS[args.workload]
    p = synth.make_problem(wl)
    npts = wl.nx * wl.ny
    dev = torch.device("cuda:0")
    xb = torch.from_numpy(p.xb).to(dev)
    xa = torch.empty_like(xb)
    obs = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                (p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl)],
                        flags=L.LETKF_FLAG_PHASE_TIMING)
    io = [L.make_io(0, xb, xa, obs)]
    stream = torch.cuda.current_stream()
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 17            # doubles
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        L.letkf_analyze(plan, io, stream)
    torch.cuda.synchronize()
    L.letkf_phase_times(plan)                     # drop the warm-up calls
    st = L.letkf_status(plan, sync=True)
    if st != L.LETKF_OK:
        raise SystemExit(f"warm-up analysis failed: {L.letkf_strerror(st)}")

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L.letkf_analyze(plan, io, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    calls, phase_ms, launches = L.letkf_phase_times(plan)
    st = L.letkf_status(plan, sync=True)
    L.letkf_plan_destroy(plan)
    if st != L.LETKF_OK:
        raise SystemExit(f"timed analysis failed: {L.letkf_strerror(st)}")
    ms_step = ms_total / args.steps
    value = npts * args.steps / (ms_total / 1e3)

    flops = algorithmic_flops(wl)
    per_call = {k: v / max(calls, 1) for k, v in phase_ms.items()}
    kernels = {}
    for ph, bound in (("gram", "mfma"), ("evd_update", "alu")):
        n_l = max(launches[ph], 1)
        ms_launch = per_call[ph] / n_l
        ach = flops[ph] / n_l / (ms_launch / 1e3) / 1e12
        kernels[ph] = {"bound": bound, "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                       "ms_per_launch": round(ms_launch, 4), "launches_per_step": n_l,
                       "flops_per_launch": flops[ph] / n_l}
    dom = max(kernels, key=lambda ph: per_call[ph])
    kname = {"gram": "k_gram_f64", "evd_update": "k_evd"}[dom]
    roof = {k: kernels[dom][k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof["kernel"] = kname
    roof["traffic"] = stored_traffic(kname, wl.name)

    out = {
        "metric": "LETKF grid-point analyses/s",
        "value": round(value, 1),
        "unit": "grid-point analyses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "k": wl.k,
                   "obs_stride": wl.stride, "obs_kinds": "u,v", "n_obs": int(len(p.obs_ix)),
                   "L": wl.L, "infl": wl.infl, "sigma": wl.sigma, "precision": "fp64",
                   "localization": "gauss(2L cutoff)"},
        "roofline": roof,
        "kernels": kernels,
        "phases_ms_per_step": {k: round(v, 4) for k, v in per_call.items()},
        "host_wall_s": round(wall, 3),
    }
    if args.serving_requests > 0:
        from paper_2308_03310_amd import serving
        srv = serving.AssimilationServer(serving.default_specs(16), budget_bytes=200 << 30,
                                         n_slots=8)
        try:
            srv.run_poisson(args.serving_rate, 16, seed=40)       # warm-up: admit every session
            out["serving"] = srv.run_poisson(args.serving_rate, args.serving_requests, seed=4)
            out["serving"]["sessions"] = len(srv.sessions)
            out["serving"]["cycle"] = "50 BGK steps (tau 0.52, Kolmogorov forcing 1e-5) + analysis"
        finally:
            srv.close()
    if args.precision_steps > 0 or args.batching_problems > 0:
        del xb, xa, obs
        torch.cuda.empty_cache()
    if args.precision_steps > 0:
        out["precision_form"] = precision_form(L, torch, args.precision_steps)
    if args.batching_problems > 0:
        out["batching_form"] = batching_form(L, torch, args.batching_problems,
                                             tuple(int(g) for g in args.batching_grids.split(",")),
                                             args.batching_precision)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
