#!/usr/bin/env python3
"""Throughput of the LETKF local analysis on one MI355X: mixed precision
against plain FP64.

One step = one whole analysis (observation binning, transpose, forecast
observations, localized Gram, eigensolve + transform + update, transpose
back) of the 1024 x 1024, k = 64 synthetic D2Q9 ensemble, already resident in
HBM.  The headline `value` is the mixed-precision form (Gram and update
contractions in FP32 on MFMA with FP32 accumulation, FP64 eigensolve and
eigenvalue scaling); the same K steps are timed in the plain FP64 form and
the BF16 form, and their ratio is reported.  Prints one JSON line with
per-phase GPU times from HIP events recorded on the analysis stream, the
roofline position of the dominant kernel, each form's error against the FP64
oracle at sampled grid points (whole, mean, spread), the oracle's own rate on
the host's cores, and the secondary measurements: the 256 x 256, k = 32 FP64
workload, the batched eigensolve at the shapes of the paper's Table I, the
serving run and the batching form.
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
FORMS = (("fp64", 0), ("fp32", 1), ("bf16", 2))
KERNEL_NAMES = {"gram": {"fp64": "k_gram_f64", "fp32": "k_gram_lp", "bf16": "k_gram_lp"},
                "evd_update": "k_evd_xf", "fused": "k_fused"}
# Batched EVD of 16,384 matrices from the LBM-LETKF model on one A100 (FP32,
# the paper's Table I, EigenG column): context for the eigensolve record.
PAPER_TABLE1_EIGENG_MS = {16: 1.3, 32: 2.4, 48: 7.8, 64: 14.2}


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
    """Per-analysis algorithmic flop counts of the two dominant kernels, per
    grid point:

    gram:       SYRK of the local perturbations p k (k+1) plus the right-hand
                side 2 p k, p = scalar local observations of the point;
    evd_update: symmetric eigendecomposition with vectors 9 k^3 (Golub & Van
                Loan's count), the transform V diag V^T of the symmetric square
                root 2 k^3 + 4 k^2, and the update of the nine components
                2 * 9 k^2.
    """
    k = wl.k
    p = local_counts_regular(wl).astype(np.float64) * len(wl.kinds)
    gram = float(np.sum(p * (k * (k + 1) + 2 * k)))
    evd = float(wl.nx * wl.ny * (11 * k ** 3 + 22 * k ** 2))
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


def dev_obs(torch, p, dev):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
                 (p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var))


def timed_analyses(L, torch, wl, xb, obs, precision, steps, warmup, flags=0, form=None):
    """steps whole analyses of one problem in one precision form on torch's
    current stream, bracketed by synchronizations: returns (analyses/s, ms per
    analysis, per-phase ms per analysis, launches per phase, the analysis).
    form: a kernel form (LETKF_FORM_*) set on the plan, else its default."""
    xa = torch.empty_like(xb)
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, int(obs[0].numel()), wl.L, wl.infl,
                                        precision=precision)],
                        flags=L.LETKF_FLAG_PHASE_TIMING | flags)
    try:
        if form is not None:
            L.letkf_set_tuning(plan, 8, form)
        io = [L.make_io(0, xb, xa, obs)]
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            L.letkf_analyze(plan, io, stream)
        torch.cuda.synchronize()
        L.letkf_phase_times(plan)                      # drop the warm-up calls
        st = L.letkf_status(plan, sync=True)
        if st != L.LETKF_OK:
            raise SystemExit(f"{wl.name} precision {precision} warm-up: {L.letkf_strerror(st)}")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
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


def kernel_roofline(wl, form, per_call, launches):
    """Achieved rate of the Gram and eigensolve/update kernels (split forms)
    or of the fused kernel: algorithmic flops per launch over the average
    launch time from the HIP events.  The fused kernel does both kinds of
    work, so its peak is the rate at which it would finish both at their own
    peaks: (F_gram + F_evd) / (F_gram / P_gram + F_evd / P_fp64) -- the FP64
    peak itself in the FP64 form."""
    flops = algorithmic_flops(wl)
    out = {}
    if launches.get("fused", 0) > 0:
        fg, fe = flops["gram"], flops["evd_update"]
        peak = (fg + fe) / (fg / PEAK_GRAM_TFLOPS[form] + fe / PEAK_FP64_TFLOPS)
        phases = (("fused", "alu", round(peak, 3), fg + fe),)
    else:
        phases = (("gram", "mfma", PEAK_GRAM_TFLOPS[form], flops["gram"]),
                  ("evd_update", "alu", PEAK_FP64_TFLOPS, flops["evd_update"]))
    for ph, bound, peak, fl in phases:
        n_l = max(launches[ph], 1)
        ms_launch = per_call[ph] / n_l
        ach = fl / n_l / (ms_launch / 1e3) / 1e12
        name = KERNEL_NAMES[ph][form] if isinstance(KERNEL_NAMES[ph], dict) else KERNEL_NAMES[ph]
        out[ph] = {"kernel": name, "bound": bound, "achieved": round(ach, 3), "peak": peak,
                   "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                   "ms_per_launch": round(ms_launch, 4), "launches_per_step": n_l,
                   "flops_per_launch": fl / n_l}
    return out


def oracle_errors(wl, p, xa, refs):
    """Errors of an analysis against the FP64 oracle at the seeded sample
    points whose oracle values the CPU-baseline leg computed (refs = (points,
    [n, k, 9] values)): relative L2 of the whole, of the increment, of the
    analysis mean and of the spread, and the largest error of one point
    relative to its norm."""
    pts, ref = refs
    iy, ix = pts // wl.nx, pts % wl.nx
    got = np.moveaxis(xa[:, :, iy, ix].cpu().numpy(), -1, 0)        # [n, k, 9]
    xb = np.moveaxis(p.xb[:, :, iy, ix], -1, 0)
    d = got - ref
    gm, rm = got.mean(axis=1, keepdims=True), ref.mean(axis=1, keepdims=True)
    pt = np.linalg.norm(d.reshape(len(pts), -1), axis=1) / np.linalg.norm(
        ref.reshape(len(pts), -1), axis=1)
    return {"points": int(len(pts)),
            "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "increment_rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref - xb)),
            "mean_rel_l2": float(np.linalg.norm(gm - rm) / np.linalg.norm(rm)),
            "spread_rel_l2": float(np.linalg.norm((got - gm) - (ref - rm)) /
                                   np.linalg.norm(ref - rm)),
            "max_point_rel": float(pt.max())}


def eigh_table1(L, torch, batch=16384, ks=(16, 32, 48, 64), reps=10):
    """The standalone batched eigensolve at the shapes of the paper's Table I
    (16,384 matrices per batch): LETKF-form matrices ((k-1)/rho) I + Y^T Y
    with Y of 2k centred rows (cond about 1.05); beside it the Newton-Schulz
    inverse square root (the transform's other route, no EVD) of the same
    matrices and of a spread family whose Y^T Y is scaled to cond(Q) = 1e3
    (the step count of the iteration grows with cond, the EVD's does not)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(7)
    out = {"batch": batch, "unit": "ns per matrix", "precision": "fp64",
           "context": "paper Table I (EigenG, FP32, one A100), ms per 16,384 matrices"}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    st = torch.zeros(1, dtype=torch.int32, device=dev)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        if int(st.item()) != 0:
            raise SystemExit(f"k={k}: not converged")
        return e0.elapsed_time(e1) / reps

    for k in ks:
        Y = torch.randn(batch, 2 * k, k, generator=g, device=dev, dtype=torch.float64)
        Y = Y - Y.mean(dim=2, keepdim=True)
        C = torch.matmul(Y.transpose(1, 2).contiguous(), Y) * (1.0 / (2 * k))
        del Y
        eye = (k - 1) / 1.1 * torch.eye(k, device=dev, dtype=torch.float64)
        lam = torch.empty(batch, k, dtype=torch.float64, device=dev)
        vec = torch.empty(batch, k, k, dtype=torch.float64, device=dev)
        xs = torch.empty(batch, k, k, dtype=torch.float64, device=dev)
        nst = torch.empty(batch, dtype=torch.int32, device=dev)
        i = torch.arange(0, batch, batch // 8, device=dev)
        rec = {}
        for fam in ("table1", "cond1e3"):
            if fam == "table1":
                A = (C + eye).contiguous()
            else:
                lmax = torch.linalg.eigvalsh(C[:64]).amax(dim=1).mean()
                A = (C * ((1e3 - 1.0) * (k - 1) / 1.1 / lmax) + eye).contiguous()
            ms = timed(lambda: L.letkf_eigh_batched(A, lam, vec, st))
            R = torch.matmul(vec[i] * lam[i][:, None, :], vec[i].transpose(1, 2).contiguous()) - A[i]
            res = float((torch.linalg.matrix_norm(R) / torch.linalg.matrix_norm(A[i])).max())
            cond = float((lam[i].amax(dim=1) / lam[i].amin(dim=1)).median())
            tf = 9 * k ** 3 * batch / (ms / 1e3) / 1e12
            ms_ns = timed(lambda: L.letkf_invsqrt_batched(A, xs, st, nst))
            steps = float(nst.double().mean())
            R = torch.matmul(vec[i] * lam[i].rsqrt()[:, None, :], vec[i].transpose(1, 2).contiguous())
            dif = float((torch.linalg.matrix_norm(xs[i] - R) / torch.linalg.matrix_norm(R)).max())
            tf_ns = 6 * k ** 3 * steps * batch / (ms_ns / 1e3) / 1e12
            r = {"median_cond": round(cond, 3),
                 "eigh": {"ms": round(ms, 4), "ns_per_matrix": round(ms * 1e6 / batch, 1),
                          "tflops_9k3": round(tf, 3),
                          "frac_fp64_peak": round(tf / PEAK_FP64_TFLOPS, 4),
                          "max_rel_residual": res},
                 "nsqrt": {"ms": round(ms_ns, 4), "ns_per_matrix": round(ms_ns * 1e6 / batch, 1),
                           "mean_steps": round(steps, 2), "tflops_6k3_per_step": round(tf_ns, 3),
                           "frac_fp64_peak": round(tf_ns / PEAK_FP64_TFLOPS, 4),
                           "speedup_vs_eigh": round(ms / ms_ns, 3),
                           "max_rel_diff_vs_evd_form": dif}}
            rec[fam] = r
            del A
        # the Table I record keeps its flat keys (the EVD on the Table I form)
        t1 = rec["table1"]["eigh"]
        out[f"k{k}"] = dict(t1, paper_a100_fp32_ms=PAPER_TABLE1_EIGENG_MS.get(k),
                            nsqrt=rec["table1"]["nsqrt"], cond1e3=rec["cond1e3"])
        del C, lam, vec, xs, nst
    torch.cuda.empty_cache()
    return out


def batching_form(L, torch, n: int, grids, precision: str, reps: int, tune: bool):
    """The batching form: n independent problems drawn by the mixed-batch
    recipe (lattice sizes from grids, k from {16, 32, 64}, random masks with
    clustered gaps), in the given precision form, timed as one batched call
    and as one call per problem (and after letkf_tune when asked).  The
    ensembles are generated on the device by the recipe's generator."""
    dev = torch.device("cuda:0")
    prec = dict(FORMS)[precision]
    wls = synth.batching_workloads(n, seed=3, grids=grids)
    probs, ios, keep, n_obs = [], [], [], []
    for i, wl in enumerate(wls):
        if i % 8 == 0:
            print(f"batching form: generating problem {i} of {n}", file=sys.stderr, flush=True)
        xb, p = synth.make_problem_device(wl, dev)
        obs = dev_obs(torch, p, dev)
        xa = torch.empty_like(xb)
        keep.append((xb, xa, obs))
        probs.append(L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                                    precision=prec))
        ios.append(L.make_io(i, xb, xa, obs))
        n_obs.append(len(p.obs_ix))
    points = sum(w.nx * w.ny for w in wls)
    plan = L.letkf_plan(probs)
    stream = torch.cuda.current_stream()

    def timed(calls):
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
        print("batching form: timing one batched call", file=sys.stderr, flush=True)
        ms_batched = timed([ios])
        print("batching form: timing one call per problem", file=sys.stderr, flush=True)
        ms_single = timed([[io] for io in ios])
        out = {"problems": n, "grids": list(grids), "precision": precision, "grid_points": points,
               "obs_per_problem": [min(n_obs), max(n_obs)], "reps": reps}
        if tune:
            setting = L.letkf_tune(plan, ios, stream)
            out["batched_tuned"] = {"ms": round(timed([ios]), 3), "setting": setting}
        st = L.letkf_status(plan, sync=True)
        if st != L.LETKF_OK:
            raise SystemExit(f"batching form: {L.letkf_strerror(st)}")
    finally:
        L.letkf_plan_destroy(plan)
        del keep
        torch.cuda.empty_cache()
    rate = lambda ms: round(points / (ms / 1e3), 1)
    out["batched"] = {"ms": round(ms_batched, 3), "value": rate(ms_batched)}
    out["one_call_per_problem"] = {"ms": round(ms_single, 3), "value": rate(ms_single)}
    out["batched_speedup"] = round(ms_single / ms_batched, 3)
    out["unit"] = "grid-point analyses/s"
    return out


_ORACLE = None     # the oracle's Analysis, inherited by the forked workers


def _oracle_worker(args):
    pts, nx, seconds = args
    from threadpoolctl import threadpool_limits
    an = _ORACLE
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for q in pts:
            an.point(int(q) % nx, int(q) // nx)
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return done, dt


def cpu_baseline(wl, p, seconds: float, max_cores: int, error_points: int):
    """The oracle, as it is, on a bounded sample of the workload's grid points:
    one process with one BLAS thread, then one such process per host core
    (forked after the forecast observations are computed, so every process
    evaluates points of the same analysis; the workers inherit it rather than
    receive a copy).  Runs before the GPU is initialised, so the forks carry
    no device state.  Also returns the oracle's values at error_points seeded
    points (points, [n, k, 9]), the references the GPU forms are checked
    against; this leg is the only one that runs the oracle."""
    import multiprocessing as mp
    from oracle import letkf_oracle as orc
    global _ORACLE
    pts = synth.sample_points(wl.nx, wl.ny, min(wl.nx * wl.ny, 200000), seed=3)
    _ORACLE = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                           wl.infl)
    refs = None
    if error_points > 0:
        rp = synth.sample_points(wl.nx, wl.ny, error_points, seed=11)
        print(f"oracle values at {len(rp)} sample points", file=sys.stderr, flush=True)
        refs = (rp, _ORACLE.run(rp))
    print(f"cpu baseline: oracle on 1 core for {seconds:.0f} s", file=sys.stderr, flush=True)
    done1, dt1 = _oracle_worker((pts, wl.nx, seconds))
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0))))
    chunks = [pts[i::cores] for i in range(cores)]
    print(f"cpu baseline: oracle on {cores} processes for {seconds:.0f} s", file=sys.stderr,
          flush=True)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(c, wl.nx, seconds) for c in chunks])
    _ORACLE = None
    done_n = sum(r[0] for r in res)
    rate_n = sum(r[0] / r[1] for r in res)
    return refs, {"value": rate_n, "unit": "grid-point analyses/s", "cores": cores, "kind": "oracle",
            "single_core_value": done1 / dt1,
            "sample": f"seeded random grid points of {wl.name} (forecast observations of all "
                      f"{len(p.obs_ix)} observations computed first): {done1} points in "
                      f"{dt1:.1f} s on 1 core; {done_n} points in about {seconds:.0f} s on "
                      f"{cores} processes of 1 BLAS thread each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid1024_k64", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=("fp32", "bf16"),
                    help="the mixed form of the headline value")
    ap.add_argument("--forms", default="fp64,fp32,bf16",
                    help="precision forms timed (the headline's and fp64 are always included)")
    ap.add_argument("--error-points", type=int, default=24,
                    help="sample points at which each form is compared with the oracle (0: "
                         "skip; the oracle runs in the CPU-baseline leg, which "
                         "--no-cpu-baseline skips with them)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-cores", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--secondary-steps", type=int, default=10,
                    help="timed steps of the 256^2, k = 32 FP64 workload (0 to skip)")
    ap.add_argument("--kernel-form", default="auto", choices=("auto", "grid", "persistent", "fused"),
                    help="kernel form of every timed analysis of the workload (auto: the library's "
                         "default, fused at k = 64)")
    ap.add_argument("--split-steps", type=int, default=3,
                    help="analyses timed in the split kernel form (Gram and eigensolve "
                         "launches per slab) for the FP64 and headline forms (0: skip)")
    ap.add_argument("--nsqrt-steps", type=int, default=3,
                    help="analyses timed with the Newton-Schulz route to the transform "
                         "(LETKF_FLAG_NSQRT, FP64 form) beside the EVD route (0: skip)")
    ap.add_argument("--eigh-reps", type=int, default=10,
                    help="timed batches of the Table I eigensolve shapes (0 to skip)")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="requests of the serving run (0 to skip)")
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB before the "
                         "timed loop (the known-size reference for HBM byte counters)")
    ap.add_argument("--batching-problems", type=int, default=256,
                    help="problems of the mixed-batch measurement (0 to skip)")
    ap.add_argument("--batching-grids", default="64,128,256,512",
                    help="lattice edges the mixed batch draws from")
    ap.add_argument("--batching-precision", default="fp32", choices=("fp64", "fp32", "bf16"),
                    help="precision form of the mixed batch (its recipe names the FP32 path)")
    ap.add_argument("--batching-reps", type=int, default=2)
    ap.add_argument("--twin-cycles", type=int, default=24,
                    help="cycles of the twin experiment on the 256 x 256, k = 32 workload (0: skip)")
    ap.add_argument("--batching-small-problems", type=int, default=256,
                    help="problems of the small-lattice batch (64 x 64 only; 0: skip)")
    ap.add_argument("--batching-tune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the analysis is measured on one MI355X; DESIGN.md describes how it shards)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_03310_amd import letkf as L

    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS[args.workload]
    print(f"generating {wl.name}", file=sys.stderr, flush=True)
    p = synth.make_problem(wl)
    cpu = refs = None
    if not args.no_cpu_baseline:
        refs, cpu = cpu_baseline(wl, p, args.cpu_seconds, args.cpu_cores, args.error_points)
    xb = torch.from_numpy(p.xb).to(dev)
    obs = dev_obs(torch, p, dev)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 17            # doubles
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    kform = {"auto": L.LETKF_FORM_AUTO, "grid": L.LETKF_FORM_GRID,
             "persistent": L.LETKF_FORM_PERSISTENT, "fused": L.LETKF_FORM_FUSED}[args.kernel_form]
    forms = [f for f, _ in FORMS if f in set(args.forms.split(",")) | {"fp64", args.precision}]
    res = {}
    wall0 = time.perf_counter()
    for name in forms:
        print(f"timing the {name} form", file=sys.stderr, flush=True)
        rate, ms, ph, launches, xa = timed_analyses(L, torch, wl, xb, obs, dict(FORMS)[name],
                                                    args.steps, args.warmup, form=kform)
        r = {"value": round(rate, 1), "ms_per_analysis": round(ms, 3),
             "phases_ms": {k: round(v, 4) for k, v in ph.items()},
             "kernels": kernel_roofline(wl, name, ph, launches)}
        if refs is not None:
            r["errors_vs_oracle"] = oracle_errors(wl, p, xa, refs)
        del xa
        res[name] = r
    wall = time.perf_counter() - wall0
    nsq = None
    if args.nsqrt_steps > 0:
        print("timing the FP64 form with the Newton-Schulz transform", file=sys.stderr, flush=True)
        rate, ms, ph, launches, xa = timed_analyses(L, torch, wl, xb, obs, 0, args.nsqrt_steps, 1,
                                                    L.LETKF_FLAG_NSQRT)
        nsq = {"value": round(rate, 1), "ms_per_analysis": round(ms, 3),
               "phases_ms": {k: round(v, 4) for k, v in ph.items()},
               "evd_route_fp64_ms": res["fp64"]["ms_per_analysis"],
               "speedup_vs_evd_route": round(res["fp64"]["ms_per_analysis"] / ms, 3)}
        if refs is not None:
            nsq["errors_vs_oracle"] = oracle_errors(wl, p, xa, refs)
        del xa
    # the split kernel form (a Gram and an eigensolve launch per slab) of the
    # FP64 form and the headline form: the per-kernel breakdown the fused
    # launch cannot give, and the fused form's gain over it
    split = {}
    for name in (["fp64", args.precision] if args.split_steps > 0 else []):
        if name in split:
            continue
        print(f"timing the {name} form, split kernels", file=sys.stderr, flush=True)
        rate, ms, ph, launches, xa = timed_analyses(L, torch, wl, xb, obs, dict(FORMS)[name],
                                                    args.split_steps, 1, form=L.LETKF_FORM_GRID)
        del xa
        split[name] = {"value": round(rate, 1), "ms_per_analysis": round(ms, 3),
                       "phases_ms": {k: round(v, 4) for k, v in ph.items()},
                       "kernels": kernel_roofline(wl, name, ph, launches),
                       "speedup_of_timed_form": round(ms / res[name]["ms_per_analysis"], 3)}
    if "fp64" in split and args.precision in split and args.precision != "fp64":
        split[args.precision]["gram_speedup_vs_fp64"] = round(
            split["fp64"]["phases_ms"]["gram"] / split[args.precision]["phases_ms"]["gram"], 3)
    head = res[args.precision]
    base = res["fp64"]
    for name in forms:
        if name != "fp64":
            res[name]["speedup_vs_fp64"] = round(res[name]["value"] / base["value"], 3)

    dom = max(head["kernels"], key=lambda ph: head["phases_ms"][ph])
    kd = head["kernels"][dom]
    roof = {k: kd[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof["kernel"] = kd["kernel"]
    roof["traffic"] = stored_traffic(kd["kernel"], f"{wl.name}_{args.precision}")

    out = {
        "metric": "LETKF grid-point analyses/s, mixed vs FP64 plain",
        "value": head["value"],
        "unit": "grid-point analyses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_analysis"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.precision}+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "k": wl.k,
                   "obs_stride": wl.stride, "obs_kinds": "u,v", "n_obs": int(len(p.obs_ix)),
                   "L": wl.L, "infl": wl.infl, "sigma": wl.sigma,
                   "precision": f"{args.precision} Gram/update contractions (FP32 accumulation), "
                                f"fp64 eigensolve and eigenvalue scaling",
                   "localization": "gauss(2L cutoff)",
                   "kernel_form": "auto: fused at this width (Gram, eigensolve, transform "
                                  "and update of every point in one persistent launch)"
                                  if args.kernel_form == "auto" else args.kernel_form},
        "speedup_vs_fp64": head["speedup_vs_fp64"],
        "fp64_value": base["value"],
        "roofline": roof,
        "forms": res,
        "split_kernel_form": split,
        "host_wall_s": round(wall, 3),
    }
    if nsq is not None:
        out["nsqrt_route_fp64"] = nsq
    del xb, obs
    torch.cuda.empty_cache()
    if args.secondary_steps > 0:
        print("timing the 256 x 256, k = 32 FP64 workload", file=sys.stderr, flush=True)
        w2 = synth.WORKLOADS["grid256_k32"]
        p2 = synth.make_problem(w2)
        xb2 = torch.from_numpy(p2.xb).to(dev)
        rate, ms, ph, launches, xa2 = timed_analyses(L, torch, w2, xb2, dev_obs(torch, p2, dev), 0,
                                                     args.secondary_steps, 2)
        out["grid256_k32_fp64"] = {"value": round(rate, 1), "ms_per_analysis": round(ms, 4),
                                   "phases_ms": {k: round(v, 4) for k, v in ph.items()},
                                   "kernels": kernel_roofline(w2, "fp64", ph, launches)}
        del xb2, xa2
        torch.cuda.empty_cache()
    if args.eigh_reps > 0:
        print("batched eigensolve at the Table I shapes", file=sys.stderr, flush=True)
        out["eigh_table1"] = eigh_table1(L, torch, reps=args.eigh_reps)
    if args.serving_requests > 0:
        from paper_2308_03310_amd import serving
        print("serving", file=sys.stderr, flush=True)
        specs = serving.default_specs(12)
        srv = serving.AssimilationServer(specs, budget_bytes=200 << 30, n_slots=8)
        try:
            for i in range(len(specs)):                   # warm-up: admit every session once
                srv.submit(serving.Request(i, i, time.perf_counter()))
            srv.drain()
            out["serving"] = srv.run_poisson(args.serving_rate, args.serving_requests, seed=4)
            out["serving"]["sessions"] = [s.spec.name for s in srv.sessions]
            out["serving"]["cycle"] = "50 BGK steps (tau 0.52, Kolmogorov forcing 1e-5) + analysis"
            # the offered rate above is several times what one GPU serves, so
            # its p50 / p99 are queueing delays; the same mix offered at 80 %
            # of the throughput just measured gives the service latency
            cap = out["serving"]["throughput_cycles_per_s"]
            if cap > 0:
                out["serving_sustainable"] = srv.run_poisson(0.8 * cap, args.serving_requests // 2,
                                                             seed=6)
            # a budget that holds about a third of the sessions: admissions evict
            fp = sorted((s.footprint() for s in srv.sessions), reverse=True)
            srv.close()
            tight = fp[0] + sum(fp[1:]) // 3
            srv = serving.AssimilationServer(specs, budget_bytes=tight, n_slots=8)
            out["serving_tight_budget"] = srv.run_poisson(args.serving_rate,
                                                          args.serving_requests // 2, seed=5)
        finally:
            srv.close()
            torch.cuda.empty_cache()
    if args.batching_problems > 0:
        out["batching_form"] = batching_form(L, torch, args.batching_problems,
                                             tuple(int(g) for g in args.batching_grids.split(",")),
                                             args.batching_precision, args.batching_reps,
                                             args.batching_tune)
    if args.twin_cycles > 0:
        # the cycled twin experiment on the 256 x 256, k = 32 workload: a nature
        # run of the forced BGK model, its (u, v) observed every cycle
        from paper_2308_03310_amd import twin
        print(f"twin experiment, {args.twin_cycles} cycles", file=sys.stderr, flush=True)
        tw = twin.run_twin(twin.TwinConfig(synth.WORKLOADS["grid256_k32"], n_cycles=args.twin_cycles,
                                           n_steps=50), dev)
        r3 = lambda xs: [float(f"{x:.3g}") for x in xs]
        out["twin"] = dict(tw["summary"], forecast_rmse=r3(tw["forecast_rmse"]),
                           analysis_rmse=r3(tw["analysis_rmse"]), free_rmse=r3(tw["free_rmse"]),
                           spread=r3(tw["spread"]),
                           all_status_ok=all(s_ == L.LETKF_OK for s_ in tw["status"]))
        torch.cuda.empty_cache()
    if args.batching_small_problems > 0:
        # the same recipe restricted to 64 x 64 lattices: problems too small to
        # fill the device alone, where one call each leaves it idle between
        # launches and a batched call does not
        print("batching form, small problems", file=sys.stderr, flush=True)
        out["batching_form_small"] = batching_form(L, torch, args.batching_small_problems, (64,),
                                                   args.batching_precision, args.batching_reps,
                                                   False)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
