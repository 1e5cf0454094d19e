"""Cycled twin experiment (Sec. II-B DA cycle on a synthetic nature run):
forecast with letkf_advance, analysis with letkf_analyze, observations drawn
from the truth every cycle.  The filter must do what a filter does: while the
ensemble error is well above its converged level the analysis lowers it every
cycle, on average it stays below the forecast error, and the cycled ensemble
ends far below a free-running ensemble started from the same members; every
cycle's device status is clean.  (Once converged, a single cycle's analysis
can land a hair above its forecast: the observation noise is larger than the
error left, so the per-cycle ordering is a statistical, not a strict, one.)"""
import sys

import numpy as np
import pytest

from paper_2308_03310_amd import synth, twin
from paper_2308_03310_amd import letkf as L

pytestmark = pytest.mark.gpu


def test_twin_experiment_reduces_error(device):
    wl = synth.Workload("twin64_k16", 64, 64, 16, 2, 0.005, 4.0, 1.1, 7)
    cfg = twin.TwinConfig(wl, n_cycles=24, n_steps=20)
    print(f"twin: {wl.nx}x{wl.ny} k={wl.k}, {cfg.n_cycles} cycles x {cfg.n_steps} steps", flush=True)
    out = twin.run_twin(cfg, device)
    sys.stdout.flush()
    fc, an, fr = (np.array(out[k]) for k in ("forecast_rmse", "analysis_rmse", "free_rmse"))
    print("forecast", np.round(fc, 6), "\nanalysis", np.round(an, 6), "\nfree", np.round(fr, 6),
          flush=True)
    assert all(s == L.LETKF_OK for s in out["status"])
    assert np.all(an[:4] < fc[:4])
    s = out["summary"]
    assert s["mean_analysis_rmse_2nd_half"] < s["mean_forecast_rmse_2nd_half"]
    assert an[-1] < 0.5 * fr[-1]
    assert s["mean_analysis_rmse_2nd_half"] < 0.5 * s["mean_free_rmse_2nd_half"]
    # the analysis error sits near the observation noise, not far above it
    assert s["mean_analysis_rmse_2nd_half"] < 2.0 * wl.sigma


def test_advance_matches_cycle_without_analysis(device):
    """letkf_advance equals the model part of letkf_cycle bit for bit: a cycle
    whose observation is rejected on the device keeps the advanced state."""
    import torch
    wl = synth.WORKLOADS["cpu32_k16"]
    p = synth.make_problem(wl)
    x0 = torch.from_numpy(p.xb).to(device)
    a = x0.clone()
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, 1, wl.L, wl.infl)],
                        flags=L.LETKF_FLAG_CYCLE)
    try:
        for n in (1, 2, 3):
            a.copy_(x0)
            L.letkf_advance(plan, [L.make_cycle_io(0, a, None, n)])
            b = x0.clone()
            bad = (torch.tensor([wl.nx + 5], dtype=torch.int32, device=device),
                   torch.tensor([0], dtype=torch.int32, device=device),
                   torch.tensor([1], dtype=torch.int32, device=device),
                   torch.tensor([0.0], dtype=torch.float64, device=device),
                   torch.tensor([1e-4], dtype=torch.float64, device=device))
            L.letkf_cycle(plan, [L.make_cycle_io(0, b, bad, n)])
            st = L.letkf_status(plan, sync=True)
            assert st == L.LETKF_EINVAL
            assert torch.equal(a, b), f"n_steps {n}"
            assert not torch.equal(a, x0)
    finally:
        L.letkf_plan_destroy(plan)
