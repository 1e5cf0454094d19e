"""Cycled twin experiment through the library (an analogue of the paper's
OSSE, Sec. V, on synthetic data): a nature run of the forced lattice-BGK
model, observations of it drawn every cycle, and an ensemble cycled with the
forecast (letkf_advance) and the analysis (letkf_analyze) -- the DA cycle of
Sec. II-B.  Reports, per cycle, the forecast and analysis RMSE of the
ensemble-mean velocity against the truth, the ensemble spread, and the RMSE
of a free-running ensemble started from the same members and never analysed.

Every model step and analysis runs in the library's kernels; this module only
draws the observation noise and evaluates the diagnostics (velocity moments
of ensemble means) with torch on the device.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import letkf as L
from . import synth


@dataclasses.dataclass
class TwinConfig:
    wl: synth.Workload            # lattice, ensemble size, observation lattice, L, rho, sigma
    n_cycles: int = 24
    n_steps: int = 50             # BGK steps per forecast
    tau: float = 0.52
    force_amp: float = 1e-5
    force_kx: int = 4
    seed: int = 4                 # observation-noise draws


def _velocity(torch, f):
    """(u, v) of the D2Q9 populations f [..., 9, ny, nx] (moments, FP64)."""
    cx = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=f.dtype, device=f.device)
    cy = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=f.dtype, device=f.device)
    rho = f.sum(dim=-3)
    u = (f * cx[:, None, None]).sum(dim=-3) / rho
    v = (f * cy[:, None, None]).sum(dim=-3) / rho
    return u, v


def _rmse(torch, u, v, ut, vt) -> float:
    """Root-mean-square velocity error over every grid point and both components."""
    return float(torch.sqrt(0.5 * torch.mean((u - ut) ** 2 + (v - vt) ** 2)))


def _mean_velocity(torch, ens):
    return _velocity(torch, ens.mean(dim=0))


def run_twin(cfg: TwinConfig, device=None, stream=None) -> dict:
    """The twin experiment of cfg on one GPU; returns per-cycle diagnostics."""
    import torch
    dev = device or torch.device("cuda:0")
    wl = cfg.wl
    p = synth.make_problem(wl)
    # nature run: the truth the members scatter around, at uniform density; a
    # two-member "ensemble" of identical copies, advanced by the same kernel
    rho1 = np.ones((wl.ny, wl.nx))
    ft = synth.equilibrium(rho1, p.truth_u, p.truth_v)
    truth = torch.from_numpy(np.stack([ft, ft])).to(dev)
    ens = torch.from_numpy(p.xb).to(dev)
    free = ens.clone()
    # observation lattice of the workload (its stride), u and v at each point
    obs_ix = torch.from_numpy(p.obs_ix).to(dev)
    obs_iy = torch.from_numpy(p.obs_iy).to(dev)
    obs_kind = torch.from_numpy(p.obs_kind).to(dev)
    obs_var = torch.from_numpy(p.obs_var).to(dev)
    n_obs = int(obs_ix.numel())
    gen = torch.Generator(device=dev).manual_seed(cfg.seed)
    plan_t = L.letkf_plan([L.make_problem(wl.nx, wl.ny, 2, 0, wl.L, 1.0)], flags=L.LETKF_FLAG_CYCLE)
    plan_e = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, n_obs, wl.L, wl.infl)],
                          flags=L.LETKF_FLAG_CYCLE)
    adv = lambda x: L.make_cycle_io(0, x, None, cfg.n_steps, cfg.tau, cfg.force_amp, cfg.force_kx)
    out = {"cycles": [], "forecast_rmse": [], "analysis_rmse": [], "free_rmse": [],
           "spread": [], "status": []}
    try:
        for c in range(cfg.n_cycles):
            L.letkf_advance(plan_t, [adv(truth)], stream)
            L.letkf_advance(plan_e, [adv(ens)], stream)
            L.letkf_advance(plan_e, [adv(free)], stream)
            ut, vt = _velocity(torch, truth[0])
            # observations of the truth: u or v at each observation point, plus noise
            tval = torch.where(obs_kind == L.LETKF_OBS_U, ut[obs_iy.long(), obs_ix.long()],
                               vt[obs_iy.long(), obs_ix.long()])
            noise = torch.randn(n_obs, generator=gen, device=dev, dtype=torch.float64)
            obs_val = tval + torch.sqrt(obs_var) * noise
            uf, vf = _mean_velocity(torch, ens)
            fc = _rmse(torch, uf, vf, ut, vt)
            obs = (obs_ix, obs_iy, obs_kind, obs_val, obs_var)
            L.letkf_analyze(plan_e, [L.make_io(0, ens, ens, obs)], stream)
            st = L.letkf_status(plan_e, sync=True)
            ua, va = _mean_velocity(torch, ens)
            an = _rmse(torch, ua, va, ut, vt)
            uo, vo = _mean_velocity(torch, free)
            fr = _rmse(torch, uo, vo, ut, vt)
            u_m, v_m = _velocity(torch, ens)
            spread = float(torch.sqrt(0.5 * torch.mean(u_m.var(dim=0) + v_m.var(dim=0))))
            out["cycles"].append(c + 1)
            out["forecast_rmse"].append(fc)
            out["analysis_rmse"].append(an)
            out["free_rmse"].append(fr)
            out["spread"].append(spread)
            out["status"].append(int(st))
    finally:
        L.letkf_plan_destroy(plan_t)
        L.letkf_plan_destroy(plan_e)
    half = cfg.n_cycles // 2
    out["summary"] = {
        "workload": wl.name, "nx": wl.nx, "ny": wl.ny, "k": wl.k, "n_obs": n_obs,
        "n_cycles": cfg.n_cycles, "n_steps": cfg.n_steps, "tau": cfg.tau,
        "force_amp": cfg.force_amp,
        "mean_forecast_rmse_2nd_half": float(np.mean(out["forecast_rmse"][half:])),
        "mean_analysis_rmse_2nd_half": float(np.mean(out["analysis_rmse"][half:])),
        "mean_free_rmse_2nd_half": float(np.mean(out["free_rmse"][half:])),
        "mean_spread_2nd_half": float(np.mean(out["spread"][half:])),
        "obs_sigma": wl.sigma,
        "rmse": "sqrt(mean over grid points of ((u - u_t)^2 + (v - v_t)^2) / 2), ensemble-mean velocity",
    }
    return out
