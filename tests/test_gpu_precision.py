"""Reduced-precision forms against the FP64 oracle: Gram and transform
contractions in FP32 or BF16 (FP32 accumulation), FP64 eigensolve and
eigenvalue scaling.  Bars on the relative L2 error of the whole analysis
ensemble: FP32 1e-5, BF16 1e-3; the analysis-mean and spread errors are
checked separately (each relative to its own norm)."""
import sys

import numpy as np
import pytest

from oracle import letkf_oracle as orc
from paper_2308_03310_amd import letkf as L
from paper_2308_03310_amd import synth

pytestmark = pytest.mark.gpu

BARS = {L.LETKF_PREC_FP32: 1e-5, L.LETKF_PREC_BF16: 1e-3}


def _run(p, prec):
    import torch
    wl = p.wl
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
    obs = (f(p.obs_ix, torch.int32), f(p.obs_iy, torch.int32), f(p.obs_kind, torch.int32),
           f(p.obs_val, torch.float64), f(p.obs_var, torch.float64))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                                        precision=prec)])
    try:
        xb = f(p.xb, torch.float64)
        xa = torch.empty_like(xb)
        L.letkf_analyze(plan, [L.make_io(0, xb, xa, obs)])
        assert L.letkf_status(plan) == L.LETKF_OK
        return xa.cpu().numpy()
    finally:
        L.letkf_plan_destroy(plan)


def errors(got, ref, xb):
    """Relative L2 errors: whole ensemble, increment, analysis mean, spread."""
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    inc = np.linalg.norm(got - ref) / np.linalg.norm(ref - xb)
    gm, rm = got.mean(axis=0), ref.mean(axis=0)
    mean = np.linalg.norm(gm - rm) / np.linalg.norm(rm)
    gs, rs = got - gm, ref - rm
    spread = np.linalg.norm(gs - rs) / np.linalg.norm(rs)
    return rel, inc, mean, spread


@pytest.mark.parametrize("prec", [L.LETKF_PREC_FP32, L.LETKF_PREC_BF16])
@pytest.mark.parametrize("name", ["cpu32_k16", "ragged"])
def test_reduced_precision_full_field(name, prec):
    wl = synth.WORKLOADS[name] if name in synth.WORKLOADS else \
        synth.Workload("ragged", 40, 27, 20, 3, 0.01, 3.3, 1.15, 60)
    p = synth.make_problem(wl)
    print(f"precision {prec} on {wl.name} ({wl.nx}x{wl.ny}, k={wl.k})", flush=True)
    got = _run(p, prec)
    ref = orc.letkf_analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                             wl.infl)
    rel, inc, mean, spread = errors(got, ref, p.xb)
    print(f"  rel {rel:.2e} increment {inc:.2e} mean {mean:.2e} spread {spread:.2e}", flush=True)
    assert rel <= BARS[prec]
    assert spread <= (2e-4 if prec == L.LETKF_PREC_FP32 else 5e-2)


@pytest.mark.parametrize("prec", [L.LETKF_PREC_FP32, L.LETKF_PREC_BF16])
def test_reduced_precision_grid1024_sampled(prec):
    wl = synth.WORKLOADS["grid1024_k64"]
    print(f"generate grid1024_k64; precision {prec}", flush=True)
    p = synth.make_problem(wl)
    got = _run(p, prec)
    pts = synth.sample_points(wl.nx, wl.ny, 10, seed=11)
    ref = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                       wl.infl).run(pts)
    g = np.stack([got[:, :, q // wl.nx, q % wl.nx] for q in pts])
    xb = np.stack([p.xb[:, :, q // wl.nx, q % wl.nx] for q in pts])
    rel, inc, mean, spread = errors(np.moveaxis(g, 0, -1), np.moveaxis(ref, 0, -1),
                                    np.moveaxis(xb, 0, -1))
    print(f"  rel {rel:.2e} increment {inc:.2e} mean {mean:.2e} spread {spread:.2e}", flush=True)
    assert rel <= BARS[prec]
