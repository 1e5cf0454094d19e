"""GPU parity of the assimilation cycle: lattice-BGK steps (HIP) against the
BGK oracle, and a whole cycle (steps + analysis) against oracle advance +
oracle analysis."""
import numpy as np
import pytest

from oracle import lbm_oracle as lbm
from oracle import letkf_oracle as orc
from paper_2308_03310_amd import letkf as L
from paper_2308_03310_amd import synth

pytestmark = pytest.mark.gpu


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


@pytest.mark.parametrize("n_steps", [0, 1, 6, 7])
def test_cycle_matches_oracle(device, n_steps):
    import torch
    wl = synth.Workload("cyc", 40, 24, 12, 2, 0.005, 3.0, 1.1, 21)
    p = synth.make_problem(wl)
    print(f"cycle 40x24 k=12 n_steps={n_steps}", flush=True)
    tau, amp, kx = 0.52, 1e-5, 4
    obs = (_dev(p.obs_ix, torch.int32), _dev(p.obs_iy, torch.int32), _dev(p.obs_kind, torch.int32),
           _dev(p.obs_val, torch.float64), _dev(p.obs_var, torch.float64))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl)],
                        flags=L.LETKF_FLAG_CYCLE)
    try:
        x = _dev(p.xb, torch.float64)
        L.letkf_cycle(plan, [L.make_cycle_io(0, x, obs, n_steps, tau, amp, kx)])
        assert L.letkf_status(plan) == L.LETKF_OK
        got = x.cpu().numpy()
    finally:
        L.letkf_plan_destroy(plan)
    fc = lbm.advance(p.xb, n_steps, tau, amp, kx)
    ref = orc.letkf_analysis(fc, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                             wl.infl)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-10


def test_bgk_only_cycle_with_ignored_observations(device):
    """Every variance +inf and rho = 1: the analysis is the identity, so the
    cycle output is the BGK advance alone (checked to 1e-13)."""
    import torch
    wl = synth.Workload("bgk", 33, 17, 5, 3, 0.005, 2.0, 1.0, 22)
    p = synth.make_problem(wl)
    print("cycle 33x17 k=5, 9 steps, observations ignored", flush=True)
    var = np.full_like(p.obs_var, np.inf)
    obs = (_dev(p.obs_ix, torch.int32), _dev(p.obs_iy, torch.int32), _dev(p.obs_kind, torch.int32),
           _dev(p.obs_val, torch.float64), _dev(var, torch.float64))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, 1.0)],
                        flags=L.LETKF_FLAG_CYCLE)
    try:
        x = _dev(p.xb, torch.float64)
        L.letkf_cycle(plan, [L.make_cycle_io(0, x, obs, 9, 0.6, 3e-4, 2)])
        assert L.letkf_status(plan) == L.LETKF_OK
        got = x.cpu().numpy()
    finally:
        L.letkf_plan_destroy(plan)
    ref = lbm.advance(p.xb, 9, 0.6, 3e-4, 2)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_cycle_needs_flag_and_inplace(device):
    import torch
    wl = synth.WORKLOADS["cpu32_k16"]
    p = synth.make_problem(wl)
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, 0, wl.L, wl.infl)])
    try:
        x = _dev(p.xb, torch.float64)
        with pytest.raises(L.LetkfError):
            L.letkf_cycle(plan, [L.make_cycle_io(0, x, None, 3)])
        io = L.make_cycle_io(0, x, None, 0)
        io.io.xa = torch.empty_like(x).data_ptr()
        with pytest.raises(L.LetkfError):
            L.letkf_cycle(plan, [io])
    finally:
        L.letkf_plan_destroy(plan)


@pytest.mark.parametrize("n_steps", [1, 2, 5])
def test_invalid_observation_keeps_the_advance(device, n_steps):
    """A cycle whose observations hold an invalid record reports LETKF_EINVAL
    and leaves the ensemble at the model advance of all n_steps steps (odd
    and even counts alike), unanalysed."""
    import torch
    wl = synth.Workload("cycbad", 24, 20, 8, 2, 0.005, 3.0, 1.1, 23)
    p = synth.make_problem(wl)
    print(f"cycle 24x20 k=8 n_steps={n_steps} with an invalid observation", flush=True)
    var = p.obs_var.copy()
    var[5] = -1.0
    obs = (_dev(p.obs_ix, torch.int32), _dev(p.obs_iy, torch.int32), _dev(p.obs_kind, torch.int32),
           _dev(p.obs_val, torch.float64), _dev(var, torch.float64))
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl)],
                        flags=L.LETKF_FLAG_CYCLE)
    try:
        x = _dev(p.xb, torch.float64)
        L.letkf_cycle(plan, [L.make_cycle_io(0, x, obs, n_steps, 0.52, 1e-5, 4)])
        assert L.letkf_status(plan) == L.LETKF_EINVAL
        got = x.cpu().numpy()
    finally:
        L.letkf_plan_destroy(plan)
    ref = lbm.advance(p.xb, n_steps, 0.52, 1e-5, 4)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
