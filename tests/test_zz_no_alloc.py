"""The allocation-free entry point (letkf_analyze_noalloc) against the plan
entry point (letkf_analyze) on the same inputs, through the C-ABI.

Both run the same kernels; the no-allocation form takes its workspace from the
library's static device array and sizes its Gram slab to what is left of it.
Held to the FP64 bar (1e-10 relative L2, and element-wise via _parity) on two
calls in a row, the second with a smaller problem, and on an FP32-form call;
an oversized problem is refused on the host before anything is enqueued.
"""
import sys

import numpy as np
import pytest

from paper_2308_03310_amd import synth
from paper_2308_03310_amd import letkf as L
from _parity import assert_parity

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(wl, torch):
    p = synth.make_problem(wl)
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
    obs = (f(p.obs_ix, torch.int32), f(p.obs_iy, torch.int32), f(p.obs_kind, torch.int32),
           f(p.obs_val, torch.float64), f(p.obs_var, torch.float64))
    return p, torch.from_numpy(p.xb).cuda(), obs


def _with_plan(wl, prob, xb, obs, torch):
    xa = torch.empty_like(xb)
    plan = L.letkf_plan([prob])
    try:
        L.letkf_analyze(plan, [L.make_io(0, xb, xa, obs)])
        st = L.letkf_status(plan, sync=True)
    finally:
        L.letkf_plan_destroy(plan)
    assert st == L.LETKF_OK, L.letkf_strerror(st)
    return xa


# a 96 x 80 lattice, k = 32 (several Gram slabs of the static workspace), then
# the 32 x 32, k = 16 workload; then an FP32-form call
SHAPES = [
    synth.Workload("noalloc_96x80_k32", 96, 80, 32, 2, 0.005, 6.0, 1.1, 21),
    synth.WORKLOADS["cpu32_k16"],
]


def test_noalloc_equals_plan_two_calls(device):
    import torch
    status = torch.full((1,), -1, dtype=torch.int32, device=device)
    for wl in SHAPES:
        say(f"noalloc vs plan: {wl.name} {wl.nx}x{wl.ny} k={wl.k}")
        p, xb, obs = _inputs(wl, torch)
        prob = L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl)
        ref = _with_plan(wl, prob, xb, obs, torch).cpu().numpy()
        xa = torch.full_like(xb, float("nan"))
        L.letkf_analyze_noalloc(prob, L.make_io(0, xb, xa, obs), status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0, f"device status {int(status.item())}"
        got = xa.cpu().numpy()
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        say(f"  rel-L2 vs plan entry point {err:.3e}, bitwise equal {np.array_equal(got, ref)}")
        assert err <= TOL_FP64
        assert_parity(got, ref, TOL_FP64, xb=p.xb, inc_tol=1e-8, label=wl.name)


def test_noalloc_fp32_form_in_place(device):
    import torch
    wl = SHAPES[1]
    p, xb, obs = _inputs(wl, torch)
    prob = L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                          precision=L.LETKF_PREC_FP32)
    ref = _with_plan(wl, prob, xb, obs, torch).cpu().numpy()
    x = xb.clone()
    status = torch.full((1,), -1, dtype=torch.int32, device=device)
    L.letkf_analyze_noalloc(prob, L.make_io(0, x, x, obs), status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    got = x.cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    say(f"noalloc FP32 form in place: rel-L2 vs plan entry point {err:.3e}")
    assert err <= TOL_FP64


def test_noalloc_refuses_oversized_problem(device):
    import torch
    # 512 x 512, k = 64: the ensemble alone is 1.2 GB, far beyond the static workspace
    prob = L.make_problem(512, 512, 64, 100, 8.0, 1.1)
    xb = torch.zeros(1, dtype=torch.float64, device=device)
    io = L.letkf_io(0, 0, xb.data_ptr(), xb.data_ptr(), 0, 0, 0, 0, 0)
    status = torch.zeros(1, dtype=torch.int32, device=device)
    rc = L.load_library().letkf_analyze_noalloc(
        L.ctypes.byref(prob), L.ctypes.byref(io), status.data_ptr(),
        torch.cuda.current_stream().cuda_stream)
    assert rc == L.LETKF_ENOMEM
