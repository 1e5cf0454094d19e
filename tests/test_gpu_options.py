"""Plan options of the C-ABI on the GPU: observations in host memory, the
tuning cache, the DETERMINISTIC and GRAPH_CAPTURE flags, and the status read
that does not wait for the analysis stream."""
import os

import numpy as np
import pytest

from paper_2308_03310_amd import letkf as L
from paper_2308_03310_amd import synth

pytestmark = pytest.mark.gpu


def _problem():
    return synth.make_problem(synth.Workload("opt", 40, 32, 16, 2, 0.005, 4.0, 1.1, 71))


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def _obs(p, torch, host=False, pin=False):
    arrs = ((p.obs_ix, torch.int32), (p.obs_iy, torch.int32), (p.obs_kind, torch.int32),
            (p.obs_val, torch.float64), (p.obs_var, torch.float64))
    if not host:
        return tuple(_dev(a, dt) for a, dt in arrs)
    out = []
    for a, dt in arrs:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(dt)
        out.append(t.pin_memory() if pin else t)
    return tuple(out)


def _mk(p, **kw):
    wl = p.wl
    return L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl)], **kw)


def _analyse(plan, p, obs, host=False):
    import torch
    xb = _dev(p.xb, torch.float64)
    xa = torch.full_like(xb, -3.0)
    L.letkf_analyze(plan, [L.make_io(0, xb, xa, obs, obs_on_host=host)])
    torch.cuda.synchronize()
    return xa.cpu().numpy()


def test_obs_on_host_equals_device(device):
    import torch
    p = _problem()
    print("device observations", flush=True)
    plan = _mk(p)
    try:
        ref = _analyse(plan, p, _obs(p, torch))
        assert L.letkf_status(plan) == L.LETKF_OK
    finally:
        L.letkf_plan_destroy(plan)
    plan = _mk(p, flags=L.LETKF_FLAG_OBS_ON_HOST)
    try:
        for pin in (False, True):
            print(f"host observations, pinned={pin}", flush=True)
            got = _analyse(plan, p, _obs(p, torch, host=True, pin=pin), host=True)
            assert L.letkf_status(plan) == L.LETKF_OK
            assert np.array_equal(got, ref)
        with pytest.raises(ValueError):            # device tensors refused by the binding
            _analyse(plan, p, _obs(p, torch), host=False)
        print("host observations with an invalid record: refused before enqueue", flush=True)
        bad = list(_obs(p, torch, host=True))
        bad[4] = bad[4].clone()
        bad[4][3] = float("nan")
        xb = _dev(p.xb, torch.float64)
        xa = torch.full_like(xb, -3.0)
        with pytest.raises(L.LetkfError) as ei:
            L.letkf_analyze(plan, [L.make_io(0, xb, xa, tuple(bad), obs_on_host=True)])
        assert ei.value.code == L.LETKF_EINVAL
        torch.cuda.synchronize()
        assert torch.all(xa == -3.0)
        assert L.letkf_status(plan) == L.LETKF_OK
    finally:
        L.letkf_plan_destroy(plan)


def test_binding_checks_sizes(device):
    import torch
    p = _problem()
    plan = _mk(p)
    try:
        xb = _dev(p.xb, torch.float64)
        obs = _obs(p, torch)
        with pytest.raises(ValueError):
            L.letkf_analyze(plan, [L.make_io(0, xb, xb[:-1].contiguous(), obs)])
        short = list(obs)
        short[3] = short[3][:-1].contiguous()
        with pytest.raises(ValueError):
            L.letkf_analyze(plan, [L.make_io(0, xb, torch.empty_like(xb), tuple(short))])
    finally:
        L.letkf_plan_destroy(plan)


def test_tune_cache_roundtrip(device, tmp_path):
    import torch
    p = _problem()
    path = str(tmp_path / "tune.txt")
    obs = _obs(p, torch)
    plan = _mk(p, tune_cache_path=path)
    try:
        xb = _dev(p.xb, torch.float64)
        xa = torch.empty_like(xb)
        print("tune with a cache path", flush=True)
        t = L.letkf_tune(plan, [L.make_io(0, xb, xa, obs)])
        tuned = xa.cpu().numpy()
    finally:
        L.letkf_plan_destroy(plan)
    line = open(path).read().split()
    assert len(line) == 4 and int(line[1]) == t["cell"] and int(line[2]) == t["form"]
    print(f"  chose {t}; a new plan loads it", flush=True)
    plan = _mk(p, tune_cache_path=path)
    try:
        got = _analyse(plan, p, obs)
        assert L.letkf_status(plan) == L.LETKF_OK
        assert np.array_equal(got, tuned)
    finally:
        L.letkf_plan_destroy(plan)
    # the cache holds one line per key: tuning again replaces it
    plan = _mk(p, tune_cache_path=path)
    try:
        xb = _dev(p.xb, torch.float64)
        L.letkf_tune(plan, [L.make_io(0, xb, torch.empty_like(xb), obs)])
    finally:
        L.letkf_plan_destroy(plan)
    assert len(open(path).read().strip().splitlines()) == 1


def test_deterministic_tune_keeps_cell(device, tmp_path):
    import torch
    p = _problem()
    obs = _obs(p, torch)
    plan = _mk(p)
    try:
        ref = _analyse(plan, p, obs)
    finally:
        L.letkf_plan_destroy(plan)
    path = str(tmp_path / "tune.txt")
    plan = _mk(p, flags=L.LETKF_FLAG_DETERMINISTIC, tune_cache_path=path)
    try:
        xb = _dev(p.xb, torch.float64)
        xa = torch.empty_like(xb)
        t = L.letkf_tune(plan, [L.make_io(0, xb, xa, obs)])
        print(f"deterministic tune chose {t}", flush=True)
        assert t["cell"] == 8
        assert np.array_equal(xa.cpu().numpy(), ref)
    finally:
        L.letkf_plan_destroy(plan)
    # a cache entry with another cell edge is not applied to a deterministic plan
    key = open(path).read().split()[0]
    open(path, "w").write(f"{key} 4 0 1.0\n")
    plan = _mk(p, flags=L.LETKF_FLAG_DETERMINISTIC, tune_cache_path=path)
    try:
        assert np.array_equal(_analyse(plan, p, obs), ref)
    finally:
        L.letkf_plan_destroy(plan)


@pytest.mark.parametrize("form", [L.LETKF_FORM_GRID, L.LETKF_FORM_FUSED])
def test_graph_capture_plan_replays(device, form):
    import torch
    p = _problem()
    obs = _obs(p, torch)
    plan = _mk(p, flags=L.LETKF_FLAG_GRAPH_CAPTURE)
    try:
        L.letkf_set_tuning(plan, 8, form)
        xb = _dev(p.xb, torch.float64)
        xa = torch.empty_like(xb)
        io = [L.make_io(0, xb, xa, obs)]
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            L.letkf_analyze(plan, io, s)
        torch.cuda.synchronize()
        eager = xa.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            L.letkf_analyze(plan, io, s)
        for rep in range(3):
            print(f"graph replay {rep}", flush=True)
            xa.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(xa, eager)
            torch.randn(1 << 18, device="cuda").sum()
            torch.cuda.synchronize()
        assert L.letkf_status(plan) == L.LETKF_OK
        del g
    finally:
        torch.cuda.synchronize()
        L.letkf_plan_destroy(plan)


def test_status_read_clears_only_what_it_read(device):
    import torch
    p = _problem()
    var = p.obs_var.copy()
    var[0] = -1.0
    plan = _mk(p)
    try:
        bad = list(_obs(p, torch))
        bad[4] = _dev(var, torch.float64)
        _analyse(plan, p, tuple(bad))
        assert L.letkf_status(plan, sync=False) == L.LETKF_EINVAL
        assert L.letkf_status(plan, sync=False) == L.LETKF_OK
        _analyse(plan, p, _obs(p, torch))
        assert L.letkf_status(plan, sync=True) == L.LETKF_OK
    finally:
        L.letkf_plan_destroy(plan)
