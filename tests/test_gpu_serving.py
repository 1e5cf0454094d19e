"""Serving form: continuous batching of assimilation cycles over resident
ensembles.  Each session's result must be the same alone and in a mix with
other sessions (bitwise: sessions own all their device memory), also when the
memory budget forces evictions (state swapped to host and back).  Every
cycle's device status must be LETKF_OK."""
import dataclasses

import numpy as np
import pytest

from paper_2308_03310_amd import letkf as L
from paper_2308_03310_amd import serving, synth

pytestmark = pytest.mark.gpu


def _specs():
    mk = lambda i, n, k, st, Lr: serving.SessionSpec(
        f"t{i}", synth.Workload(f"t{i}", n, n, k, st, 0.005, Lr, 1.1, 200 + i), n_steps=12)
    return [mk(0, 32, 16, 2, 3.0), mk(1, 48, 32, 3, 4.0), mk(2, 40, 20, 2, 3.0),
            mk(3, 24, 64, 2, 2.5)]


def _alone(spec, n_cycles):
    srv = serving.AssimilationServer([spec], budget_bytes=1 << 36, n_slots=1)
    try:
        for c in range(n_cycles):
            srv.submit(serving.Request(c, 0, 0.0))
            srv.drain()
        assert all(r.status == L.LETKF_OK for r in srv.done)
        return srv.sessions[0].state()
    finally:
        srv.close()


@pytest.mark.parametrize("budget_sessions", [None, 2])
def test_alone_equals_mix(device, budget_sessions):
    specs = _specs()
    n_cycles = 3
    ref = [_alone(sp, n_cycles) for sp in specs]
    srv = serving.AssimilationServer(specs, budget_bytes=1 << 34, n_slots=4)
    if budget_sessions:
        # room for two resident sessions at a time: forces evictions
        fp = sorted(s.footprint() for s in srv.sessions)
        srv.budget = fp[-1] + fp[-2]
    print(f"mix of {len(specs)} sessions x {n_cycles} cycles, budget {srv.budget}", flush=True)
    try:
        order = np.random.default_rng(5).permutation(np.repeat(np.arange(len(specs)), n_cycles))
        for r, sid in enumerate(order):
            srv.submit(serving.Request(r, int(sid), 0.0))
            srv.step()
        srv.drain()
        got = [s.state() for s in srv.sessions]
        if budget_sessions:
            assert srv.evictions > 0
        assert all(s.cycles_done == n_cycles for s in srv.sessions)
        assert all(r.status == L.LETKF_OK for r in srv.done)
    finally:
        srv.close()
    for i in range(len(specs)):
        assert np.array_equal(got[i], ref[i]), i


def test_large_session_alone_equals_mix(device):
    """A session of the 1024^2, k = 64 workload (FP32 form) among small FP64
    ones: two cycles each, alone and in the mix, bitwise equal."""
    big = serving.SessionSpec("big", dataclasses.replace(synth.WORKLOADS["grid1024_k64"],
                                                         seed=500),
                              n_steps=4, precision=L.LETKF_PREC_FP32)
    specs = [big] + _specs()[:2]
    print("large session alone", flush=True)
    ref = [_alone(sp, 2) for sp in specs]
    srv = serving.AssimilationServer(specs, budget_bytes=1 << 36, n_slots=3)
    try:
        print("large session in a mix of three", flush=True)
        for r, sid in enumerate([0, 1, 2, 1, 0, 2]):
            srv.submit(serving.Request(r, sid, 0.0))
            srv.step()
        srv.drain()
        got = [s.state() for s in srv.sessions]
        assert all(r.status == L.LETKF_OK for r in srv.done)
    finally:
        srv.close()
    for i in range(len(specs)):
        assert np.array_equal(got[i], ref[i]), i


def test_poisson_run_reports_latency(device):
    specs = _specs()
    srv = serving.AssimilationServer(specs, budget_bytes=1 << 34, n_slots=4)
    try:
        st = srv.run_poisson(rate_hz=200.0, n_requests=40, seed=9)
    finally:
        srv.close()
    print(st, flush=True)
    assert st["requests"] == 40
    assert st["served"] == 40 and st["failed"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["throughput_cycles_per_s"] > 0
