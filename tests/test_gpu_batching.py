"""The batching form on the mixed-batch recipe: independent problems of
different lattice sizes, ensemble sizes, localization lengths, error
variances and random observation masks with clustered gaps (local
observation counts from 0 to thousands), analysed in one call; and the
launch settings the autotuner chooses between (observation-cell edge, grid
or persistent Gram kernels)."""
import numpy as np
import pytest

from oracle import letkf_oracle as orc
from paper_2308_03310_amd import letkf as L
from paper_2308_03310_amd import synth

pytestmark = pytest.mark.gpu

N_PROBLEMS = 24


@pytest.fixture(scope="module")
def batch(device):
    import torch
    wls = synth.batching_workloads(N_PROBLEMS, seed=3, grids=(64, 128))
    items, probs, ios = [], [], []
    for i, wl in enumerate(wls):
        p = synth.make_problem(wl)
        f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
        obs = (f(p.obs_ix, torch.int32), f(p.obs_iy, torch.int32), f(p.obs_kind, torch.int32),
               f(p.obs_val, torch.float64), f(p.obs_var, torch.float64))
        xb = f(p.xb, torch.float64)
        xa = torch.empty_like(xb)
        items.append((p, xb, xa, obs))
        probs.append(L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl))
        ios.append(L.make_io(i, xb, xa, obs))
    print(f"{len(wls)} problems: grids {sorted({w.nx for w in wls})}, "
          f"k {sorted({w.k for w in wls})}, obs {min(len(it[0].obs_ix) for it in items)}-"
          f"{max(len(it[0].obs_ix) for it in items)}", flush=True)
    return items, probs, ios


def _outputs(items):
    return [xa.cpu().numpy() for (_, _, xa, _) in items]


def test_mixed_batch_equals_alone_and_oracle(batch):
    items, probs, ios = batch
    plan = L.letkf_plan(probs)
    try:
        print("one batched call over every problem", flush=True)
        L.letkf_analyze(plan, ios)
        assert L.letkf_status(plan) == L.LETKF_OK
        batched = _outputs(items)
        print("one call per problem", flush=True)
        for io in ios:
            L.letkf_analyze(plan, [io])
        assert L.letkf_status(plan) == L.LETKF_OK
        alone = _outputs(items)
    finally:
        L.letkf_plan_destroy(plan)
    for i in range(len(items)):
        assert np.array_equal(batched[i], alone[i]), i
    for i in (0, 3, 7, 12, 18, 23):
        p = items[i][0]
        wl = p.wl
        pts = synth.sample_points(wl.nx, wl.ny, 4, seed=20 + i)
        ref = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                           wl.infl).run(pts)
        got = np.stack([batched[i][:, :, q // wl.nx, q % wl.nx] for q in pts])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"  problem {i} ({wl.nx}^2, k={wl.k}, L={wl.L:.1f}, {len(p.obs_ix)} obs): "
              f"rel-L2 {err:.2e}", flush=True)
        assert err <= 1e-10, i


def test_tuning_settings_and_autotuner(batch):
    items, probs, ios = batch
    plan = L.letkf_plan(probs)
    try:
        res = {}
        for cell in (4, 8, 16):
            for pers in (0, 1):
                print(f"setting cell {cell}, persistent {pers}", flush=True)
                L.letkf_set_tuning(plan, cell, pers)
                L.letkf_analyze(plan, ios)
                assert L.letkf_status(plan) == L.LETKF_OK
                res[(cell, pers)] = _outputs(items)
        for cell in (4, 8, 16):
            for i in range(len(items)):                  # same points, same order: same bits
                assert np.array_equal(res[(cell, 0)][i], res[(cell, 1)][i]), (cell, i)
        for cell in (4, 16):                             # other summation order only
            for i in range(len(items)):
                a, b = res[(cell, 0)][i], res[(8, 0)][i]
                assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-13, (cell, i)
        print("autotuner", flush=True)
        t = L.letkf_tune(plan, ios)
        print(f"  chose {t}", flush=True)
        assert t["cell"] in (4, 8, 16) and t["gram_persistent"] in (0, 1) and t["ms_per_call"] > 0
        tuned = _outputs(items)
        for i in range(len(items)):
            assert np.array_equal(tuned[i], res[(t["cell"], t["gram_persistent"])][i]), i
        assert L.letkf_status(plan) == L.LETKF_OK
        with pytest.raises(L.LetkfError):
            L.letkf_set_tuning(plan, 12, 0)
    finally:
        L.letkf_plan_destroy(plan)
