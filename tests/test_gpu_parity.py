"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

FP64 bar 1e-10, held element-wise (tests/_parity.py): relative L2 over every
entry, relative L2 of each grid point, |error| <= 1e-10 max|x^a| per entry,
and each point's error <= 1e-8 of its own analysis increment -- on whole
fields of small grids and on sampled points at full size, plus structural
properties that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

from oracle import letkf_oracle as orc
from paper_2308_03310_amd import synth
from paper_2308_03310_amd import letkf as L
from _parity import assert_parity

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
INC_TOL = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_obs(p, torch):
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
    return (f(p.obs_ix, torch.int32), f(p.obs_iy, torch.int32), f(p.obs_kind, torch.int32),
            f(p.obs_val, torch.float64), f(p.obs_var, torch.float64))


def gpu_analysis(p, L_len=None, infl=None, loc=L.LETKF_LOC_GAUSS, inplace=False, obs=True,
                 var=None, xa_fill=None, flags=0):
    import torch
    wl = p.wl
    L_len = wl.L if L_len is None else L_len
    infl = wl.infl if infl is None else infl
    n_obs = len(p.obs_ix)
    plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, n_obs, L_len, infl, loc)],
                        flags=flags)
    try:
        xb = torch.from_numpy(p.xb).cuda()
        if inplace:
            xa = xb
        else:
            xa = torch.full_like(xb, xa_fill) if xa_fill is not None else torch.empty_like(xb)
        o = None
        if obs:
            o = list(dev_obs(p, torch))
            if var is not None:
                o[4] = torch.from_numpy(var).cuda()
        L.letkf_analyze(plan, [L.make_io(0, xb, xa, o)])
        st = L.letkf_status(plan, sync=True)
        return xa.cpu().numpy(), st
    finally:
        L.letkf_plan_destroy(plan)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module", autouse=True)
def _torch(device):
    import torch
    return torch


# ------------------------------------------------------------ eigensolver
@pytest.mark.parametrize("k", [2, 3, 16, 17, 31, 32, 33, 48, 64])
def test_eigh_batched_random(k):
    import torch
    say(f"eigh_batched k={k} batch=37")
    rng = np.random.default_rng(100 + k)
    B = rng.standard_normal((37, k, k))
    A = B @ B.transpose(0, 2, 1) / k + np.eye(k) * (k - 1) / 1.1
    A[5] = np.diag(rng.permutation(np.repeat([1.0, 2.0], (k + 1) // 2)[:k]))   # exact ties
    A[6] = 3.0 * np.eye(k)
    y = rng.standard_normal(k)
    A[7] = 2.0 * np.eye(k) + np.outer(y, y)                                     # multiplicity k-1
    A[8] = rng.standard_normal((k, k))
    A[8] = A[8] + A[8].T                                                        # indefinite
    a = torch.from_numpy(A).cuda()
    lam = torch.empty(37, k, dtype=torch.float64, device="cuda")
    vec = torch.empty(37, k, k, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.letkf_eigh_batched(a, lam, vec, st)
    torch.cuda.synchronize()
    lam, vec = lam.cpu().numpy(), vec.cpu().numpy()
    assert int(st.cpu()[0]) == 0
    for i in range(37):
        nrm = np.linalg.norm(A[i])
        ref = np.linalg.eigvalsh(A[i])
        np.testing.assert_allclose(np.sort(lam[i]), ref, rtol=0, atol=1e-13 * nrm)
        V = vec[i]
        assert np.linalg.norm(V @ np.diag(lam[i]) @ V.T - A[i]) <= 1e-13 * nrm * k
        assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-13 * k


def _hard_matrices(k, family, n, rng):
    """Batches of symmetric k x k matrices that stress a divide-and-conquer
    eigensolver: nearly equal eigenvalues, Wilkinson's close pairs, weakly
    coupled blocks, a graded spectrum, entries of magnitude 1e+-90 and
    1e+-140, and the LETKF form with multiplicity."""
    def orth(m):
        q, r = np.linalg.qr(rng.standard_normal((m, m)))
        return q * np.sign(np.diag(r))
    out = np.empty((n, k, k))
    for b in range(n):
        if family == "clusters":          # clusters of 2-4 eigenvalues 1e-10 apart (relative)
            lam = []
            while len(lam) < k:
                c = rng.uniform(1.0, 100.0)
                lam += [c * (1.0 + 1e-10 * j) for j in range(rng.integers(2, 5))]
            lam = np.array(lam[:k])
            Q = orth(k)
            out[b] = (Q * lam) @ Q.T
        elif family == "wilkinson":       # W+: d_i = |m - i|, e = 1 (pairs agreeing to many digits)
            m = (k - 1) / 2.0
            out[b] = np.diag(np.abs(m - np.arange(k))) + np.diag(np.ones(k - 1), 1) + \
                np.diag(np.ones(k - 1), -1)
            if b % 2:
                P = np.eye(k)[rng.permutation(k)]
                out[b] = P @ out[b] @ P.T
        elif family == "glued":           # blocks of 8 coupled by 1e-14
            A = np.zeros((k, k))
            for a0 in range(0, k, 8):
                a1 = min(a0 + 8, k)
                B = rng.standard_normal((a1 - a0, a1 - a0))
                A[a0:a1, a0:a1] = B + B.T + 10.0 * np.eye(a1 - a0)
                if a0 > 0:
                    A[a0 - 1, a0] = A[a0, a0 - 1] = 1e-14
            out[b] = A
        elif family == "graded":          # eigenvalues from 1e-6 to 1e6
            Q = orth(k)
            out[b] = (Q * np.logspace(-6, 6, k)) @ Q.T
        elif family == "scaled":          # random, scaled to 1e+-90 and 1e+-140
            B = rng.standard_normal((k, k))
            out[b] = (B + B.T) * (1e-140, 1e-90, 1e90, 1e140)[b % 4]
        else:                             # letkf: alpha I + rank-r PSD, r < k
            r = int(rng.integers(1, k))
            Y = rng.standard_normal((r, k)) * np.sqrt(rng.uniform(0.1, 1e4, r))[:, None]
            Y -= Y.mean(axis=1, keepdims=True)
            out[b] = Y.T @ Y + (k - 1) / 1.1 * np.eye(k)
    return 0.5 * (out + out.transpose(0, 2, 1))


@pytest.mark.parametrize("family", ["clusters", "wilkinson", "glued", "graded", "scaled", "letkf"])
@pytest.mark.parametrize("k", [16, 21, 33, 64])
def test_eigh_batched_hard_families(k, family):
    import torch
    n = 96
    say(f"eigh_batched {family} k={k} batch={n}")
    rng = np.random.default_rng(1000 + k)
    A = _hard_matrices(k, family, n, rng)
    lam = torch.empty(n, k, dtype=torch.float64, device="cuda")
    vec = torch.empty(n, k, k, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.letkf_eigh_batched(torch.from_numpy(A).cuda(), lam, vec, st)
    torch.cuda.synchronize()
    lam, vec = lam.cpu().numpy(), vec.cpu().numpy()
    assert int(st.cpu()[0]) == 0
    for i in range(n):
        nrm = np.linalg.norm(A[i])
        np.testing.assert_allclose(np.sort(lam[i]), np.linalg.eigvalsh(A[i]), rtol=0,
                                   atol=1e-13 * nrm)
        V = vec[i]
        assert np.linalg.norm(V @ np.diag(lam[i]) @ V.T - A[i]) <= 1e-13 * nrm * k
        assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-13 * k


@pytest.mark.parametrize("k", [1, 5, 16, 33, 64])
def test_eigh_batched_power_of_two_scaling(k):
    """Scaling the input by 2^s (exact) scales the eigenvalues by 2^s and
    leaves the eigenvectors unchanged, bit for bit, up to magnitudes near the
    ends of the FP64 range (each matrix is brought to a largest entry in
    [0.5, 1) before the solve); the unscaled run matches numpy.  A zero
    matrix and k = 1 are the degenerate cases."""
    import torch
    n = 16
    rng = np.random.default_rng(500 + k)
    B = rng.standard_normal((n, k, k))
    A = B + B.transpose(0, 2, 1)
    A[3] = 0.0

    def run(M):
        lam = torch.empty(n, k, dtype=torch.float64, device="cuda")
        vec = torch.empty(n, k, k, dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        L.letkf_eigh_batched(torch.from_numpy(M).cuda(), lam, vec, st)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 0
        return lam.cpu().numpy(), vec.cpu().numpy()

    say(f"eigh_batched k={k}: scales 2^0, 2^-900, 2^900")
    lam0, vec0 = run(A)
    for i in range(n):
        nrm = max(np.linalg.norm(A[i]), 1e-300)
        np.testing.assert_allclose(np.sort(lam0[i]), np.linalg.eigvalsh(A[i]), rtol=0,
                                   atol=1e-13 * nrm)
        V = vec0[i]
        assert np.linalg.norm(V @ np.diag(lam0[i]) @ V.T - A[i]) <= 1e-13 * nrm * k
        assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-13 * k
    for e in (-900, 900):
        lam, vec = run(np.ldexp(A, e))
        assert np.array_equal(lam, np.ldexp(lam0, e))
        assert np.array_equal(vec, vec0)


@pytest.mark.parametrize("k", [51, 52, 60])
def test_eigh_batched_secular_near_pole_pairs(k):
    # Wilkinson batches at these orders give merges where a root lies within
    # ~1e-11 of a pole that has a second pole ~1e-11 on its other side: the
    # secular iteration must still converge (status clean) and stay accurate.
    import torch
    n = 24
    for rep in range(3):
        say(f"eigh_batched wilkinson k={k} seed {rep}")
        A = _hard_matrices(k, "wilkinson", n, np.random.default_rng(100000 * rep + 1000 * k + 2))
        lam = torch.empty(n, k, dtype=torch.float64, device="cuda")
        vec = torch.empty(n, k, k, dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        L.letkf_eigh_batched(torch.from_numpy(A).cuda(), lam, vec, st)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 0
        lam, vec = lam.cpu().numpy(), vec.cpu().numpy()
        for i in range(n):
            nrm = np.linalg.norm(A[i])
            np.testing.assert_allclose(np.sort(lam[i]), np.linalg.eigvalsh(A[i]), rtol=0,
                                       atol=1e-13 * nrm)
            V = vec[i]
            assert np.linalg.norm(V @ np.diag(lam[i]) @ V.T - A[i]) <= 1e-13 * nrm * k
            assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-13 * k


# ------------------------------------------------------------ whole analyses
def _oracle_full(p, L_len=None, infl=None, loc=orc.LOC_GAUSS, var=None):
    wl = p.wl
    return orc.letkf_analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val,
                              p.obs_var if var is None else var,
                              wl.L if L_len is None else L_len, wl.infl if infl is None else infl,
                              loc)


# the two routes to the transform: the eigendecomposition (default) and the
# Newton-Schulz inverse square root (LETKF_FLAG_NSQRT)
ROUTES = [0, L.LETKF_FLAG_NSQRT]


@pytest.mark.parametrize("flags", ROUTES)
def test_cpu32_k16_full_field(flags):
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    say(f"analysis cpu32_k16 (32x32, k=16) full field flags={flags}")
    got, st = gpu_analysis(p, flags=flags)
    assert st == L.LETKF_OK
    ref = _oracle_full(p)
    assert_parity(got, ref, TOL_FP64, p.xb, INC_TOL, "cpu32_k16")


@pytest.mark.parametrize("flags", ROUTES)
@pytest.mark.parametrize("loc", [orc.LOC_GAUSS, orc.LOC_GC, orc.LOC_NONE])
@pytest.mark.parametrize("k", [5, 20, 40])
def test_ragged_grid(loc, k, flags):
    """Grid and ensemble sizes that are not multiples of any tile: 40 x 27
    lattice (ragged 64-point tiles and 8-point cells), obs of all three kinds
    on a stride-3 mask, L = 3.3 (window wraps around the periodic box for
    NONE)."""
    wl = synth.Workload("ragged", 40, 27, k, 3, 0.01, 3.3, 1.15, 40 + k,
                        kinds=(synth.OBS_RHO, synth.OBS_U, synth.OBS_V))
    p = synth.make_problem(wl)
    say(f"analysis ragged 40x27 k={k} loc={loc} flags={flags}")
    got, st = gpu_analysis(p, loc=loc, flags=flags)
    assert st == L.LETKF_OK
    ref = _oracle_full(p, loc=loc)
    assert_parity(got, ref, TOL_FP64, p.xb, INC_TOL, f"ragged k={k} loc={loc}")


def test_small_periodic_window_wraps():
    """2L larger than half the box: windows wrap onto themselves; every
    observation must be counted once at its minimum-image distance."""
    wl = synth.Workload("wrap", 12, 10, 8, 2, 0.01, 3.0, 1.1, 9)
    p = synth.make_problem(wl)
    say("analysis wrap 12x10 k=8 L=3")
    got, st = gpu_analysis(p)
    assert st == L.LETKF_OK
    assert_parity(got, _oracle_full(p), TOL_FP64, p.xb, INC_TOL, "wrap")


def test_inplace_and_determinism():
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    say("analysis cpu32_k16 in-place vs out-of-place, twice")
    a1, _ = gpu_analysis(p)
    a2, _ = gpu_analysis(p)
    a3, st = gpu_analysis(p, inplace=True)
    assert st == L.LETKF_OK
    assert np.array_equal(a1, a2)
    assert np.array_equal(a1, a3)


@pytest.mark.parametrize("flags", ROUTES)
def test_infinite_variance_returns_inflated_background(flags):
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    say(f"analysis cpu32_k16 with every variance +inf flags={flags}")
    var = np.full_like(p.obs_var, np.inf)
    got, st = gpu_analysis(p, var=var, flags=flags)
    assert st == L.LETKF_OK
    xbar = p.xb.mean(axis=0, keepdims=True)
    ref = xbar + math.sqrt(p.wl.infl) * (p.xb - xbar)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)
    got1, _ = gpu_analysis(p, var=var, infl=1.0, flags=flags)
    np.testing.assert_allclose(got1, p.xb, rtol=0, atol=1e-15)


@pytest.mark.parametrize("flags", ROUTES)
def test_no_observations(flags):
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    say(f"analysis cpu32_k16 with n_obs = 0 flags={flags}")
    got, st = gpu_analysis(p, obs=False, infl=1.0, flags=flags)
    assert st == L.LETKF_OK
    np.testing.assert_allclose(got, p.xb, rtol=0, atol=1e-15)


def test_invalid_observation_sets_status_and_skips():
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    for what in ("var_neg", "var_nan", "ix_range", "kind"):
        q = synth.make_problem(p.wl)
        if what == "var_neg":
            q.obs_var = q.obs_var.copy(); q.obs_var[7] = -1.0
        elif what == "var_nan":
            q.obs_var = q.obs_var.copy(); q.obs_var[3] = np.nan
        elif what == "ix_range":
            q.obs_ix = q.obs_ix.copy(); q.obs_ix[11] = 32
        else:
            q.obs_kind = q.obs_kind.copy(); q.obs_kind[0] = 3
        say(f"analysis cpu32_k16 with invalid observation ({what})")
        got, st = gpu_analysis(q, xa_fill=-7.0)
        assert st == L.LETKF_EINVAL
        assert np.all(got == -7.0)
    got, st = gpu_analysis(p)            # the plan's next call is clean again
    assert st == L.LETKF_OK


# ------------------------------------------------------------ full sizes, sampled
@pytest.mark.parametrize("name,npts", [("grid256_k32", 48), ("grid1024_k64", 12)])
def test_full_size_sampled(name, npts):
    wl = synth.WORKLOADS[name]
    say(f"generate {name}")
    p = synth.make_problem(wl)
    pts = synth.sample_points(wl.nx, wl.ny, npts, seed=7)
    say(f"oracle on {len(pts)} sampled points")
    ref = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L,
                       wl.infl).run(pts)
    xb = np.stack([p.xb[:, :, q // wl.nx, q % wl.nx] for q in pts])
    for flags in ROUTES:
        say(f"analysis {name} ({wl.nx}x{wl.ny}, k={wl.k}) on the GPU, flags={flags}")
        got, st = gpu_analysis(p, flags=flags)
        assert st == L.LETKF_OK
        # properties at every point: analysis perturbations sum to zero
        mean = got.mean(axis=0, keepdims=True)
        assert np.abs((got - mean).sum(axis=0)).max() <= 1e-14 * wl.k
        assert np.isfinite(got).all()
        g = np.stack([got[:, :, q // wl.nx, q % wl.nx] for q in pts])
        assert_parity(g, ref, TOL_FP64, xb, INC_TOL, f"{name} flags={flags}")
        del got, g
