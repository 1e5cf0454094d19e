"""Pins of the CPU oracle against things other than itself (CPU only).

Each test targets a plausible mistake: a wrong velocity table or moment, a
dropped inflation or sqrt(M-1) factor, a transposed transform, a wrong sign in
the mean update, an exclusive instead of inclusive cutoff, a wrong distance.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import letkf_oracle as orc
from oracle import kf_bruteforce as kf
from paper_2308_03310_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- moments
def test_moments_of_equilibrium_are_exact():
    """H(f_eq(rho,u,v)) = (rho,u,v): the D2Q9 equilibrium reproduces its own
    moments (Sec. II-A moment equations).  Catches a wrong velocity table."""
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.05 * rng.standard_normal((1, 5, 7))
    u = 0.05 * rng.standard_normal((1, 5, 7))
    v = 0.05 * rng.standard_normal((1, 5, 7))
    f = synth.equilibrium(rho, u, v)          # [1, 9, 5, 7]
    iy, ix = np.meshgrid(np.arange(5), np.arange(7), indexing="ij")
    iy, ix = iy.ravel(), ix.ravel()
    for kind, ref in ((orc.OBS_RHO, rho), (orc.OBS_U, u), (orc.OBS_V, v)):
        y = orc.forecast_observations(f, ix, iy, np.full(ix.size, kind))
        np.testing.assert_allclose(y[0], ref[0][iy, ix], rtol=0, atol=2e-16 * 8)
        for j in range(0, ix.size, 7):   # scalar form agrees with the vector form
            assert orc.observe_member(f[0, :, iy[j], ix[j]], kind) == pytest.approx(y[0, j], abs=1e-16)


# ---------------------------------------------------------------- brute-force KF
def _tiny_linear_case(seed, k=8, nx=4, ny=4, n_obs=6):
    rng = np.random.default_rng(seed)
    xb = 0.1 + 0.02 * rng.random((k, 9, ny, nx))
    cells = rng.choice(nx * ny, size=n_obs, replace=False)
    obs_ix = (cells % nx).astype(np.int32)
    obs_iy = (cells // nx).astype(np.int32)
    kind = np.full(n_obs, orc.OBS_RHO, dtype=np.int32)        # rho is linear in f
    var = (0.01 + 0.02 * rng.random(n_obs)) ** 2
    yo = xb[:, :, obs_iy, obs_ix].sum(axis=1).mean(axis=0) + 0.01 * rng.standard_normal(n_obs)
    return xb, obs_ix, obs_iy, kind, yo, var


@pytest.mark.parametrize("infl", [1.0, 1.3])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_letkf_equals_bruteforce_kalman_filter(seed, infl):
    """Linear H, no localization: the LETKF mean and covariance equal the
    model-space KF (eqs. kfx/kfp/kfk) with P^f = rho * dX dX^T/(M-1)."""
    xb, ix, iy, kind, yo, var = _tiny_linear_case(seed)
    k, _, ny, nx = xb.shape
    N = 9 * ny * nx
    xa = orc.letkf_analysis(xb, ix, iy, kind, yo, var, L=1.0, infl=infl, loc=orc.LOC_NONE)
    X = xb.reshape(k, N)
    H = np.zeros((len(yo), N))
    for j in range(len(yo)):
        for i in range(9):
            H[j, (i * ny + iy[j]) * nx + ix[j]] = 1.0
    Pf = infl * kf.ensemble_covariance(X)
    xa_kf, Pa_kf, _ = kf.kalman_update(X.mean(axis=0), Pf, H, np.diag(var), yo)
    Xa = xa.reshape(k, N)
    np.testing.assert_allclose(Xa.mean(axis=0), xa_kf, rtol=1e-12, atol=1e-14)
    Pa = kf.ensemble_covariance(Xa)
    scale = np.abs(Pa_kf).max()
    assert np.abs(Pa - Pa_kf).max() <= 1e-11 * scale


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("k,infl", [(4, 1.0), (16, 1.1), (64, 1.25)])
def test_single_observation_closed_form(k, infl):
    """One scalar observation: Q has eigenvalue a + w|y|^2 along y and
    a = (k-1)/rho elsewhere, so W and wbar have closed forms."""
    rng = np.random.default_rng(k)
    y = rng.standard_normal(k)
    y -= y.mean()
    w, d = 3.7, 0.4
    tr = orc.local_transform(y[None, :], np.array([d]), np.array([w]), k, infl)
    a = (k - 1) / infl
    n2 = float(y @ y)
    yh = y / math.sqrt(n2)
    P = np.outer(yh, yh)
    W_ref = math.sqrt(infl) * (np.eye(k) - P) + math.sqrt((k - 1) / (a + w * n2)) * P
    wbar_ref = w * d * y / (a + w * n2)
    np.testing.assert_allclose(tr["W"], W_ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tr["wbar"], wbar_ref, rtol=0, atol=1e-15)


def test_no_local_observation_gives_inflated_background():
    """Infinite error variance everywhere (R^-1 = 0): xa = xbar + sqrt(rho) dX,
    and with rho = 1 the background itself."""
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    var = np.full_like(p.obs_var, np.inf)
    for infl in (1.0, 1.21):
        an = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, var, 4.0, infl)
        pts = [0, 37, 1023]
        got = an.run(pts)
        for n, q in enumerate(pts):
            xp = p.xb[:, :, q // 32, q % 32]
            ref = xp.mean(axis=0) + math.sqrt(infl) * (xp - xp.mean(axis=0))
            np.testing.assert_allclose(got[n], ref, rtol=0, atol=1e-15)
    an = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, var, 4.0, 1.0)
    np.testing.assert_allclose(an.run([5])[0], p.xb[:, :, 0, 5], rtol=0, atol=1e-15)


def test_dense_single_obs_points_match_closed_form():
    """L = 0.4: each point sees only an observation at itself (r = 0), so the
    local problem is the single-observation one (the paper's dense case, l_max = 1)."""
    wl = synth.Workload("dense", 16, 16, 8, 2, 0.005, 0.4, 1.1, 7, kinds=(synth.OBS_U,))
    p = synth.make_problem(wl)
    an = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, wl.L, wl.infl)
    for (x, yy) in [(0, 0), (2, 4), (3, 3)]:
        xa, tr = an.point(x, yy, detail=True)
        xp = p.xb[:, :, yy, x]
        xbar = xp.mean(axis=0)
        dX = (xp - xbar).T
        if x % 2 or yy % 2:
            assert len(tr["sel"]) == 0
            np.testing.assert_allclose(xa, (xbar[:, None] + math.sqrt(wl.infl) * dX).T, atol=1e-15)
            continue
        assert len(tr["sel"]) == 1
        j = tr["sel"][0]
        yv = an.dY[j]
        w = 1.0 / p.obs_var[j]
        a = (wl.k - 1) / wl.infl
        n2 = yv @ yv
        P = np.outer(yv, yv) / n2
        W = math.sqrt(wl.infl) * (np.eye(wl.k) - P) + math.sqrt((wl.k - 1) / (a + w * n2)) * P
        wbar = w * an.d[j] * yv / (a + w * n2)
        ref = (xbar[:, None] + dX @ (wbar[:, None] + W)).T
        np.testing.assert_allclose(xa, ref, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def cfg0():
    p = synth.make_problem(synth.WORKLOADS["cpu32_k16"])
    an = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, p.wl.L, p.wl.infl)
    return p, an


@pytest.mark.parametrize("pt", [(0, 0), (5, 9), (31, 31), (16, 3)])
def test_transform_invariants(cfg0, pt):
    p, an = cfg0
    k, infl = p.wl.k, p.wl.infl
    xa, tr = an.point(*pt, detail=True)
    C, b, Q, lam, V, Pa, W, wbar = (tr[n] for n in ("C", "b", "Q", "lam", "V", "Pa", "W", "wbar"))
    one = np.ones(k)
    scale = np.abs(C).max()
    # perturbations sum to zero -> C 1 = 0, b . 1 = 0
    assert np.abs(C @ one).max() <= 1e-12 * scale * k
    assert abs(b @ one) <= 1e-12 * np.abs(b).max() * k
    # 1/sqrt(k) is an eigenvector of Q with eigenvalue (k-1)/rho
    a = (k - 1) / infl
    np.testing.assert_allclose(Q @ one, a * one, rtol=1e-12)
    assert lam.min() >= a * (1 - 1e-12)
    # eigen reconstruction and orthogonality
    eps = np.finfo(float).eps
    assert np.linalg.norm(V @ np.diag(lam) @ V.T - Q) <= 10 * k * eps * np.linalg.norm(Q)
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 10 * k * eps
    # Pa is the inverse of Q (direct Cholesky solve)
    Pa_direct = scipy.linalg.cho_solve(scipy.linalg.cho_factor(Q), np.eye(k))
    np.testing.assert_allclose(Pa, Pa_direct, rtol=1e-12, atol=1e-15 * np.abs(Pa).max())
    # W symmetric, W^2 = (k-1) Pa, W 1 = sqrt(rho) 1
    np.testing.assert_allclose(W, W.T, atol=1e-14)
    np.testing.assert_allclose(W @ W, (k - 1) * Pa, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(W @ one, math.sqrt(infl) * one, rtol=1e-12)
    # analysis perturbations sum to zero; analysis mean = xbar + dX wbar
    xp = p.xb[:, :, pt[1], pt[0]]
    xbar = xp.mean(axis=0)
    np.testing.assert_allclose(xa.mean(axis=0), xbar + (xp - xbar).T @ wbar, rtol=1e-13, atol=1e-16)
    assert np.abs((xa - xa.mean(axis=0)).sum(axis=0)).max() <= 1e-15 * k


def test_wide_gaussian_equals_no_localization():
    """L -> infinity: every observation is local with g -> 1 (the global ETKF)."""
    wl = synth.Workload("tiny", 16, 16, 8, 4, 0.01, 1.0, 1.1, 3)
    p = synth.make_problem(wl)
    a1 = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, 1e7, 1.1,
                      orc.LOC_GAUSS).run([0, 77, 255])
    a2 = orc.Analysis(p.xb, p.obs_ix, p.obs_iy, p.obs_kind, p.obs_val, p.obs_var, 1.0, 1.1,
                      orc.LOC_NONE).run([0, 77, 255])
    np.testing.assert_allclose(a1, a2, rtol=1e-9)


# ---------------------------------------------------------------- localization
def _window_count(x, y, nx, ny, stride, L):
    """Brute force over lattice offsets (independent of the oracle's obs-list
    distance code): observation points within Euclidean radius 2L, inclusive."""
    R = int(math.floor(2 * L))
    n = 0
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            if dx * dx + dy * dy <= 4 * L * L and ((x + dx) % nx) % stride == 0 \
                    and ((y + dy) % ny) % stride == 0:
                n += 1
    return n


@pytest.mark.parametrize("name,lo,hi", [("cpu32_k16", 10, 14), ("grid256_k32", 196, 208),
                                        ("grid1024_k64", 108, 116)])
def test_local_window_counts(name, lo, hi):
    wl = synth.WORKLOADS[name]
    counts = {_window_count(x, y, 10**6, 10**6, wl.stride, wl.L)
              for y in range(wl.stride) for x in range(wl.stride)}
    assert min(counts) == lo and max(counts) == hi


def test_oracle_weights_agree_with_window_enumeration():
    wl = synth.WORKLOADS["cpu32_k16"]
    p = synth.make_problem(wl)
    for (x, y) in [(0, 0), (1, 2), (31, 30), (17, 5)]:
        w = orc.local_weights(x, y, p.obs_ix, p.obs_iy, p.obs_var, wl.nx, wl.ny, wl.L, orc.LOC_GAUSS)
        assert np.count_nonzero(w) == 2 * _window_count(x, y, wl.nx, wl.ny, wl.stride, wl.L)
        # r = 2L exactly is inside (inclusive cutoff) with g = exp(-2)
        r2 = orc.periodic_r2(x, y, p.obs_ix, p.obs_iy, wl.nx, wl.ny)
        edge = r2 == 64
        if edge.any():
            np.testing.assert_allclose(w[edge] * p.obs_var[edge], math.exp(-2.0), rtol=1e-15)


def test_paper_local_window_sizes():
    """Sec. V-B: obs every p=4 points with cutoff d=6 gives l_max = 16 local
    observation points (a square extraction window) and a local-observation
    array 16*3/9 = 5.3x the state; Sec. V-A: N_x/M = 256 points per GPU."""
    g = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))
    sp = g["sparse"]
    n, p, d = sp["grid"], sp["p"], sp["d"]
    best = 0
    for y in range(p):
        for x in range(p):
            c = sum(1 for dy in range(-d, d + 1) for dx in range(-d, d + 1)
                    if (x + dx) % p == 0 and (y + dy) % p == 0)
            best = max(best, c)
    assert best == sp["l_max"]
    assert round(best * sp["V"] / sp["Nv"], 1) == sp["yloc_over_state"]
    # a Euclidean disc of radius d would give far fewer than the printed l_max
    disc = max(sum(1 for dy in range(-d, d + 1) for dx in range(-d, d + 1)
                   if dx * dx + dy * dy <= d * d and (x + dx) % p == 0 and (y + dy) % p == 0)
               for y in range(p) for x in range(p))
    assert disc < sp["l_max"]
    dn = g["dense"]
    assert dn["Nx"] // dn["M"] == dn["points_per_gpu"]
    assert _window_count(0, 0, 128, 128, 1, 0.0) == dn["l_max"]


def test_gaspari_cohn_shape():
    """GC(0)=1, both branches give 5/24 at r=c with matching slope, and the
    function and its slope vanish at r=2c (Gaspari & Cohn 1999, eq. 4.10)."""
    c = 3.0
    assert orc.gaspari_cohn(np.array([0.0]), c)[0] == 1.0
    z1 = orc.gaspari_cohn(np.array([c * (1 - 1e-9), c * (1 + 1e-9)]), c)
    np.testing.assert_allclose(z1, 5.0 / 24.0, rtol=1e-8)
    h = 1e-6
    s_lo = (orc.gaspari_cohn(np.array([c]), c) - orc.gaspari_cohn(np.array([c - h]), c)) / h
    s_hi = (orc.gaspari_cohn(np.array([c + h]), c) - orc.gaspari_cohn(np.array([c]), c)) / h
    np.testing.assert_allclose(s_lo, s_hi, rtol=1e-4)
    near = orc.gaspari_cohn(np.array([2 * c * (1 - 1e-4)]), c)[0]
    assert 0 < near < 1e-10
    assert orc.gaspari_cohn(np.array([2 * c, 3 * c]), c).tolist() == [0.0, 0.0]
    r = np.linspace(0, 2 * c, 200)
    assert np.all(np.diff(orc.gaspari_cohn(r, c)) <= 1e-15)
