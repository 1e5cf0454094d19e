"""Seeded synthetic inputs for LETKF analyses of a D2Q9 lattice-Boltzmann ensemble.

This module only *makes inputs*: background ensembles ``f[k][9][ny][nx]`` and
observation lists.  It holds none of the assimilation arithmetic (no
observation operator, no weights, no transform), so both the CPU oracle's
tests and the GPU path can take the very same arrays from it.

Recipe (the paper's nature run and turbulence set-up are not available, so a
2D turbulence-like field stands in for them, cf. the OSSE description in
Sec. V of the paper):

* truth streamfunction  psi = sum_{0<|kappa|<=8} a_kappa cos(2 pi kappa.x/n + phi_kappa)
  with a ~ N(0,1), phi ~ U[0, 2 pi); u = d psi/dy, v = -d psi/dx, scaled so
  that max |(u, v)| = 0.05 (lattice units);
* member m: truth + an independent field from the same generator scaled to an
  RMS of 0.01 per velocity component; rho = 1 + N(0, 1e-3^2) per point/member;
  f = D2Q9 equilibrium of (rho, u, v);
* observations: (u, v) of the truth at every ``stride``-th point in x and y
  plus N(0, sigma^2) noise, error variance sigma^2.

The D2Q9 direction order used for ``f`` is
``c = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Direction order and weights of the D2Q9 equilibrium used to build inputs.
_CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
_CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
_WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)

OBS_RHO, OBS_U, OBS_V = 0, 1, 2


@dataclasses.dataclass
class Workload:
    """One analysis problem: grid, ensemble size, localization and obs layout."""
    name: str
    nx: int
    ny: int
    k: int
    stride: int          # observations at every stride-th point in x and y
    sigma: float         # observation error standard deviation
    L: float             # localization length (lattice units)
    infl: float          # multiplicative inflation rho
    seed: int
    kinds: tuple = (OBS_U, OBS_V)
    # random observation mask instead of the stride lattice: Bernoulli(density)
    # per point, minus n_gaps discs with radii in gap_radius (clustered gaps)
    density: float = 0.0
    n_gaps: int = 0
    gap_radius: tuple = (8, 32)


# The five shapes the method is exercised on (see the bench / tests).
WORKLOADS = {
    "cpu32_k16": Workload("cpu32_k16", 32, 32, 16, 4, 0.005, 4.0, 1.1, 0),
    "grid256_k32": Workload("grid256_k32", 256, 256, 32, 2, 0.005, 8.0, 1.1, 1),
    "grid1024_k64": Workload("grid1024_k64", 1024, 1024, 64, 4, 0.005, 12.0, 1.1, 2),
}


def equilibrium(rho: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """D2Q9 equilibrium; returns f with the direction axis inserted at -3.

    rho, u, v have shape [..., ny, nx]; the result has [..., 9, ny, nx].
    """
    cu = (_CX[:, None, None] * u[..., None, :, :] + _CY[:, None, None] * v[..., None, :, :])
    uu = (u * u + v * v)[..., None, :, :]
    return _WQ[:, None, None] * rho[..., None, :, :] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


def _fill_modes(rng: np.random.Generator, spec: np.ndarray, nx: int, ny: int, kmax: int):
    """Random amplitudes and phases of the modes 0 < |kappa| <= kmax (one of
    each +-kappa pair), added into the spectrum array."""
    for ky in range(-kmax, kmax + 1):
        for kx in range(-kmax, kmax + 1):
            if kx * kx + ky * ky == 0 or kx * kx + ky * ky > kmax * kmax:
                continue
            if ky < 0 or (ky == 0 and kx < 0):
                continue  # one of each +-kappa pair
            a = rng.standard_normal()
            ph = rng.uniform(0.0, 2.0 * np.pi)
            spec[ky % ny, kx % nx] += a * np.exp(1j * ph)


def random_mode_velocity(rng: np.random.Generator, nx: int, ny: int, kmax: int = 8):
    """Divergence-free velocity from a random-mode streamfunction, |kappa| <= kmax.

    Returns (u, v), each [ny, nx], unnormalised.
    """
    spec = np.zeros((ny, nx), dtype=np.complex128)
    _fill_modes(rng, spec, nx, ny, kmax)
    kxs = np.fft.fftfreq(nx, 1.0 / nx)[None, :]
    kys = np.fft.fftfreq(ny, 1.0 / ny)[:, None]
    scale = nx * ny
    u = np.real(np.fft.ifft2(spec * (1j * 2 * np.pi * kys / ny))) * scale
    v = -np.real(np.fft.ifft2(spec * (1j * 2 * np.pi * kxs / nx))) * scale
    return u, v


@dataclasses.dataclass
class Problem:
    """A generated analysis input (host numpy arrays, float64/int32)."""
    wl: Workload
    xb: np.ndarray        # [k, 9, ny, nx] float64
    obs_ix: np.ndarray    # [n_obs] int32
    obs_iy: np.ndarray
    obs_kind: np.ndarray
    obs_val: np.ndarray   # [n_obs] float64
    obs_var: np.ndarray
    truth_u: np.ndarray   # [ny, nx]
    truth_v: np.ndarray


def make_problem(wl: Workload, seed: Optional[int] = None, dtype=np.float64) -> Problem:
    """Build the background ensemble and observations of one workload."""
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    nx, ny, k = wl.nx, wl.ny, wl.k
    ut, vt = random_mode_velocity(rng, nx, ny)
    s = 0.05 / np.sqrt(np.max(ut * ut + vt * vt))
    ut, vt = ut * s, vt * s
    xb = np.empty((k, 9, ny, nx), dtype=dtype)
    for m in range(k):
        up, vp = random_mode_velocity(rng, nx, ny)
        sp = 0.01 / np.sqrt(0.5 * np.mean(up * up + vp * vp))
        rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
        xb[m] = equilibrium(rho, ut + sp * up, vt + sp * vp)
    return _observations(rng, wl, ut, vt, xb)


def _observations(rng: np.random.Generator, wl: Workload, ut, vt, xb) -> Problem:
    """The observation list of a workload from the truth velocity (the draws
    that follow the ensemble's in the generator)."""
    nx, ny = wl.nx, wl.ny
    if wl.density > 0.0:
        mask = obs_mask(rng, nx, ny, wl.density, wl.n_gaps, wl.gap_radius)
        iy, ix = np.nonzero(mask)
    else:
        iy, ix = np.meshgrid(np.arange(0, ny, wl.stride), np.arange(0, nx, wl.stride),
                             indexing="ij")
    iy = iy.ravel().astype(np.int32)
    ix = ix.ravel().astype(np.int32)
    n_pts = ix.size
    nk = len(wl.kinds)
    obs_ix = np.repeat(ix, nk)
    obs_iy = np.repeat(iy, nk)
    obs_kind = np.tile(np.array(wl.kinds, dtype=np.int32), n_pts)
    truth = {OBS_U: ut, OBS_V: vt, OBS_RHO: np.ones_like(ut)}
    val = _gather_truth(truth, obs_kind, obs_iy, obs_ix)
    val = val + wl.sigma * rng.standard_normal(val.shape)
    var = np.full(val.shape, wl.sigma ** 2)
    return Problem(wl, xb, obs_ix.astype(np.int32), obs_iy.astype(np.int32),
                   obs_kind.astype(np.int32), val.astype(np.float64), var, ut, vt)


def make_problem_device(wl: Workload, device, seed: Optional[int] = None):
    """make_problem with the background ensemble built on a torch device: the
    same draws from the same generator, in the same order, with the inverse
    FFTs and the equilibrium evaluated there (so the members never pass
    through host memory).  The inputs equal make_problem's up to the rounding
    of the FFTs.  Returns (xb device tensor [k, 9, ny, nx] float64, Problem
    whose xb is None)."""
    import torch
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    nx, ny, k = wl.nx, wl.ny, wl.k
    kxs = torch.fft.fftfreq(nx, 1.0 / nx, dtype=torch.float64, device=device)[None, :]
    kys = torch.fft.fftfreq(ny, 1.0 / ny, dtype=torch.float64, device=device)[:, None]
    cx = torch.tensor(_CX, dtype=torch.float64, device=device)[:, None, None]
    cy = torch.tensor(_CY, dtype=torch.float64, device=device)[:, None, None]
    wq = torch.tensor(_WQ, dtype=torch.float64, device=device)[:, None, None]

    def velocity():
        spec = np.zeros((ny, nx), dtype=np.complex128)
        _fill_modes(rng, spec, nx, ny, 8)
        sp = torch.from_numpy(spec).to(device)
        u = torch.fft.ifft2(sp * (1j * 2 * np.pi * kys / ny)).real * (nx * ny)
        v = -torch.fft.ifft2(sp * (1j * 2 * np.pi * kxs / nx)).real * (nx * ny)
        return u, v

    ut, vt = velocity()
    s = 0.05 / torch.sqrt(torch.max(ut * ut + vt * vt))
    ut, vt = ut * s, vt * s
    xb = torch.empty((k, 9, ny, nx), dtype=torch.float64, device=device)
    for m in range(k):
        up, vp = velocity()
        sp = 0.01 / torch.sqrt(0.5 * torch.mean(up * up + vp * vp))
        rho = 1.0 + 1e-3 * torch.from_numpy(rng.standard_normal((ny, nx))).to(device)
        u, v = ut + sp * up, vt + sp * vp
        cu = cx * u + cy * v
        xb[m] = wq * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u * u + v * v))
    truth = (ut.cpu().numpy(), vt.cpu().numpy())
    prob = _observations(rng, wl, truth[0], truth[1], None)
    return xb, prob


def obs_mask(rng: np.random.Generator, nx: int, ny: int, density: float, n_gaps: int,
             gap_radius=(8, 32)) -> np.ndarray:
    """[ny, nx] bool: Bernoulli(density) observation sites with n_gaps
    periodic discs (radius uniform in gap_radius, capped at a quarter of the
    box) emptied -- observation gaps clustered in space."""
    mask = rng.random((ny, nx)) < density
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for _ in range(n_gaps):
        r = min(rng.uniform(*gap_radius), min(nx, ny) / 4)
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        dx = np.abs(xx - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(yy - cy)
        dy = np.minimum(dy, ny - dy)
        mask &= dx * dx + dy * dy > r * r
    return mask


def batching_workloads(n: int, seed: int = 3, grids=(64, 128, 256, 512), ks=(16, 32, 64)):
    """The mixed batch: n independent problems with lattice sizes drawn from
    grids, k from ks, L ~ U[4, 16], sigma ~ U[0.002, 0.01], rho = 1.1, random
    observation masks of density U[0.05, 0.5] with 1-6 clustered gaps of
    radius 8-32 (so local observation counts range from 0 to several
    hundred).  Every draw comes from one seeded generator."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        g = int(rng.choice(grids))
        out.append(Workload(f"batch{seed}_{i}", g, g, int(rng.choice(ks)), 1,
                            float(rng.uniform(0.002, 0.01)), float(rng.uniform(4.0, 16.0)), 1.1,
                            int(rng.integers(1 << 30)), density=float(rng.uniform(0.05, 0.5)),
                            n_gaps=int(rng.integers(1, 7))))
    return out


def _gather_truth(truth, kind, iy, ix):
    out = np.empty(kind.shape, dtype=np.float64)
    for kd, fld in truth.items():
        sel = kind == kd
        out[sel] = fld[iy[sel], ix[sel]]
    return out


def sample_points(nx: int, ny: int, n: int, seed: int = 12345) -> np.ndarray:
    """Seeded sample of flat point indices (iy*nx+ix): the four corners, the
    edges' midpoints and n random interior points, without repeats."""
    rng = np.random.default_rng(seed)
    fixed = [0, nx - 1, (ny - 1) * nx, ny * nx - 1, (ny // 2) * nx, (ny // 2) * nx + nx - 1, nx // 2,
             (ny - 1) * nx + nx // 2]
    pts = list(dict.fromkeys(p for p in fixed if 0 <= p < nx * ny))
    seen = set(pts)
    extra = rng.choice(nx * ny, size=min(n, nx * ny), replace=False)
    for p in extra:
        if len(pts) >= n + len(fixed):
            break
        if int(p) not in seen:
            seen.add(int(p))
            pts.append(int(p))
    return np.array(sorted(pts), dtype=np.int64)
