"""CPU oracle for the LETKF local analysis over a D2Q9 lattice-Boltzmann ensemble.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything under ``oracle/``;
the GPU library never calls it and shares no code with it.

It is a plain, slow FP64 implementation of what the paper defines, written for
readability: one grid point at a time, following the three-step LETKF
procedure of Sec. II-B (forecast observations, local observations, local
transform + update; Algorithm 1 "Basic implementation of the LETKF") and the
equations of Sec. II-B:

* ensemble mean / perturbations          eq. (xmean), (xspread)
* analysis members                       eq. (letkf_xa)
* mean weight  wbar = Pa dY^T R^-1 (yo - ybar)        eq. (letkf_wa)
* perturbation weights dW = sqrt(M-1) Pa^(1/2)         eq. (letkf_dwa)
* Pa = Q^-1,  Q = (M-1) I + dY^T R^-1 dY              eq. (letkf_q)
* forecast observation mean / perturbations           eq. (enkf_ybar), (enkf_deltay)
* R-localization R_loc^-1 = G o R^-1 with diagonal G   Sec. II-B, R-localization paragraph
* observed variables: density and velocity moments     Sec. II-A, moment equations

Readings where the paper is silent (each also listed in the design doc):

* inflation rho enters as Q = ((M-1)/rho) I + dY^T R_loc^-1 dY, i.e. P^f is
  multiplied by rho; rho = 1 gives the paper's eq. (letkf_q) unchanged;
* localization "gauss": g(r) = exp(-r^2 / (2 L^2)) for r^2 <= (2L)^2, else 0
  (inclusive cutoff, r = periodic minimum-image Euclidean lattice distance);
  "gc": the Gaspari-Cohn 5th-order function with half-width c = L (zero for
  r >= 2L); "none": g = 1 for every observation;
* an observation with infinite error variance has R^-1 = 0 and is ignored;
* the symmetric square root (Pa)^(1/2) is the principal one, taken through the
  eigendecomposition of Q (unique, so eigenvector signs and the order of equal
  eigenvalues do not matter).

D2Q9 direction order: c = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, Optional

import numpy as np

LOC_GAUSS, LOC_GC, LOC_NONE = 0, 1, 2
OBS_RHO, OBS_U, OBS_V = 0, 1, 2

# Discrete velocities c_ij of the D2Q9 lattice (Sec. II-A), in the API's order.
D2Q9_CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
D2Q9_CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)


# --------------------------------------------------------------------------
# Step 1: forecast observations Y^f = H(X^f)  (Sec. II-B step 1; Sec. II-A moments)
# --------------------------------------------------------------------------
def observe_member(f_pt: np.ndarray, kind: int) -> float:
    """Observed variable of one member at one lattice point.

    f_pt: the 9 distribution functions at the point.  rho = sum_i f_i and
    u = (1/rho) sum_i c_i f_i (Sec. II-A moment equations).
    """
    rho = float(np.sum(f_pt))
    if kind == OBS_RHO:
        return rho
    if kind == OBS_U:
        return float(np.dot(D2Q9_CX, f_pt)) / rho
    if kind == OBS_V:
        return float(np.dot(D2Q9_CY, f_pt)) / rho
    raise ValueError(f"unknown observation kind {kind}")


def forecast_observations(xb: np.ndarray, obs_ix, obs_iy, obs_kind) -> np.ndarray:
    """y[m, j] = H_j(x_m) for every member m and observation j -> [k, n_obs]."""
    k = xb.shape[0]
    n_obs = len(obs_ix)
    y = np.empty((k, n_obs), dtype=np.float64)
    f = xb[:, :, np.asarray(obs_iy), np.asarray(obs_ix)]  # [k, 9, n_obs]
    rho = f.sum(axis=1)
    ju = np.einsum("i,kin->kn", D2Q9_CX, f)
    jv = np.einsum("i,kin->kn", D2Q9_CY, f)
    kind = np.asarray(obs_kind)
    y[:] = np.where(kind == OBS_RHO, rho, np.where(kind == OBS_U, ju / rho, jv / rho))
    return y


def obs_mean_and_perturbations(y: np.ndarray):
    """ybar = (1/M) sum_m y_m (eq. enkf_ybar); dY[j, m] = y_m - ybar (eq. enkf_deltay)."""
    ybar = y.mean(axis=0)
    dY = (y - ybar[None, :]).T.copy()  # [n_obs, k]
    return ybar, dY


# --------------------------------------------------------------------------
# Step 2: local observations through R-localization (Sec. II-B)
# --------------------------------------------------------------------------
def gaspari_cohn(r: np.ndarray, c: float) -> np.ndarray:
    """Gaspari & Cohn (1999) 5th-order compactly supported function, eq. (4.10),
    half-width c: 1 at r = 0, zero for r >= 2c."""
    z = np.abs(np.asarray(r, dtype=np.float64)) / c
    out = np.zeros_like(z)
    a = z <= 1.0
    za = z[a]
    out[a] = -0.25 * za**5 + 0.5 * za**4 + 0.625 * za**3 - (5.0 / 3.0) * za**2 + 1.0
    b = (z > 1.0) & (z < 2.0)
    zb = z[b]
    out[b] = (zb**5 / 12.0 - 0.5 * zb**4 + 0.625 * zb**3 + (5.0 / 3.0) * zb**2
              - 5.0 * zb + 4.0 - 2.0 / (3.0 * zb))
    return out


def periodic_r2(x: int, y: int, obs_ix, obs_iy, nx: int, ny: int) -> np.ndarray:
    """Squared minimum-image lattice distance from (x, y) to each observation."""
    dx = np.abs(np.asarray(obs_ix, dtype=np.int64) - x)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(np.asarray(obs_iy, dtype=np.int64) - y)
    dy = np.minimum(dy, ny - dy)
    return dx * dx + dy * dy


def localization(r2: np.ndarray, L: float, loc: int) -> np.ndarray:
    """Diagonal of G at squared distances r2 (the build's readings, see module doc)."""
    r2 = np.asarray(r2, dtype=np.float64)
    if loc == LOC_NONE:
        return np.ones_like(r2)
    if loc == LOC_GAUSS:
        return np.where(r2 <= 4.0 * L * L, np.exp(-r2 / (2.0 * L * L)), 0.0)
    if loc == LOC_GC:
        return gaspari_cohn(np.sqrt(r2), L)
    raise ValueError(f"unknown localization {loc}")


def local_weights(x: int, y: int, obs_ix, obs_iy, obs_var, nx: int, ny: int, L: float, loc: int):
    """Diagonal of R_loc^-1 = G o R^-1 at grid point (x, y): g_j / sigma_j^2."""
    g = localization(periodic_r2(x, y, obs_ix, obs_iy, nx, ny), L, loc)
    var = np.asarray(obs_var, dtype=np.float64)
    rinv = np.where(np.isinf(var), 0.0, 1.0 / var)
    return g * rinv


# --------------------------------------------------------------------------
# Step 3: local transform (Sec. II-B, eqs. letkf_wa, letkf_dwa, letkf_q)
# --------------------------------------------------------------------------
def local_transform(dY_loc: np.ndarray, d_loc: np.ndarray, w_loc: np.ndarray, k: int,
                    infl: float) -> Dict[str, np.ndarray]:
    """Ensemble-space solution at one grid point.

    dY_loc [p, k]: local forecast-observation perturbations; d_loc [p]:
    yo - ybar; w_loc [p]: diagonal of R_loc^-1.  Returns the Gram matrix C,
    the right-hand side b, Q, its eigenpairs, Pa, wbar and W = dW^a.
    """
    C = dY_loc.T @ (w_loc[:, None] * dY_loc)            # dY^T R_loc^-1 dY
    b = dY_loc.T @ (w_loc * d_loc)                     # dY^T R_loc^-1 (yo - ybar)
    Q = ((k - 1) / infl) * np.eye(k) + C               # eq. (letkf_q), inflated
    lam, V = np.linalg.eigh(Q)                         # EVD of Q (Sec. II-B, Sec. III)
    Pa = (V / lam[None, :]) @ V.T                      # Pa = Q^-1
    wbar = Pa @ b                                      # eq. (letkf_wa)
    W = math.sqrt(k - 1) * (V / np.sqrt(lam)[None, :]) @ V.T   # eq. (letkf_dwa)
    return {"C": C, "b": b, "Q": Q, "lam": lam, "V": V, "Pa": Pa, "wbar": wbar, "W": W}


def update_point(xp: np.ndarray, wbar: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Analysis members at one grid point, eq. (letkf_xa).

    xp [k, 9]: forecast members' 9 distribution functions at the point (the
    nine components share one transform, Sec. II-B).  Returns [k, 9].
    """
    xbar = xp.mean(axis=0)                 # eq. (xmean)
    dX = (xp - xbar[None, :]).T            # [9, k], eq. (xspread)
    Xa = xbar[:, None] + dX @ (wbar[:, None] + W)   # column m: xbar + dX (wbar + dw_m)
    return Xa.T


class Analysis:
    """Precomputed forecast observations for one analysis; evaluates points on demand."""

    def __init__(self, xb, obs_ix, obs_iy, obs_kind, obs_val, obs_var, L, infl, loc=LOC_GAUSS):
        self.xb = np.asarray(xb, dtype=np.float64)
        self.k, _, self.ny, self.nx = self.xb.shape
        self.obs_ix = np.asarray(obs_ix)
        self.obs_iy = np.asarray(obs_iy)
        self.obs_var = np.asarray(obs_var, dtype=np.float64)
        self.L, self.infl, self.loc = float(L), float(infl), int(loc)
        y = forecast_observations(self.xb, obs_ix, obs_iy, obs_kind)     # step 1
        self.ybar, self.dY = obs_mean_and_perturbations(y)
        self.d = np.asarray(obs_val, dtype=np.float64) - self.ybar

    def point(self, x: int, y: int, detail: bool = False):
        """Analysis at grid point (x, y): returns xa [k, 9] (and the transform)."""
        w = local_weights(x, y, self.obs_ix, self.obs_iy, self.obs_var, self.nx, self.ny,
                          self.L, self.loc)                              # step 2
        sel = np.nonzero(w > 0.0)[0]
        tr = local_transform(self.dY[sel], self.d[sel], w[sel], self.k, self.infl)   # step 3
        xa = update_point(self.xb[:, :, y, x], tr["wbar"], tr["W"])
        if detail:
            tr["sel"] = sel
            tr["w"] = w[sel]
            return xa, tr
        return xa

    def run(self, points: Optional[Iterable[int]] = None) -> np.ndarray:
        """Whole field (points=None -> xa [k, 9, ny, nx]) or the listed flat
        point indices iy*nx+ix (-> [n_points, k, 9])."""
        if points is None:
            xa = np.empty_like(self.xb)
            for iy in range(self.ny):
                for ix in range(self.nx):
                    xa[:, :, iy, ix] = self.point(ix, iy)
            return xa
        pts = list(points)
        out = np.empty((len(pts), self.k, 9), dtype=np.float64)
        for n, p in enumerate(pts):
            out[n] = self.point(int(p) % self.nx, int(p) // self.nx)
        return out


def letkf_analysis(xb, obs_ix, obs_iy, obs_kind, obs_val, obs_var, L, infl, loc=LOC_GAUSS,
                   points=None):
    """One LETKF analysis (Algorithm 1): forecast ensemble in, analysis ensemble out."""
    return Analysis(xb, obs_ix, obs_iy, obs_kind, obs_val, obs_var, L, infl, loc).run(points)
