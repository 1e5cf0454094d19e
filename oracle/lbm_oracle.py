"""CPU oracle of the D2Q9 lattice-BGK step used between analyses (Sec. II-A).

TEST INFRASTRUCTURE ONLY (see oracle/letkf_oracle.py).

One step is the lattice Boltzmann equation of Sec. II-A in collide-then-stream
order, f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i, with the lattice-BGK
collision (single relaxation time tau) and a body force.  Readings where the
paper gives no formula (listed in the design doc): the equilibrium is the standard
second-order D2Q9 polynomial, the force F enters as the source term
3 w_i (c_i . F) added after relaxation (no velocity shift), and the
Kolmogorov forcing is F_x(y) = A sin(2 pi n y / ny), F_y = 0.  Periodic box.
"""
from __future__ import annotations

import numpy as np

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)


def moments(f: np.ndarray):
    """rho = sum_i f_i, u = sum_i c_i f_i / rho (Sec. II-A); f [..., 9, ny, nx]."""
    rho = f.sum(axis=-3)
    ux = np.tensordot(CX.astype(np.float64), f, axes=([0], [f.ndim - 3])) / rho
    uy = np.tensordot(CY.astype(np.float64), f, axes=([0], [f.ndim - 3])) / rho
    return rho, ux, uy


def equilibrium(rho, ux, uy):
    out = []
    for i in range(9):
        cu = CX[i] * ux + CY[i] * uy
        out.append(WQ[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)))
    return np.stack(out, axis=-3)


def kolmogorov_force(ny: int, amp: float, kx: int):
    y = np.arange(ny, dtype=np.float64)
    return amp * np.sin(2.0 * np.pi * kx * y / ny)          # F_x(y); F_y = 0


def bgk_step(f: np.ndarray, tau: float, amp: float = 0.0, kx: int = 1) -> np.ndarray:
    """One collide-then-stream step of every member: f [k, 9, ny, nx] -> new f."""
    ny = f.shape[-2]
    rho, ux, uy = moments(f)
    feq = equilibrium(rho, ux, uy)
    post = f - (f - feq) / tau
    if amp != 0.0:
        Fx = kolmogorov_force(ny, amp, kx)[:, None]          # [ny, 1]
        for i in range(9):
            post[..., i, :, :] += 3.0 * WQ[i] * CX[i] * Fx
    out = np.empty_like(f)
    for i in range(9):
        out[..., i, :, :] = np.roll(post[..., i, :, :], shift=(CY[i], CX[i]), axis=(-2, -1))
    return out


def advance(f: np.ndarray, n_steps: int, tau: float, amp: float = 0.0, kx: int = 1) -> np.ndarray:
    for _ in range(n_steps):
        f = bgk_step(f, tau, amp, kx)
    return f
