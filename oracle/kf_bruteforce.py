"""Brute-force Kalman filter in model space (Sec. II-B, eqs. kfx, kfp, kfk).

TEST INFRASTRUCTURE ONLY (see oracle/letkf_oracle.py).  Used on tiny grids to
pin the LETKF oracle: with a linear observation operator and no localization
the ensemble transform is an exact square-root form of these equations, with
the forecast covariance taken from the ensemble (eq. enkf_p) times the
inflation factor.
"""
from __future__ import annotations

import numpy as np


def kalman_update(xf: np.ndarray, Pf: np.ndarray, H: np.ndarray, R: np.ndarray, yo: np.ndarray):
    """xa = xf + K (yo - H xf),  Pa = (I - K H) Pf,  K = Pf H^T (H Pf H^T + R)^-1."""
    S = H @ Pf @ H.T + R
    K = np.linalg.solve(S.T, (Pf @ H.T).T).T      # Pf H^T S^-1 without forming S^-1
    xa = xf + K @ (yo - H @ xf)
    Pa = (np.eye(Pf.shape[0]) - K @ H) @ Pf
    return xa, Pa, K


def ensemble_covariance(X: np.ndarray) -> np.ndarray:
    """P = dX dX^T / (M-1) with dX the perturbations about the ensemble mean (eq. enkf_p).

    X: [M, N] members as rows.
    """
    dX = X - X.mean(axis=0, keepdims=True)
    return dX.T @ dX / (X.shape[0] - 1)
