"""Element-wise parity checks of an analysis ensemble against the oracle.

Arrays are either whole fields [k, 9, ny, nx] or sampled points [n, k, 9];
both are viewed as one row of 9 k values per grid point.  A check passes
only if every one of these holds:

* relative L2 over every entry            <= tol;
* relative L2 of each grid point's values <= tol (no point hides in the norm);
* |got - ref| <= tol * max|ref| for every entry;
* each point's error relative to its own analysis increment ||ref - xb||
  <= inc_tol (when given): the increment is what the analysis changes, so a
  bar on the whole state alone would say little about it.
"""
import numpy as np


def per_point(a):
    a = np.asarray(a)
    if a.ndim == 4:                                  # [k, 9, ny, nx]
        k = a.shape[0]
        return np.moveaxis(a.reshape(k * 9, -1), 0, -1)
    return a.reshape(a.shape[0], -1)                 # [n, k, 9]


def parity_errors(got, ref, xb=None):
    g, r = per_point(got), per_point(ref)
    d = g - r
    out = {
        "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(r)),
        "max_point_rel": float(np.max(np.linalg.norm(d, axis=1) / np.linalg.norm(r, axis=1))),
        "max_abs_rel": float(np.max(np.abs(d)) / np.max(np.abs(r))),
    }
    if xb is not None:
        inc = np.linalg.norm(r - per_point(xb), axis=1)
        out["inc_rel"] = float(np.linalg.norm(d) / np.linalg.norm(r - per_point(xb)))
        out["max_point_inc_rel"] = float(np.max(np.linalg.norm(d, axis=1) / inc))
    return out


def assert_parity(got, ref, tol, xb=None, inc_tol=None, label=""):
    e = parity_errors(got, ref, xb)
    msg = f"{label}: " + " ".join(f"{k} {v:.2e}" for k, v in e.items())
    print("  " + msg, flush=True)
    assert e["rel_l2"] <= tol, msg
    assert e["max_point_rel"] <= tol, msg
    assert e["max_abs_rel"] <= tol, msg
    if inc_tol is not None:
        assert e["max_point_inc_rel"] <= inc_tol, msg
    return e


def mean_spread_errors(got, ref):
    """Relative L2 errors of the analysis mean and of the spread (the
    perturbations about the mean), each against its own norm; member axis is
    the first of a field [k, ...] and the second of samples [n, k, 9]."""
    got, ref = np.asarray(got), np.asarray(ref)
    ax = 0 if got.ndim == 4 else 1
    gm, rm = got.mean(axis=ax, keepdims=True), ref.mean(axis=ax, keepdims=True)
    mean = np.linalg.norm(gm - rm) / np.linalg.norm(rm)
    spread = np.linalg.norm((got - gm) - (ref - rm)) / np.linalg.norm(ref - rm)
    return float(mean), float(spread)
