"""GPU parity of letkf_invsqrt_batched (Newton-Schulz inverse square root on
MFMA) against the oracle's symmetric square-root transform: for LETKF-form
Q = ((k-1)/rho) I + dY^T R^-1 dY built by the oracle (eq. letkf_q),
sqrt(k-1) Q^-1/2 from the GPU must equal the oracle's W (eq. letkf_dwa,
formed there from numpy's EVD) within the FP64 bar 1e-10, relative in the
Frobenius norm and per entry against max|W|.  Also: c I -> c^-1/2 I exactly
enough, a graded spectrum, and the not-converged status bit on an indefinite
input (the iteration diverges; the kernel stops after its bounded steps)."""
import math
import sys

import numpy as np
import pytest

from oracle import letkf_oracle as orc
from paper_2308_03310_amd import letkf as L

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(A, with_steps=False):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    x = torch.empty_like(a)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    steps = torch.full((len(A),), -1, dtype=torch.int32, device="cuda")
    L.letkf_invsqrt_batched(a, x, st, steps)
    torch.cuda.synchronize()
    if with_steps:
        return x.cpu().numpy(), int(st.cpu()[0]), steps.cpu().numpy()
    return x.cpu().numpy(), int(st.cpu()[0])


def _letkf_q(k, n, rng):
    """n oracle transforms at random local problems: p observations, weights
    from Gaussian localization, ensemble spreads and observation errors around
    those of the LBM runs (sigma 1e-3 .. 1e-2; cond Q up to about 1e4)."""
    Qs, Ws = [], []
    for _ in range(n):
        p = int(rng.integers(1, 4 * k))
        dY = rng.standard_normal((p, k)) * rng.uniform(1e-3, 3e-2)
        dY -= dY.mean(axis=1, keepdims=True)
        d = rng.standard_normal(p) * 1e-2
        w = np.exp(-rng.uniform(0, 4, p)) / rng.uniform(1e-3, 1e-2) ** 2
        t = orc.local_transform(dY, d, w, k, 1.1)
        Qs.append(t["Q"])
        Ws.append(t["W"])
    return np.array(Qs), np.array(Ws)


@pytest.mark.parametrize("k", [2, 3, 15, 16, 17, 32, 33, 48, 64])
def test_invsqrt_matches_oracle_transform(k):
    n = 64
    say(f"invsqrt_batched letkf-form k={k} batch={n}")
    rng = np.random.default_rng(300 + k)
    Q, W = _letkf_q(k, n, rng)
    X, st, steps = _run(Q, with_steps=True)
    assert st == 0
    # about log_2.25(cond Q) + 5 steps; cond Q here stays below 1e4
    assert steps.min() >= 1 and steps.max() <= 20, steps
    Wg = math.sqrt(k - 1) * X
    for i in range(n):
        assert np.linalg.norm(Wg[i] - W[i]) <= 1e-10 * np.linalg.norm(W[i]), i
        assert np.abs(Wg[i] - W[i]).max() <= 1e-10 * np.abs(W[i]).max(), i
        assert np.array_equal(Wg[i], Wg[i].T) or np.abs(Wg[i] - Wg[i].T).max() <= 1e-13 * np.abs(
            W[i]).max()


@pytest.mark.parametrize("k", [1, 16, 64])
def test_invsqrt_scaled_identity(k):
    say(f"invsqrt_batched c*I k={k}")
    c = np.array([1.0, 4.0, 1e-6, 3e5])
    A = c[:, None, None] * np.eye(k)[None]
    X, st, steps = _run(A, with_steps=True)
    assert st == 0
    assert np.all(steps == 1)          # B = I after scaling: the first residual is 0
    for i, ci in enumerate(c):
        np.testing.assert_allclose(X[i], np.eye(k) / math.sqrt(ci), rtol=1e-13, atol=0)


@pytest.mark.parametrize("k", [16, 40, 64])
def test_invsqrt_graded_spectrum(k):
    # eigenvalues 1 .. 1e6 (condition 1e6, about 22 steps, ending at the
    # rounding floor of the residual): the result against V diag(lam^-1/2) V^T
    # from the exact eigenpairs the matrix was built from
    say(f"invsqrt_batched graded k={k}")
    rng = np.random.default_rng(7 + k)
    n = 16
    A = np.empty((n, k, k))
    R = np.empty((n, k, k))
    for b in range(n):
        q, r = np.linalg.qr(rng.standard_normal((k, k)))
        q *= np.sign(np.diag(r))
        lam = np.logspace(0, 6, k)
        A[b] = (q * lam) @ q.T
        A[b] = 0.5 * (A[b] + A[b].T)
        R[b] = (q / np.sqrt(lam)) @ q.T
    X, st = _run(A)
    assert st == 0
    for b in range(n):
        assert np.linalg.norm(X[b] - R[b]) <= 1e-10 * np.linalg.norm(R[b]), b


def test_invsqrt_indefinite_sets_status():
    say("invsqrt_batched indefinite input -> ENOTCONV bit")
    k = 8
    A = np.stack([np.eye(k), np.diag(np.r_[-1.0, np.ones(k - 1)])])
    X, st, steps = _run(A, with_steps=True)
    assert st & (1 << L.LETKF_ENOTCONV)
    assert steps[0] == 1 and steps[1] > 1
    np.testing.assert_allclose(X[0], np.eye(k), rtol=1e-13, atol=1e-15)
