"""Differentiable solve x = A^-1 b (paper_1305_2353_amd.autograd) on the GPU:
analytic gradients against the oracle's adjoint, and directional
derivatives against finite differences computed with the GPU solve itself
(fourth-order central differences, h = 1e-3, each forward solve refined in
FP64: the error of this scheme on these matrices, |lambda| >= 1e-2, is
about 1e-10 to 1e-9; the plain two-point difference at h = 1e-6 with one refinement
step stops near 4e-7)."""

import numpy as np
import pytest
import torch

from gpu_helpers import require_gpu, rel_err
from oracle.dense import solve_adjoint
from workloads import dense_indefinite

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _batch(S, N, nrhs, seed):
    As, Bs = [], []
    for s in range(S):
        A, lam, B = dense_indefinite(N, seed=seed + s, lam_lo=1e-2, nrhs=nrhs)
        As.append(A)
        Bs.append(B)
    return np.stack(As), np.stack(Bs)


@pytest.mark.parametrize("S,N,nrhs,pw", [(3, 256, 4, 64), (2, 600, 2, 256)])
def test_gradients_match_oracle_adjoint(S, N, nrhs, pw):
    from paper_1305_2353_amd.autograd import ldlt_solve
    print("case: autograd", S, N, nrhs, pw, flush=True)
    As, Bs = _batch(S, N, nrhs, seed=100 + N)
    rng = np.random.default_rng(0)
    W = rng.standard_normal(Bs.shape)
    A = torch.tensor(As, device="cuda", requires_grad=True)
    B = torch.tensor(Bs, device="cuda", requires_grad=True)
    X = ldlt_solve(A, B, pw=pw)
    loss = (torch.tensor(W, device="cuda") * X).sum()
    loss.backward()
    for s in range(S):
        x_ref = np.linalg.solve(As[s], Bs[s])
        assert rel_err(X[s].detach().cpu().numpy(), x_ref) < 1e-10
        bbar, abar = solve_adjoint(As[s], x_ref, W[s])
        assert rel_err(A.grad[s].cpu().numpy(), abar) < 1e-8
        assert rel_err(B.grad[s].cpu().numpy(), bbar) < 1e-8
        g = A.grad[s].cpu().numpy()
        assert np.array_equal(g, g.T)


def test_directional_derivatives_match_finite_differences():
    from paper_1305_2353_amd import ctp
    from paper_1305_2353_amd.autograd import ldlt_solve
    N, nrhs, pw = 256, 4, 64
    print("case: autograd finite differences", N, flush=True)
    A0, lam, B0 = dense_indefinite(N, seed=5, lam_lo=1e-2, nrhs=nrhs)
    rng = np.random.default_rng(1)
    W = rng.standard_normal(B0.shape)
    A = torch.tensor(A0, device="cuda", requires_grad=True)
    X = ldlt_solve(A, torch.tensor(B0, device="cuda"), pw=pw)
    (torch.tensor(W, device="cuda") * X).sum().backward()
    G = A.grad.cpu().numpy()
    opts = ctp.ctp_default_opts("relaxed")

    def loss(M):
        a = ctp.device_panel(M)
        a0 = ctp.device_panel(M)
        work = ctp.dense_workspace(N, pw, opts, nrhs)
        f = ctp.ctp_ldlt_dense(a, pw, opts, work)
        x, steps, hist = ctp.ctp_ldlt_refine(a0, a, f, ctp.device_panel(B0), opts, work, tol=0.0, max_steps=3)
        return float((W * x.cpu().numpy()).sum())

    h = 1e-3
    worst = 0.0
    for _ in range(32):
        Z = rng.standard_normal((N, N))
        E = (Z + Z.T) / 2
        E /= np.linalg.norm(E)
        d1 = loss(A0 + h * E) - loss(A0 - h * E)
        d2 = loss(A0 + 2 * h * E) - loss(A0 - 2 * h * E)
        fd = (8 * d1 - d2) / (12 * h)
        an = float((G * E).sum())
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    print(f"worst relative error of the directional derivatives: {worst:.2e}", flush=True)
    assert worst < 1e-8, worst
