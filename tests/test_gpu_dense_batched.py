"""Batches of dense systems on the GPU (ctp_ldlt_dense_batched, its batched
solve and adjoint): every system against the oracle and against the
single-system driver, whose bits it must reproduce (same decisions, same
per-tile arithmetic of the trailing updates)."""

import numpy as np
import pytest
import torch

from gpu_helpers import rel_err, require_gpu
from oracle.dense import backward_error, ldlt_dense, solve_adjoint
from workloads import dense_indefinite, supernode

pytestmark = pytest.mark.gpu



def _tol(A, ref, u=0.01):
    """D and L against the oracle: later pivots are Schur complement values
    after up to N/pw trailing updates summed in another order, so their
    error is bounded by about N (1/u) eps growth (max |l| <= 1/u), growth =
    max |factor entry| / max |A| of this draw (relative to max |entry|)."""
    growth = max(np.abs(ref.M).max() / np.abs(A).max(), 1.0)
    return A.shape[0] * (1.0 / u) * np.finfo(float).eps * growth


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _announce(*args):
    print("case:", *args, flush=True)


def _sym(N, seed, n_small=0, scale=1e-8):
    A = supernode(N, N, seed=seed, n_small=n_small, small_scale=scale)
    return np.tril(A) + np.tril(A, -1).T


def _batch(mats):
    from paper_1305_2353_amd import ctp
    return ctp.batch_colmajor(torch.tensor(np.stack(mats), device="cuda"))


def _single(A, pw, opts):
    from paper_1305_2353_amd import ctp
    a = ctp.device_panel(A)
    work = ctp.dense_workspace(A.shape[0], pw, opts, 4)
    f = ctp.ctp_ldlt_dense(a, pw, opts, work)
    return a, f


@pytest.mark.parametrize("method", ["relaxed", "strict", "restricted"])
@pytest.mark.parametrize("S,N,pw,n_small", [(3, 300, 64, 12), (3, 700, 256, 20), (2, 40, 64, 3), (1, 200, 32, 8)])
def test_batched_dense_matches_oracle_and_single_driver(method, S, N, pw, n_small):
    from paper_1305_2353_amd import ctp
    _announce("dense batched", method, S, N, pw)
    As = [_sym(N, seed=N + pw + 7 * s, n_small=n_small) for s in range(S)]
    opts = ctp.ctp_default_opts(method)
    refs, too_wide = [], []
    for s, A in enumerate(As):
        try:
            ref = ldlt_dense(A, pw, method)
        except ValueError:
            too_wide.append(s)          # delays grow a panel past 512 columns
            continue
        if ref.fragile:
            pytest.skip("near-tie decision in this draw")
        refs.append(ref)
    if too_wide:
        # (strict pivoting on the N = 700 draws: its delays pile up) both
        # drivers refuse with CTP_ERR_PANEL_TOO_WIDE where the oracle does
        work = ctp.dense_batched_workspace(S, N, pw, opts)
        with pytest.raises(ctp.CtpError, match=str(ctp.CTP_ERR_PANEL_TOO_WIDE)):
            ctp.ctp_ldlt_dense_batched(_batch(As), pw, opts, work)
        for s in too_wide:
            with pytest.raises(ctp.CtpError, match=str(ctp.CTP_ERR_PANEL_TOO_WIDE)):
                _single(As[s], pw, opts)
        torch.cuda.synchronize()
        return
    a = _batch(As)
    work = ctp.dense_batched_workspace(S, N, pw, opts)
    f = ctp.ctp_ldlt_dense_batched(a, pw, opts, work)
    torch.cuda.synchronize()
    assert f["nsteps"] == max(len(r.panels) for r in refs)
    for s, ref in enumerate(refs):
        # the single-system driver's bits (same decisions, same per-tile arithmetic)
        a1, f1 = _single(As[s], pw, opts)
        assert torch.equal(f1["perm"], f["perm"][s]), s
        assert torch.equal(f1["piv"], f["piv"][s]), s
        assert torch.equal(f1["d"], f["d"][s]), s
        assert torch.equal(a1, a[s]), s
        # the status words agree except for the rescan bit: it reports how
        # the relaxed compression found C (the batched one walks top-8 lists
        # and rescans; the single driver's panels of at most 16384 rows walk
        # exact lists and never do), not a property of the result
        keep = ~ctp.CTP_STATUS_RELAXED_RESCAN
        assert int(f1["status"].item()) & keep == int(f["status"][s].item()) & keep, s
        # the oracle: decisions exactly, values to the bound of this draw
        assert (f["perm"][s].cpu().numpy() == ref.perm).all(), s
        assert (f["piv"][s].cpu().numpy() == ref.piv).all(), s
        tol = _tol(As[s], ref)
        assert rel_err(f["d"][s].cpu().numpy(), ref.d) <= tol, s
        M = a[s].cpu().numpy()
        assert rel_err(np.tril(M), np.tril(ref.M)) <= tol, s


def test_batched_solve_and_adjoint():
    from paper_1305_2353_amd import ctp
    S, N, pw, nrhs = 4, 515, 128, 3
    _announce("dense batched solve/adjoint", S, N, pw)
    sys = [dense_indefinite(N, seed=40 + s, lam_lo=1e-2, nrhs=nrhs) for s in range(S)]
    As, Bs = [t[0] for t in sys], [t[2] for t in sys]
    opts = ctp.ctp_default_opts("relaxed")
    a = _batch(As)
    work = ctp.dense_batched_workspace(S, N, pw, opts)
    f = ctp.ctp_ldlt_dense_batched(a, pw, opts, work)
    x = ctp.ctp_ldlt_solve_batched(a, f, _batch(Bs), opts, work)
    rng = np.random.default_rng(3)
    Xb = [rng.standard_normal((N, nrhs)) for _ in range(S)]
    bbar, abar = ctp.ctp_ldlt_adjoint_batched(a, f, x, _batch(Xb), opts, work)
    torch.cuda.synchronize()
    for s in range(S):
        xs = x[s].cpu().numpy()
        ref = np.linalg.solve(As[s], Bs[s])
        assert np.abs(xs - ref).max() / np.abs(ref).max() < 1e-11, s
        assert backward_error(As[s], xs, Bs[s]) < max(1e-13, 10 * backward_error(As[s], ref, Bs[s])), s
        # the same factors and solve as one system at a time
        a1 = ctp.device_panel(As[s])
        w1 = ctp.dense_workspace(N, pw, opts, nrhs)
        f1 = ctp.ctp_ldlt_dense(a1, pw, opts, w1)
        x1 = ctp.ctp_ldlt_solve(a1, f1, ctp.device_panel(Bs[s]), opts, w1)
        assert torch.equal(x1, x[s]), s
        bref, aref = solve_adjoint(As[s], xs, Xb[s])
        assert rel_err(bbar[s].cpu().numpy(), bref) < 1e-8, s
        g = abar[s].cpu().numpy()
        assert rel_err(g, aref) < 1e-8, s
        assert np.array_equal(g, g.T), s


def test_batched_autograd_matches_single_system_path():
    from paper_1305_2353_amd.autograd import LDLTSolve, ldlt_solve
    S, N, nrhs, pw = 3, 256, 2, 64
    _announce("autograd batched vs single", S, N)
    sys = [dense_indefinite(N, seed=60 + s, lam_lo=1e-2, nrhs=nrhs) for s in range(S)]
    A = torch.tensor(np.stack([t[0] for t in sys]), device="cuda", requires_grad=True)
    B = torch.tensor(np.stack([t[2] for t in sys]), device="cuda", requires_grad=True)
    W = torch.tensor(np.random.default_rng(5).standard_normal((S, N, nrhs)), device="cuda")
    (W * ldlt_solve(A, B, pw=pw)).sum().backward()
    for s in range(S):
        As = A[s].detach().clone().requires_grad_(True)
        Bs = B[s].detach().clone().requires_grad_(True)
        (W[s] * LDLTSolve.apply(As, Bs, pw, "relaxed")).sum().backward()
        assert torch.equal(As.grad, A.grad[s]), s
        assert torch.equal(Bs.grad, B.grad[s]), s


def test_batched_solve_large_grid_matches_single_system_solves():
    """Enough systems that the workgroups of one sweep launch cannot all be
    resident at once: every system's solve must still be right (each sweep
    reads one vector and writes another, so no workgroup can see a block
    another has already overwritten)."""
    from paper_1305_2353_amd import ctp
    from workloads import dense_indefinite_batch_torch
    S, N, nrhs, pw = 256, 1024, 4, 256
    _announce("dense batched solve, large grid", S, N)
    A0, B0 = dense_indefinite_batch_torch(S, N, seed=11, lam_lo=1e-2, nrhs=nrhs)
    opts = ctp.ctp_default_opts("relaxed")
    a = ctp.batch_colmajor(A0)
    work = ctp.dense_batched_workspace(S, N, pw, opts)
    f = ctp.ctp_ldlt_dense_batched(a, pw, opts, work)
    x = ctp.ctp_ldlt_solve_batched(a, f, ctp.batch_colmajor(B0), opts, work)
    R = B0 - torch.bmm(A0, x)
    den = A0.abs().sum(dim=2).amax(dim=1)[:, None] * x.abs().amax(dim=1) + B0.abs().amax(dim=1)
    berr = (R.abs().amax(dim=1) / den).amax(dim=1)
    # backward stability of LDL^T: about N eps growth, growth = max |factor
    # entry| / max |A| of each system (the overwritten blocks this guards
    # against gave errors of 1e-2)
    growth = a.abs().amax(dim=(1, 2)) / A0.abs().amax(dim=(1, 2))
    bound = N * torch.finfo(torch.float64).eps * growth
    assert bool((berr <= bound).all()), int((berr / bound).argmax())
    for s in (0, S // 2, S - 1):
        a1 = ctp.device_panel(A0[s].cpu().numpy())
        w1 = ctp.dense_workspace(N, pw, opts, nrhs)
        f1 = ctp.ctp_ldlt_dense(a1, pw, opts, w1)
        x1 = ctp.ctp_ldlt_solve(a1, f1, ctp.device_panel(B0[s].cpu().numpy()), opts, w1)
        assert torch.equal(a1, a[s]), s
        assert torch.equal(x1, x[s]), s
