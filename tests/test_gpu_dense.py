"""Dense LDL^T by supernode panels on the GPU (FP64 and the reduced-precision
trailing updates), its solve and FP64 refinement, against the oracle of
oracle/dense.py and against the backward-error target."""

import numpy as np
import pytest
import torch

from gpu_helpers import FP64_TOL, rel_err, require_gpu
from oracle.dense import backward_error, ldlt_dense, ldlt_solve
from oracle.threshold import factor_trapezoid
from workloads import dense_indefinite, supernode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _announce(*args):
    print("case:", *args, flush=True)


def _sym(N, seed, n_small=0, scale=1e-8):
    A = supernode(N, N, seed=seed, n_small=n_small, small_scale=scale)
    return np.tril(A) + np.tril(A, -1).T


def _gpu_dense(A, pw, method, prec="fp64", nrhs=4):
    from paper_1305_2353_amd import ctp
    N = A.shape[0]
    opts = ctp.ctp_default_opts(method, prec=prec)
    a = ctp.device_panel(A)
    work = ctp.dense_workspace(N, pw, opts, nrhs)
    f = ctp.ctp_ldlt_dense(a, pw, opts, work)
    torch.cuda.synchronize()
    return a, f, opts, work




@pytest.mark.parametrize("method", ["relaxed", "strict", "tpp", "restricted"])
@pytest.mark.parametrize("N,pw,n_small", [(96, 16, 6), (300, 64, 12), (700, 256, 20)])
def test_dense_fp64_matches_oracle(method, N, pw, n_small):
    A = _sym(N, seed=N + pw, n_small=n_small)
    _announce("dense fp64", method, N, pw)
    ref = ldlt_dense(A, pw, method)
    if ref.fragile:
        pytest.skip("near-tie decision in this draw")
    a, f, opts, work = _gpu_dense(A, pw, method)
    assert f["npanels"] == len(ref.panels)
    assert (f["perm"].cpu().numpy() == ref.perm).all()
    assert (f["piv"].cpu().numpy() == ref.piv).all()
    assert rel_err(f["d"].cpu().numpy(), ref.d) <= FP64_TOL
    M = a.cpu().numpy()
    assert rel_err(np.tril(M), np.tril(ref.M)) <= FP64_TOL
    # the strict upper triangle holds L^T for the solve
    L = np.tril(M, -1)
    for k in np.nonzero(ref.piv == 2)[0]:
        L[k + 1, k] = 0.0
    assert np.array_equal(np.triu(M, 1), L.T)


@pytest.mark.parametrize("N,pw", [(200, 32), (515, 128), (1024, 256)])
def test_dense_solve_and_fp64_refinement(N, pw):
    from paper_1305_2353_amd import ctp
    A, lam, B = dense_indefinite(N, seed=N, lam_lo=1e-2, nrhs=3)
    _announce("dense solve", N, pw)
    a, f, opts, work = _gpu_dense(A, pw, "relaxed")
    b = ctp.device_panel(B)
    x = ctp.ctp_ldlt_solve(a, f, b.clone(), opts, work).cpu().numpy()
    ref = np.linalg.solve(A, B)
    assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-11
    assert backward_error(A, x, B) < 1e-14
    a0 = ctp.device_panel(A)
    X, steps, hist = ctp.ctp_ldlt_refine(a0, a, f, b, opts, work, tol=1e-15, max_steps=3)
    assert backward_error(A, X.cpu().numpy(), B) == pytest.approx(hist[-1], rel=1e-6)
    assert hist[-1] < 1e-15 or steps == 3


def test_dense_solve_with_two_by_two_pivots_across_blocks():
    """Indefinite input with tiny diagonals: many 2x2 pivots, some of which
    straddle the 128-column blocks of the solve."""
    from paper_1305_2353_amd import ctp
    N, pw = 520, 64
    A = _sym(N, seed=3, n_small=N, scale=1e-6)
    _announce("dense 2x2 straddle", N, pw)
    a, f, opts, work = _gpu_dense(A, pw, "relaxed")
    piv = f["piv"].cpu().numpy()
    assert (piv == 2).sum() > 50
    rng = np.random.default_rng(1)
    B = rng.standard_normal((N, 2))
    x = ctp.ctp_ldlt_solve(a, f, ctp.device_panel(B), opts, work).cpu().numpy()
    assert backward_error(A, x, B) < 1e-13


@pytest.mark.parametrize("prec,lam_lo,fact_tol,max_steps", [("fp32", 1e-2, 1e-5, 10), ("bf16", 0.3, 5e-2, 30)])
def test_dense_reduced_precision_refines_to_target(prec, lam_lo, fact_tol, max_steps):
    """Trailing updates on the FP32 / BF16 matrix cores: the factors
    reconstruct A to the precision of the update, and FP64 refinement
    reaches a backward error of 1e-14."""
    from paper_1305_2353_amd import ctp
    N, pw = 768, 128
    A, lam, B = dense_indefinite(N, seed=11, lam_lo=lam_lo, nrhs=4)
    _announce("dense reduced precision", prec, N, pw)
    a, f, opts, work = _gpu_dense(A, pw, "relaxed", prec=prec)
    M = a.cpu().numpy()
    piv = f["piv"].cpu().numpy()
    d = f["d"].cpu().numpy()
    perm = f["perm"].cpu().numpy()
    from oracle.supernode import d_blocks, unit_lower_L11
    L = unit_lower_L11(np.tril(M), piv, N)
    err = np.abs(A[np.ix_(perm, perm)] - L @ d_blocks(piv, d, N) @ L.T).max() / np.abs(A).max()
    assert err < fact_tol
    b = ctp.device_panel(B)
    X, steps, hist = ctp.ctp_ldlt_refine(ctp.device_panel(A), a, f, b, opts, work, tol=1e-14,
                                         max_steps=max_steps)
    assert hist[-1] <= 1e-14, hist
    assert backward_error(A, X.cpu().numpy(), B) <= 2e-14


def test_root_flag_matches_oracle_fallback():
    """CTP_FLAG_ROOT on a trapezoid where every threshold test fails."""
    from paper_1305_2353_amd import ctp
    p = 6
    rng = np.random.default_rng(9)
    G = 1e-3 * rng.standard_normal((p, p))
    A11 = np.tril(G) + np.tril(G, -1).T + 1e-3 * np.eye(p)
    R = 10.0 * rng.standard_normal((3 * p, p))
    ref = factor_trapezoid(np.tril(A11), R, u=0.1, root=True)
    a = ctp.device_panel(np.vstack([A11, R]))
    opts = ctp.ctp_default_opts("tpp", u=0.1, flags=ctp.CTP_FLAG_ROOT)
    f = ctp.ctp_factor_supernode(a, opts)
    torch.cuda.synchronize()
    assert int(f["nelim"].item()) == p
    assert int(f["status"].item()) & ctp.CTP_STATUS_ROOT_FALLBACK
    assert (f["perm"].cpu().numpy() == ref.perm).all()
    assert (f["piv"].cpu().numpy() == ref.piv).all()
    assert (f["d"].cpu().numpy() == ref.d).all()
    out = a.cpu().numpy()
    assert (np.tril(out[:p]) == np.tril(ref.T)).all()
    assert (out[p:] == ref.R).all()
    # without the flag nothing is eliminated
    a2 = ctp.device_panel(np.vstack([A11, R]))
    f2 = ctp.ctp_factor_supernode(a2, ctp.ctp_default_opts("tpp", u=0.1))
    torch.cuda.synchronize()
    assert int(f2["nelim"].item()) == 0
