"""Pins for the dense panel driver, the solve and iterative refinement of the
oracle (oracle/dense.py), against facts that do not depend on it:
brute-force reconstruction, Sylvester's law of inertia, library solves,
hand-built delay and fallback cases."""

import numpy as np
import pytest

from oracle.dense import (backward_error, ldlt_dense, ldlt_solve, reconstruct, refine,
                          solve_adjoint, solve_d)
from oracle.threshold import factor_trapezoid
from workloads import dense_indefinite, supernode


def _sym(N, seed, n_small=0, scale=1e-8):
    A = supernode(N, N, seed=seed, n_small=n_small, small_scale=scale)
    return np.tril(A) + np.tril(A, -1).T


def _inertia_D(F):
    ev = np.linalg.eigvalsh(F.D())
    return int((ev < 0).sum()), int((ev == 0).sum()), int((ev > 0).sum())


@pytest.mark.parametrize("method", ["relaxed", "strict", "tpp", "restricted"])
@pytest.mark.parametrize("N,pw,n_small", [(96, 16, 6), (200, 32, 10), (130, 40, 0)])
def test_dense_reconstruction_and_inertia(method, N, pw, n_small):
    A = _sym(N, seed=N + pw, n_small=n_small)
    F = ldlt_dense(A, pw, method)
    assert sum(ne for _, _, ne in F.panels) == N
    PAP = A[np.ix_(F.perm, F.perm)]
    err = np.abs(PAP - reconstruct(F)).max() / np.abs(A).max()
    assert err < 1e-12
    ev = np.linalg.eigvalsh(A)
    neg, zero, pos = _inertia_D(F)
    assert (neg, pos) == (int((ev < 0).sum()), int((ev > 0).sum()))


def test_single_panel_is_the_root_supernode():
    A = _sym(48, seed=3, n_small=5)
    F = ldlt_dense(A, 64, "relaxed")
    T = factor_trapezoid(np.tril(A), A[:0], root=True)
    assert F.panels == [(0, 48, 48)]
    assert (F.perm == T.perm).all() and (F.piv == T.piv).all()
    assert np.array_equal(F.d, T.d)


def test_delay_is_carried_into_the_next_panel():
    """Column 0 has a tiny diagonal and couples only to column 8, which lies
    in the next panel of width 8: panel 1 must delay it, and panel 2 (width
    8 + 1) pairs it with its partner."""
    N, pw = 24, 8
    rng = np.random.default_rng(5)
    A = np.diag(rng.uniform(2.0, 3.0, N))
    for i in range(1, N):
        for j in range(1, i):
            A[i, j] = A[j, i] = 0.1 * rng.standard_normal()
    A[0, 0] = 1e-12
    A[8, 0] = A[0, 8] = 1.0
    F = ldlt_dense(A, pw, "relaxed")
    k0, w0, ne0 = F.panels[0]
    assert (k0, w0) == (0, 8) and ne0 == 7
    assert F.panels[1][1] == pw + 1
    assert F.perm[:7].tolist() == list(range(1, 8))
    PAP = A[np.ix_(F.perm, F.perm)]
    assert np.abs(PAP - reconstruct(F)).max() < 1e-12


def test_solve_matches_library_solve():
    A, lam, B = dense_indefinite(160, seed=2, nrhs=3)
    F = ldlt_dense(A, 32, "relaxed")
    X = ldlt_solve(F, B)
    ref = np.linalg.solve(A, B)
    assert np.abs(X - ref).max() / np.abs(ref).max() < 1e-11
    # a stable direct solve: backward error at the level of LAPACK's LU solve
    assert backward_error(A, X, B) < max(1e-14, 10 * backward_error(A, ref, B))


def test_solve_d_blocks():
    piv = np.array([2, -2, 1])
    d = np.array([1.0, 2.0, -3.0, 0.0, 4.0, 0.0])
    y = np.array([[1.0], [1.0], [8.0]])
    z = solve_d(piv, d, y)
    D = np.array([[1.0, 2.0, 0.0], [2.0, -3.0, 0.0], [0.0, 0.0, 4.0]])
    assert np.allclose(D @ z, y, rtol=0, atol=1e-15)


def test_backward_error_definition():
    A = np.array([[2.0, 1.0], [1.0, -1.0]])
    x = np.array([[1.0], [1.0]])
    b = A @ x + np.array([[1e-3], [0.0]])
    # ||r|| = 1e-3, ||A||_inf = 3, ||x|| = 1, ||b|| = 3.001
    assert backward_error(A, x, b) == pytest.approx(1e-3 / (3.0 + 3.001), rel=1e-12)


def test_refinement_reaches_the_target_from_a_float32_factorization():
    """Factors of A rounded to float32 give a solve accurate to about
    kappa * 6e-8; refinement with FP64 residuals drives the backward error
    below 1e-14."""
    A, lam, B = dense_indefinite(200, seed=4, lam_lo=1e-2, nrhs=2)
    F32 = ldlt_dense(A.astype(np.float32).astype(np.float64), 40, "relaxed")
    x0 = ldlt_solve(F32, B)
    assert backward_error(A, x0, B) > 1e-12
    X, steps, hist = refine(A, B, lambda R: ldlt_solve(F32, R), tol=1e-14, max_steps=10)
    assert hist[-1] <= 1e-14
    assert 1 <= steps <= 6
    assert all(b < a for a, b in zip(hist, hist[1:]))


def test_root_fallback_eliminates_every_column():
    """A11 much smaller than R: every threshold test fails, so without the
    root option nothing is eliminated, and with it every column is, with
    A11 = L D L^T still exact."""
    p = 6
    rng = np.random.default_rng(9)
    G = 1e-3 * rng.standard_normal((p, p))
    A11 = np.tril(G) + np.tril(G, -1).T + 1e-3 * np.eye(p)
    R = 10.0 * rng.standard_normal((3 * p, p))
    T0 = factor_trapezoid(np.tril(A11), R, u=0.1)
    assert T0.nelim == 0
    T1 = factor_trapezoid(np.tril(A11), R, u=0.1, root=True)
    assert T1.nelim == p
    assert any(d.kind == "fallback" for d in T1.log)
    from oracle.supernode import d_blocks, unit_lower_L11
    out = np.tril(T1.T)
    L = unit_lower_L11(out, T1.piv, p)
    P = A11[np.ix_(T1.perm, T1.perm)]
    assert np.abs(L @ d_blocks(T1.piv, T1.d, p) @ L.T - P).max() < 1e-14


def test_panel_widths_without_delays():
    """With no delays every panel has pw columns and the last takes the rest."""
    A = np.zeros((600, 600))
    A[np.arange(600), np.arange(600)] = 1.0
    F = ldlt_dense(A, 256, "relaxed")
    assert [w for _, w, _ in F.panels] == [256, 256, 88]


def test_adjoint_matches_central_differences():
    """<Abar, E> against central differences of L(A) = sum w * A^-1 b along
    symmetric directions E, and Bbar against differences in b."""
    A, lam, B = dense_indefinite(24, seed=8, lam_lo=0.1, nrhs=2)
    rng = np.random.default_rng(3)
    W = rng.standard_normal(B.shape)
    loss = lambda M, R: float((W * np.linalg.solve(M, R)).sum())
    X = np.linalg.solve(A, B)
    Bbar, Abar = solve_adjoint(A, X, W)
    assert np.allclose(Abar, Abar.T, rtol=0, atol=1e-15)
    h = 1e-6
    for _ in range(4):
        Z = rng.standard_normal(A.shape)
        E = (Z + Z.T) / 2
        E /= np.linalg.norm(E)
        fd = (loss(A + h * E, B) - loss(A - h * E, B)) / (2 * h)
        assert fd == pytest.approx(float((Abar * E).sum()), rel=1e-6, abs=1e-8)
        Eb = rng.standard_normal(B.shape)
        fdb = (loss(A, B + h * Eb) - loss(A, B - h * Eb)) / (2 * h)
        assert fdb == pytest.approx(float((Bbar * Eb).sum()), rel=1e-6, abs=1e-8)
