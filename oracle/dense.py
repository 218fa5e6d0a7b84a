"""Oracle: dense symmetric indefinite LDL^T built from supernode panels, the
solve with its factors, the backward error and FP64 iterative refinement.

Test infrastructure only (see the package header).

The paper's setting (Section 1) is a multifrontal code in which each
supernode is factorized, its failed pivots are delayed to the parent and
every pivot is eliminated in the final (root) supernode.  A dense matrix
factorized right-looking in panels of pw columns is the chain of such
supernodes with one child each:

* panel q holds the delayed columns of panel q-1 followed by the next pw
  columns of the trailing matrix, so its width is pw + (delays carried);
* each panel is one Factor + Solve of the supernode formed by those
  columns and every row below them (factor_supernode, the rule given by
  `method`), and the trailing matrix receives the Form output
  S = L21 D L21^T (subtracted);
* the panel's symmetric interchanges also reorder the rows of the L
  columns already computed (the usual bookkeeping of a right-looking
  factorization with pivoting), and they are composed into one global
  permutation;
* the last panel, which has no rows below it, eliminates every column
  (factor_trapezoid's root fallback).

Results: P A P^T = L D L^T with (P A P^T)(i, j) = A(perm[i], perm[j]), L
unit lower triangular, D block diagonal with 1x1 and 2x2 blocks (piv, d in
the supernode convention).

The backward error of a computed x for A x = b, taken column by column and
maximised over the right-hand sides, is
    ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
(Section 7's measure of accuracy, with infinity norms).  Refinement
repeats x <- x + solve(b - A x) with the residual in FP64 until it is at or
below the target or a step limit is reached.
"""

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from .supernode import d_blocks, factor_supernode, unit_lower_L11
from .threshold import PIV_2X2_FIRST

MAX_PANEL = 512


@dataclass
class DenseFactors:
    M: np.ndarray        # N x N: L below the diagonal, D on the diagonal / 2x2 sub-diagonal
    perm: np.ndarray     # global permutation
    piv: np.ndarray      # pivot types by position
    d: np.ndarray        # 2N entries of D
    panels: list = field(default_factory=list)   # (k0, width, nelim) per panel
    fallback: int = 0    # number of root fallback eliminations
    fragile: int = 0     # decisions within rounding of their threshold (all panels)

    @property
    def N(self):
        return self.M.shape[0]

    def L(self):
        return unit_lower_L11(self.M, self.piv, self.N)

    def D(self):
        return d_blocks(self.piv, self.d, self.N)


def ldlt_dense(A, pw, method="relaxed", u=0.01, small=1e-20):
    """Right-looking LDL^T of the symmetric N x N matrix A (lower triangle
    read) in panels of pw columns, delays carried into the next panel."""
    A = np.asarray(A, dtype=float)
    N = A.shape[0]
    M = np.tril(A).copy()
    perm = np.arange(N)
    piv = np.zeros(N, dtype=np.int64)
    d = np.zeros(2 * N)
    panels = []
    fallback = 0
    fragile = 0
    k0 = 0
    width = min(pw, N)
    while k0 < N:
        if width > MAX_PANEL:
            raise ValueError(f"panel of width {width} exceeds {MAX_PANEL} (too many delays)")
        n = N - k0
        root = n == width
        # The supernode: columns k0..k0+width-1, rows k0..N-1 (lower part).
        panel = M[k0:, k0:k0 + width].copy()
        F = factor_supernode(panel, width, method, u, small, root=root)
        ne = F.nelim
        fallback += sum(1 for dec in F.log if dec.kind == "fallback")
        fragile += len(F.trap.fragile_steps())
        panels.append((k0, width, ne))
        # symmetric interchanges inside the panel: earlier L rows and the
        # global permutation follow
        M[k0:k0 + width, :k0] = M[k0 + F.perm, :k0]
        perm[k0:k0 + width] = perm[k0 + F.perm]
        M[k0:, k0:k0 + width] = F.out
        M[k0:k0 + width, k0:k0 + width] = np.tril(F.out[:width])
        piv[k0:k0 + ne] = F.piv[:ne]
        d[2 * k0:2 * (k0 + ne)] = F.d[:2 * ne]
        # trailing matrix: A22 - L21 D L21^T (Form, subtracted)
        if n > width and ne:
            L21 = F.out[width:, :ne]
            S = (L21 @ d_blocks(F.piv, F.d, ne)) @ L21.T
            M[k0 + width:, k0 + width:] -= np.tril(S)
        k0 += ne
        width = min(N - k0, (width - ne) + pw)
        if ne == 0 and not root:
            # nothing eliminated: the next panel grows by pw columns
            continue
    return DenseFactors(M, perm, piv, d, panels, fallback, fragile)


def reconstruct(F):
    """L D L^T (equals P A P^T up to rounding)."""
    L = F.L()
    return L @ F.D() @ L.T


def ldlt_solve(F, B):
    """x = P^T L^-T D^-1 L^-1 P b for every column of B."""
    B = np.asarray(B, dtype=float)
    one = B.ndim == 1
    Bm = B.reshape(B.shape[0], -1)
    L = F.L()
    y = Bm[F.perm]
    y = solve_triangular(L, y, lower=True, unit_diagonal=True)
    y = solve_d(F.piv, F.d, y)
    y = solve_triangular(L.T, y, lower=False, unit_diagonal=True)
    x = np.empty_like(y)
    x[F.perm] = y
    return x[:, 0] if one else x


def solve_d(piv, d, y):
    """D^-1 y with the 1x1 / 2x2 blocks of D (each 2x2 solved directly)."""
    N = len(piv)
    z = np.array(y, dtype=float)
    k = 0
    while k < N:
        if piv[k] == PIV_2X2_FIRST:
            D2 = np.array([[d[2 * k], d[2 * k + 1]], [d[2 * k + 1], d[2 * k + 2]]])
            z[k:k + 2] = np.linalg.solve(D2, z[k:k + 2])
            k += 2
        else:
            z[k] = z[k] / d[2 * k] if d[2 * k] != 0 else 0.0
            k += 1
    return z


def backward_error(A, X, B):
    """max over columns of ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    A = np.asarray(A, dtype=float)
    X = np.asarray(X, dtype=float).reshape(A.shape[0], -1)
    B = np.asarray(B, dtype=float).reshape(A.shape[0], -1)
    R = B - A @ X
    anorm = np.abs(A).sum(axis=1).max()
    num = np.abs(R).max(axis=0)
    den = anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    return float((num / den).max())


def refine(A, B, solve, tol=1e-14, max_steps=10):
    """FP64 iterative refinement: x = solve(b); x += solve(b - A x) until
    the backward error is <= tol or max_steps corrections were applied.
    Returns (x, steps, history of backward errors)."""
    X = solve(B)
    hist = [backward_error(A, X, B)]
    steps = 0
    while hist[-1] > tol and steps < max_steps:
        R = B - A @ X
        X = X + solve(R)
        steps += 1
        hist.append(backward_error(A, X, B))
    return X, steps, hist


def solve_adjoint(A, X, Xbar):
    """Adjoint of X = A^-1 B for symmetric A with the pivots frozen (not in
    the paper): Bbar = A^-1 Xbar and Abar = -sum_c (bbar_c x_c^T +
    x_c bbar_c^T) / 2, the gradient for symmetric perturbations of A."""
    A = np.asarray(A, dtype=float)
    X = np.asarray(X, dtype=float).reshape(A.shape[0], -1)
    Xbar = np.asarray(Xbar, dtype=float).reshape(A.shape[0], -1)
    Bbar = np.linalg.solve(A, Xbar)
    Abar = -0.5 * (Bbar @ X.T + X @ Bbar.T)
    return Bbar, Abar
