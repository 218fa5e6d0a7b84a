"""Factor, Solve and Form on one dense n x p supernode -- plain CPU oracle.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path; it shares no
code with the HIP library.

Section 1 of the paper defines the three tasks on the supernodal matrix
A = [A11; A21] (A11 p x p symmetric, A21 (n-p) x p):

    Factor  A11 = L11 D11 L11^T      (with a symmetric permutation P)
    Solve   L21 = A21 (D11 L11^T)^-1
    Form    S   = L21 D11 L21^T      (the Schur complement for the parent)

Columns that cannot be eliminated stably are delayed (Section 1).  The
pivots come from one of four rules:

    'tpp'         threshold partial pivoting on the whole panel (Section 2),
    'strict'      compressed pivoting with the strict C (Section 4.1),
    'relaxed'     compressed pivoting with the relaxed C (Section 4.2),
    'restricted'  pivots tested against A11 only (Section 3.2; C = 0).

For the compressed rules the pivot search runs on the 2p x p trapezoid
[A11; C] (Fig. 4.1 (b)-(c)); the permutation is then applied to the columns
of A21 and L21 is obtained by the triangular solve of Fig. 4.1 (d)-(e).

Output layout (identical to the HIP library's so that the tests compare the
two panel for panel; all in final pivot positions, 0-based):

    rows 0..p-1 (A11 part, lower triangle):
        column k < nelim: out[k,k] = D(k,k); out[k+1,k] = D(k+1,k) if k starts
        a 2x2 pivot; every other entry below the diagonal is L(i,k).
        columns k >= nelim: the delayed block after the eliminations.
    rows p..n-1 (A21 part):
        columns k < nelim: L21; columns k >= nelim: the updated A21 columns.
"""

from dataclasses import dataclass

import numpy as np

from .threshold import (PIV_1X1, PIV_2X2_FIRST, PIV_2X2_SECOND, PIV_ZERO,
                        R_ABS, R_NORMAL, ST_NONFINITE, factor_trapezoid)

METHODS = ("tpp", "strict", "relaxed", "restricted")


# ---------------------------------------------------------------------------
# Compressed matrices (Section 4)
# ---------------------------------------------------------------------------

def compress_strict(A21):
    """Strict compressed matrix C of eq. (4.2) (Section 4.1).

    Row i of A21 belongs to J_j when column j holds its largest |a(i,k)|,
    the lowest such column on ties (an all-zero row therefore belongs to the
    first set).  Row j of C is the columnwise maximum of |A21| over J_j, and
    zero when J_j is empty.
    """
    r, p = A21.shape
    absA = np.abs(A21)
    C = np.zeros((p, p), dtype=A21.dtype)
    if r == 0 or p == 0:
        return C
    J = np.argmax(absA, axis=1)          # first maximum = lowest column
    np.maximum.at(C, J, absA)
    return C


def compress_relaxed(A21):
    """Relaxed compressed matrix (Section 4.2).

    For columns j = 1..p in order: take the unflagged row of A21 with the
    largest |a(i,j)| (the first such row on ties), flag it and copy the row,
    with its signs, into row j of C.  When every row is already flagged
    (fewer than p rows) the remaining rows of C are zero.
    Returns (C, rows) with rows[j] the A21 row used for C row j, or -1.
    """
    r, p = A21.shape
    C = np.zeros((p, p), dtype=A21.dtype)
    rows = np.full(p, -1, dtype=np.int64)
    flagged = np.zeros(r, dtype=bool)
    for j in range(p):
        if flagged.all():
            break
        vals = np.abs(A21[:, j])
        if A21.dtype == object:
            best = -1
            for i in range(r):
                # strictly larger: the first row wins a tie
                if not flagged[i] and (best < 0 or vals[i] > vals[best]):
                    best = i
        else:
            # |a| >= 0 > -1, and argmax returns the first maximum
            best = int(np.argmax(np.where(flagged, -1.0, vals)))
        flagged[best] = True
        rows[j] = best
        C[j, :] = A21[best, :]
    return C, rows


# ---------------------------------------------------------------------------
# Factor + Solve (Sections 1, 2 and 4)
# ---------------------------------------------------------------------------

@dataclass
class SupernodeFactors:
    out: np.ndarray       # n x p output panel (layout in the module docstring)
    perm: np.ndarray      # perm[k] = original column at position k
    piv: np.ndarray       # pivot type per position
    d: np.ndarray         # 2p entries of D (see threshold.TrapezoidFactors)
    nelim: int
    W: np.ndarray         # (n-p) x nelim, W = L21 D (rows of A21 times (L11^T)^-1)
    C: np.ndarray         # the compressed matrix used (None for TPP / restricted)
    crow: np.ndarray      # relaxed: A21 row behind each C row (else None)
    log: list             # decision log of the pivot search
    trap: object          # the TrapezoidFactors of the pivot search
    status: int = 0       # OR of the threshold.ST_* bits (see factor_supernode)


def d_blocks(piv, d, nelim):
    """Block diagonal D over the first nelim positions as a dense matrix."""
    D = np.zeros((nelim, nelim), dtype=d.dtype)
    k = 0
    while k < nelim:
        if piv[k] == PIV_2X2_FIRST:
            D[k, k], D[k + 1, k], D[k, k + 1], D[k + 1, k + 1] = (
                d[2 * k], d[2 * k + 1], d[2 * k + 1], d[2 * k + 2])
            k += 2
        else:
            D[k, k] = d[2 * k]
            k += 1
    return D


def unit_lower_L11(out, piv, nelim):
    """Unit lower triangular L over the first p rows / nelim columns of the
    output panel: the stored D entries (diagonal, 2x2 sub-diagonal) are
    replaced by 1 and 0."""
    p = out.shape[1]
    L = np.tril(out[:p, :nelim], -1).copy()
    for k in range(nelim):
        if piv[k] == PIV_2X2_FIRST:
            L[k + 1, k] = 0
    L[np.arange(nelim), np.arange(nelim)] = 1
    return L


def solve_a21(A21P, L, piv, d, nelim):
    """Solve task on the column-permuted A21 (Fig. 4.1 (d)-(e)).

    A21P: (n-p) x p, columns already in final pivot order.  L: p x nelim
    unit lower factor (rows of A11 in pivot order, L_EE on top of L_dE).
    Returns (L21, W, A21d) with W = A21P[:, E] (L_EE^T)^-1 = L21 D,
    L21 = W D^-1 and A21d = A21P[:, d] - W L_dE^T.  Zero pivots give zero
    columns of W and L21 (the column is dropped).
    """
    import scipy.linalg as sla
    r, p = A21P.shape
    AE = A21P[:, :nelim]
    exact = A21P.dtype == object
    if exact:
        # plain forward substitution W[:, k] = A[:, k] - sum_j<k W[:, j] L[k, j]
        W = AE.copy()
        for k in range(nelim):
            for j in range(k):
                W[:, k] = W[:, k] - W[:, j] * L[k, j]
    elif nelim:
        W = sla.solve_triangular(L[:nelim, :nelim], AE.T, lower=True, check_finite=False,
                                 unit_diagonal=True).T
    else:
        W = np.zeros((r, 0), dtype=A21P.dtype)
    zero_cols = [k for k in range(nelim) if piv[k] == PIV_ZERO]
    W[:, zero_cols] = 0
    L21 = np.zeros_like(W)
    k = 0
    while k < nelim:
        if piv[k] == PIV_2X2_FIRST:
            a11, a21, a22 = d[2 * k], d[2 * k + 1], d[2 * k + 2]
            if exact:
                det = a11 * a22 - a21 * a21
                L21[:, k] = (W[:, k] * a22 - W[:, k + 1] * a21) / det
                L21[:, k + 1] = (W[:, k + 1] * a11 - W[:, k] * a21) / det
            else:
                D = np.array([[a11, a21], [a21, a22]])
                L21[:, k:k + 2] = np.linalg.solve(D, W[:, k:k + 2].T).T
            k += 2
        elif piv[k] == PIV_ZERO:
            k += 1
        else:
            L21[:, k] = W[:, k] / d[2 * k]
            k += 1
    A21d = A21P[:, nelim:] - W @ L[nelim:, :nelim].T
    return L21, W, A21d


def factor_supernode(A, p, method="relaxed", u=0.01, small=1e-20, forced=None, root=False):
    """Factor + Solve of the n x p supernode A = [A11; A21] (Section 1).

    A: n x p array; the lower triangle of its first p rows is A11.
    root: eliminate every column (last panel of a factorization; see
    factor_trapezoid).
    status: the pivot search's bits (zero pivot, root fallback, a NaN or an
    infinity read by a pivot test), plus ST_NONFINITE when a compressed rule
    reads a non-finite A21 entry while building C (compression reads all of
    A21; restricted pivoting never reads A21, TPP reads it through its
    tests).
    """
    if method not in METHODS:
        raise ValueError(method)
    n = A.shape[0]
    A11 = A[:p, :p]
    A21 = A[p:, :p]
    C = crow = None
    if method == "tpp":
        trap = factor_trapezoid(A11, A21, u, small, R_NORMAL, forced, root)
    elif method == "strict":
        C = compress_strict(A21)
        trap = factor_trapezoid(A11, C, u, small, R_ABS, forced, root)
    elif method == "relaxed":
        C, crow = compress_relaxed(A21)
        trap = factor_trapezoid(A11, C, u, small, R_NORMAL, forced, root)
    else:
        trap = factor_trapezoid(A11, A21[:0], u, small, R_NORMAL, forced, root)

    perm, piv, d, nelim = trap.perm, trap.piv, trap.d, trap.nelim
    out = np.zeros_like(A)
    out[:p, :p] = np.tril(trap.T)
    L = unit_lower_L11(out, piv, nelim)
    if method == "tpp":
        # Listing 1 updated every row of A21 itself: its eliminated columns
        # are L21 and the others are the updated delayed columns.
        out[p:, :] = trap.R
        W = trap.R[:, :nelim] @ d_blocks(piv, d, nelim) if nelim else trap.R[:, :0]
    else:
        A21P = A21[:, perm]
        L21, W, A21d = solve_a21(A21P, L, piv, d, nelim)
        out[p:, :nelim] = L21
        out[p:, nelim:] = A21d
    status = trap.status
    if method in ("strict", "relaxed") and A21.dtype != object and not np.isfinite(A21).all():
        status |= ST_NONFINITE
    return SupernodeFactors(out, perm, piv, d, nelim, W, C, crow, trap.log, trap, status)


# ---------------------------------------------------------------------------
# Form (Section 1)
# ---------------------------------------------------------------------------

def schur_rows(F, rows):
    """Rows of the lower triangle of S = L21 D11 L21^T (Section 1, Form).

    rows: increasing indices into A21's rows.  Returns a len(rows) x
    (rows[-1]+1) array whose entry (a, j) is S(rows[a], j) for
    j <= rows[a] and 0 above the diagonal.
    """
    p = F.out.shape[1]
    L21 = F.out[p:, :F.nelim]
    D = d_blocks(F.piv, F.d, F.nelim)
    rows = np.asarray(rows)
    ncol = int(rows[-1]) + 1 if rows.size else 0
    block = (L21[rows] @ D) @ L21[:ncol].T
    for a, i in enumerate(rows):
        block[a, i + 1:] = 0
    return block


def schur_block(F, row0, nrows):
    """Rows row0..row0+nrows-1 of the lower triangle of S."""
    return schur_rows(F, np.arange(row0, row0 + nrows))


# ---------------------------------------------------------------------------
# Closed forms given the decisions (used by the checks)
# ---------------------------------------------------------------------------

def closed_forms(A, p, perm, piv, nelim):
    """Factors implied by a permutation and pivot blocks, from the original
    data alone (no pivot search): with B = P A11 P^T and G = A21 P^T split
    into eliminated (E) and delayed (d) columns,

        L_EE D L_EE^T = B_EE,  L_dE = B_dE (D L_EE^T)^-1,
        B_dd' = B_dd - B_dE B_EE^-1 B_Ed,
        L21 = G_E (D L_EE^T)^-1,  G_d' = G_d - G_E B_EE^-1 B_Ed,
        S = G_E B_EE^-1 G_E^T.

    Valid when there are no zero pivots.  Returns a dict of those blocks.
    """
    A11 = np.tril(A[:p, :p]) + np.tril(A[:p, :p], -1).T
    B = A11[np.ix_(perm, perm)]
    G = A[p:, :p][:, perm]
    E = np.arange(nelim)
    dl = np.arange(nelim, p)
    BEE = B[np.ix_(E, E)]
    BdE = B[np.ix_(dl, E)]
    Bdd = B[np.ix_(dl, dl)]
    GE = G[:, E]
    Gd = G[:, dl]
    inv_BEE_BEd = np.linalg.solve(BEE, BdE.T) if nelim else np.zeros((0, len(dl)))
    return {
        "BEE": BEE,
        "Bdd_prime": Bdd - BdE @ inv_BEE_BEd,
        "Gd_prime": Gd - GE @ inv_BEE_BEd,
        "S": GE @ np.linalg.solve(BEE, GE.T) if nelim else np.zeros((G.shape[0],) * 2),
        "B": B,
        "G": G,
    }
