"""Zero pivots, the root fallback and non-finite input in the oracle, on
small panels worked by hand in exact rational arithmetic.

Section 2's algorithm records a zero pivot when every entry of the candidate
column is below `small`: D = 0, a zero column of L, and no update of the
trailing matrix.  The expectations below were derived by hand from that rule,
the tests (2.1) / (2.2) and the updates of Section 2 (working in the
comments); none of them is computed by the oracle.  Each case is checked for
the values a plausible slip would change: a dropped zeroing of the R column
leaves a tiny entry in L21, an update after a zero pivot divides by D = 0
(an exception in exact arithmetic), a wrong interchange moves perm.
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.supernode import factor_supernode, unit_lower_L11, d_blocks
from oracle.threshold import (PIV_1X1, PIV_2X2_FIRST, PIV_2X2_SECOND, PIV_ZERO, R_NORMAL,
                              ST_NONFINITE, ST_ROOT_FALLBACK, ST_ZERO_PIVOT, factor_trapezoid)

U = Fr(1, 100)
SMALL = Fr(1, 10**20)
EPS = Fr(1, 10**30)          # below SMALL: counts as zero
METHODS = ["tpp", "strict", "relaxed", "restricted"]


def _fr(rows):
    return np.array([[Fr(x) for x in r] for r in rows], dtype=object)


def _tiny_column_panel():
    # A11 (lower triangle)       A21
    #   [ 2          ]           [  1  e  2 ]
    #   [ e  e       ]           [ -1  e  1 ]
    #   [ 1  e  3    ]
    # Column 1 (0-based) holds only e = 1e-30 < small, A21 part included.
    e = EPS
    return _fr([[2, 0, 0], [e, e, 0], [1, e, 3], [1, e, 2], [-1, e, 1]])


@pytest.mark.parametrize("method", METHODS)
def test_column_below_small_is_a_zero_pivot(method):
    # m = 1 first: |a11| = e and every other entry of the column (a10, a21
    # and the R column) is e or 0 -> zero pivot.  Interchange 1 <-> 0:
    # perm = [1, 0, 2]; D(0) = 0; L column 0 and the R column are zeroed;
    # the trailing 2 x 2 block [[2, 1], [1, 3]] is untouched.
    # m = 2, t = 1 (the only pending column): a_tt = 2, a_tm = 1, a_mm = 3,
    #  s = 1/3, det1 = 1/3, det0 = 2, det = 5/3 > max(small, 1, 1/6);
    #  R columns after the zeroing: TPP (1, -1) and (2, 1) -> maxt = 1,
    #  maxm = 2 (strict C rows (1,e,1), 0, (1,e,2) and relaxed C rows
    #  (1,e,2), (-1,e,1), 0 give the same maxima; restricted has no R and
    #  passes through max(maxt, maxm) < small);
    #  f = (1/3)/(5/3) = 1/5, |D^-1| (maxt, maxm) = (3/5 + 2/5, 1/5 + 4/5)
    #  = (1, 1) <= 100 -> 2x2 pivot on positions 1, 2.
    A = _tiny_column_panel()
    F = factor_supernode(A, 3, method, u=U, small=SMALL)
    assert [d.kind for d in F.log] == ["zero", "2x2"]
    assert list(F.perm) == [1, 0, 2]
    assert list(F.piv) == [PIV_ZERO, PIV_2X2_FIRST, PIV_2X2_SECOND]
    assert list(F.d) == [0, 0, 2, 1, 3, 0]
    assert F.nelim == 3
    assert F.status == ST_ZERO_PIVOT
    # zero L column (A11 rows and A21 rows)
    assert F.out[1, 0] == 0 and F.out[2, 0] == 0
    assert (F.out[3:, 0] == 0).all()
    # L21 of the 2x2 pivot: D^-1 = (1/5)[[3, -1], [-1, 2]] applied to the
    # A21 rows (1, 2) and (-1, 1)
    assert list(F.out[3, 1:]) == [Fr(1, 5), Fr(3, 5)]
    assert list(F.out[4, 1:]) == [Fr(-4, 5), Fr(3, 5)]
    # reconstruction of the non-zero part: positions 1, 2 of P A11 P^T and
    # A21 P^T equal L D L^T and L21 D L^T there
    A11 = np.tril(A[:3]) + np.tril(A[:3], -1).T
    B = A11[np.ix_(F.perm, F.perm)]
    L = unit_lower_L11(F.out, F.piv, 3)
    D = d_blocks(F.piv, F.d, 3)
    assert ((L @ D @ L.T)[1:, 1:] == B[1:, 1:]).all()
    G = A[3:][:, F.perm]
    assert ((F.out[3:] @ D @ L.T)[:, 1:] == G[:, 1:]).all()
    # inertia of D: one zero, two positive ([[2, 1], [1, 3]]: det 5, trace 5)
    ev = np.linalg.eigvalsh(np.array(D, dtype=float))
    assert (int((ev > 1e-12).sum()), int((ev < -1e-12).sum())) == (2, 0)
    assert int((np.abs(ev) <= 1e-12).sum()) == 1


def test_zero_pivot_leaves_the_trailing_block_alone():
    # The state right after the forced zero pivot on column 1: rows and
    # columns 0 and 1 interchanged, column 0 zeroed below the diagonal, R
    # column 0 zeroed, and the trailing block exactly the original entries.
    A = _tiny_column_panel()
    e = EPS
    T = factor_trapezoid(A[:3], A[3:], U, SMALL, R_NORMAL, forced=[("zero", 1)])
    assert T.nelim == 1 and list(T.perm) == [1, 0, 2] and T.status == ST_ZERO_PIVOT
    assert T.T[0, 0] == 0 and T.T[1, 0] == 0 and T.T[2, 0] == 0
    assert (T.T[1:, 1:] == _fr([[2, 1], [1, 3]])).all()
    assert (T.R == _fr([[0, 1, 2], [0, -1, 1]])).all()
    # the interchange put the old row 1 (all e) at the top; only its upper
    # part survives, as working storage
    assert T.T[0, 1] == e and T.T[0, 2] == e


def _zero_column_panel():
    # A11 (lower)           A21
    #   [ 0        ]        [ 0  1  1 ]
    #   [ 0  4     ]        [ 0  2 -1 ]
    #   [ 0  1  -2 ]
    # Column 0 is exactly zero, A21 part included.
    return _fr([[0, 0, 0], [0, 4, 0], [0, 1, -2], [0, 1, 1], [0, 2, -1]])


@pytest.mark.parametrize("method", METHODS)
def test_exactly_zero_column_is_found_in_the_second_pass(method):
    # m = 1, t = 0: a_tt = a_tm = 0, det = 0 -> 2x2 rejected; 1x1 on
    #  column 1: |4| >= u * 2 (TPP maxm = max(1, R 1, 2) = 2) -> position 0,
    #  perm = [1, 0, 2]; l = w / 4 with w = (0, 1): l = (0, 1/4);
    #  trailing: a22 = -2 - (1/4)(1) = -9/4, the zero column stays zero.
    #  TPP R rows (after the interchange (1, 0, 1), (2, 0, -1)): L21 column
    #  (1/4, 1/2), R column 2 becomes (1 - 1/4, -1 - 1/2) = (3/4, -3/2).
    # m = 2, t = 1: det = 0 again -> rejected; 1x1 on the old column 2:
    #  |-9/4| >= u * 3/2 -> position 1, perm = [1, 2, 0]; l = 0 for the
    #  zero row; TPP L21 column (3/4, -3/2) / (-9/4) = (-1/3, 2/3).
    # New pass, m = 2 (the old column 0): every entry 0 < small -> zero
    #  pivot at position 2.  The other rules meet the same decisions (the
    #  compressed columns carry the same zeros and no larger maxima).
    A = _zero_column_panel()
    F = factor_supernode(A, 3, method, u=U, small=SMALL)
    assert [d.kind for d in F.log] == ["1x1", "1x1", "pass", "zero"]
    assert list(F.perm) == [1, 2, 0]
    assert list(F.piv) == [PIV_1X1, PIV_1X1, PIV_ZERO]
    assert list(F.d) == [4, 0, Fr(-9, 4), 0, 0, 0]
    assert F.status == ST_ZERO_PIVOT
    assert F.out[1, 0] == Fr(1, 4) and F.out[2, 0] == 0 and F.out[2, 1] == 0
    assert F.out[2, 2] == 0
    assert list(F.out[3]) == [Fr(1, 4), Fr(-1, 3), 0]
    assert list(F.out[4]) == [Fr(1, 2), Fr(2, 3), 0]
    # P A11 P^T = L D L^T exactly, and A21 P^T = L21 D L^T
    A11 = np.tril(A[:3]) + np.tril(A[:3], -1).T
    L = unit_lower_L11(F.out, F.piv, 3)
    D = d_blocks(F.piv, F.d, 3)
    assert ((L @ D @ L.T) == A11[np.ix_(F.perm, F.perm)]).all()
    assert ((F.out[3:] @ D @ L.T) == A[3:][:, F.perm]).all()
    # inertia: 4 > 0, -9/4 < 0, one zero; A11's eigenvalues are 0 and those
    # of [[4, 1], [1, -2]] (det -9 < 0): one of each sign
    assert sorted(np.sign([float(x) for x in np.diag(D)])) == [-1, 0, 1]


def test_root_fallback_two_by_two_branch():
    # A11 = [[0, 1], [1, 0]] above the row R = (1000, 1000), TPP, root.
    # m = 1, t = 0: det = -1 is safe (|det| = 1 > 1/2), but
    #  |D^-1| = [[0, 1], [1, 0]] gives (maxm, maxt) = (1000, 1000) > 100;
    #  1x1: 0 < u * 1000 -> rejected.  Second pass: column 0 alone fails,
    #  column 1 fails again; no progress -> fallback at position 0:
    #  |a00| = 0 < small, the pair (0, 1) passes the determinant test -> 2x2
    #  regardless of u.  D^-1 = [[0, 1], [1, 0]], L21 = (1000, 1000).
    A11 = _fr([[0, 0], [1, 0]])
    R = _fr([[1000, 1000]])
    T = factor_trapezoid(A11, R, U, SMALL, R_NORMAL, root=True)
    assert [d.kind for d in T.log] == ["reject", "pass", "reject", "reject", "fallback"]
    assert T.nelim == 2 and list(T.perm) == [0, 1]
    assert list(T.piv) == [PIV_2X2_FIRST, PIV_2X2_SECOND]
    assert list(T.d) == [0, 1, 0, 0]
    assert (T.R == _fr([[1000, 1000]])).all()
    assert T.status == ST_ROOT_FALLBACK
    # without the root flag both columns stay delayed
    T0 = factor_trapezoid(A11, R, U, SMALL, R_NORMAL)
    assert T0.nelim == 0 and T0.status == 0


def test_root_fallback_zero_branch():
    # A11 = 0 (2 x 2) above R = (1, 1), TPP, root.  Neither column is a
    # zero column (the R entry is 1), the pair has |D| = 0 < small, and
    # each 1x1 has 0 < u * 1.  No progress -> fallback at position 0:
    # |a00| < small and det_ok fails (max |D| < small) -> zero pivot, R
    # column zeroed; the restart finds column 1 failing alone -> fallback
    # again, now the last column -> zero pivot.
    A11 = _fr([[0, 0], [0, 0]])
    R = _fr([[1, 1]])
    T = factor_trapezoid(A11, R, U, SMALL, R_NORMAL, root=True)
    assert [d.kind for d in T.log] == ["reject", "pass", "reject", "reject", "fallback", "reject",
                                       "fallback"]
    assert T.nelim == 2 and list(T.piv) == [PIV_ZERO, PIV_ZERO]
    assert list(T.d) == [0, 0, 0, 0]
    assert (T.R == 0).all()
    assert T.status == ST_ZERO_PIVOT | ST_ROOT_FALLBACK


def _float_panel():
    A = np.array([[4.0, 0, 0], [1, -3, 0], [0.5, 1, 2], [1, 2, 3], [-2, 1, 0.5], [0.25, -1, 1]])
    return A


@pytest.mark.parametrize("method", METHODS)
def test_finite_panel_has_no_status(method):
    assert factor_supernode(_float_panel(), 3, method).status == 0


@pytest.mark.parametrize("method,expect", [("tpp", ST_NONFINITE), ("strict", ST_NONFINITE),
                                           ("relaxed", ST_NONFINITE), ("restricted", 0)])
def test_nan_in_a21(method, expect):
    # A NaN in A21: compression reads every A21 entry (strict, relaxed), TPP
    # reads the entry when its column is tested, restricted pivoting never
    # reads A21.
    A = _float_panel()
    A[4, 1] = np.nan
    with np.errstate(invalid="ignore"):
        F = factor_supernode(A, 3, method)
    assert F.status & ST_NONFINITE == expect


@pytest.mark.parametrize("method", METHODS)
def test_infinity_on_the_diagonal(method):
    # every rule tests column 0 at some point: its diagonal is read
    A = _float_panel()
    A[0, 0] = np.inf
    with np.errstate(invalid="ignore"):
        F = factor_supernode(A, 3, method)
    assert F.status & ST_NONFINITE
