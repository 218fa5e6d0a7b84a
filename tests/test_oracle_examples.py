"""The oracle against the values the paper prints and small hand-worked runs.

These pins do not use the oracle to compute their expectations: the
compressed matrices are the paper's figures, the growth example is the
paper's display, and the short pivot runs below were worked by hand from
eqs. (2.1), (2.2), (4.3) and (4.4) in exact rational arithmetic (the working
is in the comments).
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

from golden_io import golden
from oracle.supernode import compress_relaxed, compress_strict, factor_supernode
from oracle.threshold import (PIV_1X1, PIV_2X2_FIRST, PIV_2X2_SECOND, PIV_DELAYED,
                              R_ABS, R_NORMAL, factor_trapezoid)


@pytest.mark.parametrize("exact", [False, True])
def test_fig_4_2_strict_compressed_matrix(exact):
    g = golden("fig4_2_strict.txt", exact)
    C = compress_strict(g["A21"])
    assert (C == g["C"]).all()


@pytest.mark.parametrize("exact", [False, True])
def test_fig_4_3_relaxed_compressed_matrix(exact):
    g = golden("fig4_3_relaxed.txt", exact)
    C, rows = compress_relaxed(g["A21"])
    assert (C == g["C"]).all()
    assert list(rows) == [int(r) for r in g["ROWS"][0]]


def test_relaxed_tie_order_matters():
    # Section 4.2 remarks that meeting row 3 before row 1 changes C: swap
    # the two rows and the tie at column 2 goes to the (new) first row.
    g = golden("fig4_3_relaxed.txt")
    A = g["A21"][[2, 1, 0, 3, 4]]
    C, rows = compress_relaxed(A)
    # column 2 now takes [0, 10, -3]; the old row 1 (now at index 2) wins
    # column 3 instead, since |10| > |8|.
    assert list(rows) == [3, 0, 2]
    assert (C[1] == [0, 10, -3]).all()
    assert (C[2] == [1, 10, 10]).all()


def _section5_example():
    g = golden("section5_relaxed_example.txt", exact=True)
    return g["A"], g["L"], Fr(1) / g["U"][0, 0]


def test_section5_growth_example_natural_order():
    # Forced 1x1 pivots in natural order reproduce the paper's L exactly,
    # including the entry 2(1/u - e) > 1/u in the row left out of C.
    A, L, u = _section5_example()
    F = factor_supernode(A, 2, "relaxed", u=u, small=Fr(1, 10**20),
                         forced=[("1x1", 0), ("1x1", 1)])
    assert F.nelim == 2 and list(F.perm) == [0, 1]
    assert F.out[1, 0] == L[1, 0]
    assert (F.out[2:, :] == L[2:, :]).all()
    assert F.out[4, 1] > 1 / u


def test_section5_example_under_the_pivot_rules():
    # Worked by hand with u = 1/100 (U = 100), small = 1e-20:
    #  m = col 2, t = col 1: s = 1/2, det1 = (-1/2)(-1) = 1/2,
    #  det0 = (2/2)(1) = 1, det = 1/2 <= max(small, 1/2, 1/4) -> 2x2 rejected.
    #  1x1 on col 2: maxm = max(|a12| = 1, C col 2 = (0, U)) = U and
    #  |a22| = 2 >= u U = 1 -> accepted, column 2 moves to position 1.
    #  Column 1 becomes 1 - (-1)(-1)/2 = 1/2; its C entries become U and
    #  0 - (U/2)(-1) = U/2.  New pass: 1/2 >= u U = 1 fails -> delayed.
    A, _, u = _section5_example()
    small = Fr(1, 10**20)
    for method in ("relaxed", "tpp", "strict"):
        F = factor_supernode(A, 2, method, u=u, small=small)
        assert F.nelim == 1, method
        assert list(F.perm) == [1, 0], method
        assert list(F.piv) == [PIV_1X1, PIV_DELAYED], method
        assert F.d[0] == 2
        assert F.out[1, 1] == Fr(1, 2)      # updated delayed diagonal
    # the relaxed C after the step (column 1 = the delayed column)
    F = factor_supernode(A, 2, "relaxed", u=u, small=small)
    assert (F.trap.R[:, 1] == [100, 50]).all()
    assert (F.trap.R[:, 0] == [0, 50]).all()   # L entries of the C rows


# A 3 x 3 A11 above the A21 of Figs. 4.2 / 4.3, worked by hand (u = 1/100).
A11_HAND = np.array([[4, 0, 0], [1, 2, 0], [2, 1, 3]])


def _hand_panel():
    A21 = golden("fig4_2_strict.txt", exact=True)["A21"]
    top = np.array([[Fr(int(x)) for x in r] for r in A11_HAND], dtype=object)
    return np.vstack([top, A21])


def test_hand_worked_strict_run():
    # Strict C = [[0,0,0],[4,10,10],[2,6,8]].
    # m = col 2, t = col 1: a_tt = 4, a_tm = 1, a_mm = 2; s = 1/4,
    #  det1 = 1/4, det0 = 2, det = 7/4 > max(small, 1, 1/8) = 1.
    #  maxt = max(|a31| = 2, C col 1 = 4) = 4, maxm = max(|a32| = 1, 10) = 10,
    #  f = s/|det| = 1/7: g_t = (2/7) 4 + (1/7) 10 = 18/7,
    #  g_m = (1/7) 4 + (4/7) 10 = 44/7, both <= 100 -> 2x2 accepted.
    #  D^-1 = (1/7)[[2, -1], [-1, 4]]; row 3: l = (3/7, 2/7),
    #  a33 = 3 - (6/7 + 2/7) = 13/7.
    #  |D^-1| on C rows: row 2 -> (18/7, 44/7), c23 = 10 + 36/7 + 44/7 = 150/7;
    #  row 3 -> (10/7, 26/7), c33 = 8 + 20/7 + 26/7 = 102/7.
    # New pass, col 3 alone: maxm = 150/7, 13/7 >= 1.5/7 -> 1x1;
    #  C column 3 becomes (0, 150/13, 102/13).
    A = _hand_panel()
    F = factor_supernode(A, 3, "strict", u=Fr(1, 100), small=Fr(1, 10**20))
    assert [dec.kind for dec in F.log] == ["2x2", "pass", "1x1"]
    assert F.nelim == 3 and list(F.perm) == [0, 1, 2]
    assert list(F.piv) == [PIV_2X2_FIRST, PIV_2X2_SECOND, PIV_1X1]
    assert list(F.d) == [4, 1, 2, 0, Fr(13, 7), 0]
    expect_C = np.array([[0, 0, 0],
                         [Fr(18, 7), Fr(44, 7), Fr(150, 13)],
                         [Fr(10, 7), Fr(26, 7), Fr(102, 13)]], dtype=object)
    assert (F.trap.R == expect_C).all()
    assert F.out[2, 0] == Fr(3, 7) and F.out[2, 1] == Fr(2, 7)
    dec = F.log[0]
    assert dec.vals["maxt"] == 4 and dec.vals["maxm2"] == 10


def test_hand_worked_relaxed_run():
    # Relaxed C = [[4,-5,4],[1,10,10],[0,-6,8]]: the same first decision
    # (maxt = 4, maxm = 10).  Ordinary update of the C rows with
    # D^-1 = (1/7)[[2,-1],[-1,4]] and (w1, w2) = (2, 1):
    #  row 1: l = (13/7, -24/7), c13 = 4 - (26/7 - 24/7) = 26/7
    #  row 2: l = (-8/7, 39/7),  c23 = 10 - (-16/7 + 39/7) = 47/7
    #  row 3: l = (6/7, -24/7),  c33 = 8 - (12/7 - 24/7) = 68/7
    # New pass, col 3: maxm = 68/7, 13/7 >= 0.68/7 -> 1x1; C column 3
    #  divided by 13/7: (2, 47/13, 68/13).
    A = _hand_panel()
    F = factor_supernode(A, 3, "relaxed", u=Fr(1, 100), small=Fr(1, 10**20))
    assert [dec.kind for dec in F.log] == ["2x2", "pass", "1x1"]
    expect_C = np.array([[Fr(13, 7), Fr(-24, 7), 2],
                         [Fr(-8, 7), Fr(39, 7), Fr(47, 13)],
                         [Fr(6, 7), Fr(-24, 7), Fr(68, 13)]], dtype=object)
    assert (F.trap.R == expect_C).all()
    # C rows are rows 4, 1, 5 of A21, updated exactly as the TPP run
    # updates those same rows.
    T = factor_supernode(A, 3, "tpp", u=Fr(1, 100), small=Fr(1, 10**20))
    assert (T.out[3 + np.array([3, 0, 4])] == expect_C).all()


def test_hand_worked_one_by_one_then_two_by_two():
    # A11 = [[1e-3, ., .], [0, 1e-3, .], [1, 1, 0]] with A21 = 0:
    # m = col 2, t = col 1: D = diag(1e-3, 1e-3), det = 1e-3 > 5e-4,
    #  maxt = |a31| = 1, maxm = |a32| = 1, |D^-1| (1,1) = (1000, 1000) > 100
    #  -> rejected; 1x1 on col 2: 1e-3 >= 0.01 * 1 fails -> rejected.
    # m = col 3, t = argmax(|a31|, |a32|) = col 1 (tie, lowest): D =
    #  [[1e-3, 1], [1, 0]], s = 1, det1 = 1, det0 = 0, det = -1,
    #  |det| = 1 > max(small, 0, 1/2); maxt = |a21| = 0, maxm = |a23| = 1
    #  (rows other than t, m: only col 2); |D^-1| = [[0, 1], [1, 1e-3]]
    #  -> (1, 1e-3) <= 100 -> 2x2 (col 1, col 3), positions 1 and 2.
    # Then col 2 updated: a22 - [0 1] D^-1 [0 1]^T with D^-1 =
    #  [[0, 1], [1, -1e-3]]: 1e-3 - (-1e-3) = 2e-3; new pass accepts it
    #  as a 1x1 (no other entries left).
    e = Fr(1, 1000)
    A = np.array([[e, 0, 0], [0, e, 0], [1, 1, 0], [0, 0, 0]], dtype=object)
    A = np.array([[Fr(x) for x in r] for r in A], dtype=object)
    F = factor_supernode(A, 3, "tpp", u=Fr(1, 100), small=Fr(1, 10**20))
    assert [dec.kind for dec in F.log] == ["reject", "2x2", "pass", "1x1"]
    assert list(F.perm) == [0, 2, 1]
    assert list(F.d) == [e, 1, 0, 0, 2 * e, 0]
