"""Pins of the early 2x2 rejection (oracle/threshold.py: reject_2x2_early):
the 2x2 test of eq. (2.2) decided before column t's maximum is known.

It may only reject pairs that the full test (accept_2x2) rejects for every
maxt >= 0, and it must actually fire on the two cases the rule names (the
determinant test fails; a term without maxt exceeds 1/u).
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.threshold import accept_2x2, reject_2x2_early

SMALL = 1e-20


def test_singular_pair_is_rejected_without_maxt():
    # D = [[1, 1], [1, 1]]: det = 0, the determinant test fails
    assert reject_2x2_early(Fr(1), Fr(1), Fr(1), Fr(5), Fr(1, 100), Fr(0))
    assert not accept_2x2(Fr(1), Fr(1), Fr(1), Fr(0), Fr(5), Fr(1, 100), Fr(0))[0]


def test_stability_term_without_maxt():
    # D = [[2, 1/2], [1/2, 1]] (a_tt = 2, a_tm = 1/2, a_mm = 1): big = 2,
    # s = 1/2, det0 = (1 * 1/2) * 2 = 1, det1 = (1/2 * 1/2) * 1/2 = 1/8,
    # det = 7/8 > max(1/2, 1/16); f = s / det = 4/7.  The second component
    # of |D^-1| (maxt, maxm) has the term (f |a_tt|) maxm = (8/7) maxm, so
    # with u = 1/100 it exceeds 100 by itself once maxm > 87.5.
    a_tt, a_tm, a_mm, u = Fr(2), Fr(1, 2), Fr(1), Fr(1, 100)
    assert reject_2x2_early(a_tt, a_tm, a_mm, Fr(88), u, Fr(0))
    assert not reject_2x2_early(a_tt, a_tm, a_mm, Fr(87), u, Fr(0))
    # at maxm = 87 the outcome depends on maxt: accepted with maxt = 0,
    # rejected with a large maxt
    assert accept_2x2(a_tt, a_tm, a_mm, Fr(0), Fr(87), u, Fr(0))[0]
    assert not accept_2x2(a_tt, a_tm, a_mm, Fr(1000), Fr(87), u, Fr(0))[0]


def test_small_column_branch_is_left_to_the_full_test():
    # maxm below small: the full test may accept through its small-column
    # branch (both maxima below small), so nothing is decided early
    assert not reject_2x2_early(2.0, 0.5, 1.0, 1e-30, 0.01, SMALL)
    assert accept_2x2(2.0, 0.5, 1.0, 1e-30, 1e-30, 0.01, SMALL)[0]


@pytest.mark.parametrize("u", [0.01, 0.1, 0.5])
def test_early_rejection_implies_rejection_for_every_maxt(u):
    rng = np.random.default_rng(7)
    fired = 0
    maxts = [0.0, 1e-300, 1e-20, 1e-3, 1.0, 37.0, 1e10, 1e300, np.inf]
    for _ in range(4000):
        scale = 10.0 ** rng.uniform(-6, 3, size=4)
        a_tt, a_tm, a_mm = rng.standard_normal(3) * scale[:3]
        if rng.random() < 0.2:                 # near-singular pairs
            a_mm = a_tm * a_tm / a_tt * (1 + rng.uniform(-1e-3, 1e-3))
        maxm = abs(rng.standard_normal()) * scale[3]
        if reject_2x2_early(a_tt, a_tm, a_mm, maxm, u, SMALL):
            fired += 1
            for maxt in maxts + list(np.abs(rng.standard_normal(4)) * 10.0 ** rng.uniform(-5, 5, size=4)):
                assert not accept_2x2(a_tt, a_tm, a_mm, maxt, maxm, u, SMALL)[0], (a_tt, a_tm, a_mm, maxm, maxt)
    assert fired > 400        # the rule does fire on a good share of random pairs
