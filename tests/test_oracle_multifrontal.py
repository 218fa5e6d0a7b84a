"""Pins of the Scatter oracle (oracle/multifrontal.py) on the CPU.

What fixes the answers independently of the oracle's own code:

* extend-add on a hand-worked 3 x 3 example (Section 1, Scatter);
* a contribution block is the Schur complement of its front with respect to
  the eliminated positions, F_RR - F_RE F_EE^-1 F_ER, whatever the pivot
  order (closed form with a dense solve);
* an assembled front is the Schur complement of the original matrix with
  respect to every variable eliminated below the node, the boundary x
  boundary original entries left out (they belong to an ancestor);
* the gathered factors reproduce P A P^T, the inertia of D is that of A
  (eigenvalue signs), the threshold rules keep |l| <= 1/u, and delayed
  pivots appear in the parent front (Section 1: delays move to a later
  supernode, the root eliminates everything).
"""

import numpy as np
import pytest

from oracle.multifrontal import (contribution_block, boundary_block, extend_add, global_factors,
                                 multifrontal)
from oracle.supernode import factor_supernode
from workloads import assembly_tree

RULES = ["relaxed", "strict", "tpp", "restricted"]


def test_extend_add_hand_worked():
    Fp = np.zeros((3, 3))
    Fp[1, 1] = 5.0
    C = np.array([[1.0, 2.0], [2.0, 3.0]])
    extend_add(Fp, C, [2, 0])
    assert (Fp == np.array([[3.0, 0.0, 2.0], [0.0, 5.0, 0.0], [2.0, 0.0, 1.0]])).all()
    extend_add(Fp, np.array([[1.0]]), [1])
    assert Fp[1, 1] == 6.0
    with pytest.raises(ValueError):
        extend_add(Fp, C, [1, 1])


def _front(seed, n, p, bound_scale):
    """A random symmetric front whose boundary rows are scaled up, so that
    the threshold rules delay some columns."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    Fr = np.tril(G) + np.tril(G, -1).T
    Fr[p:, :p] *= bound_scale
    Fr[:p, p:] *= bound_scale
    return Fr


@pytest.mark.parametrize("method", RULES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_contribution_is_schur_complement_of_front(method, seed):
    n, p = 40, 16
    Fr = _front(seed, n, p, 20.0)
    F = factor_supernode(Fr[:, :p].copy(), p, method)
    C = contribution_block(F, boundary_block(F, Fr[p:, p:]))
    E = F.perm[:F.nelim]
    R = np.concatenate([F.perm[F.nelim:], np.arange(p, n)])
    expect = Fr[np.ix_(R, R)] - Fr[np.ix_(R, E)] @ np.linalg.solve(Fr[np.ix_(E, E)], Fr[np.ix_(E, R)])
    assert C.shape == (n - F.nelim, n - F.nelim)
    assert np.abs(C - expect).max() <= 1e-11 * np.abs(expect).max()
    if method == "strict":
        assert F.nelim < p       # the scaled boundary makes the strict rule delay


def _subtree_eliminated(tree, fronts, q):
    out = []
    for ch in tree["children"][q]:
        out.extend(_subtree_eliminated(tree, fronts, ch))
        F = fronts[ch]["F"]
        out.extend(int(fronts[ch]["vars"][F.perm[k]]) for k in range(F.nelim))
    return out


@pytest.mark.parametrize("method", RULES)
@pytest.mark.parametrize("seed,bound_scale", [(0, 1.0), (1, 30.0), (2, 30.0)])
def test_assembled_front_is_schur_complement(method, seed, bound_scale):
    tree = assembly_tree(seed, bound_scale=bound_scale)
    A = tree["A"]
    fronts = multifrontal(tree, method)
    for q in tree["postorder"]:
        if not tree["children"][q]:
            continue
        fr = fronts[q]
        R = fr["vars"]
        E = np.asarray(_subtree_eliminated(tree, fronts, q))
        A0 = A[np.ix_(R, R)].copy()
        A0[fr["p"]:, fr["p"]:] = 0.0
        expect = A0 - A[np.ix_(R, E)] @ np.linalg.solve(A[np.ix_(E, E)], A[np.ix_(E, R)])
        assert np.abs(fr["assembled"] - expect).max() <= 1e-11 * np.abs(expect).max(), q


@pytest.mark.parametrize("method", RULES)
@pytest.mark.parametrize("seed,bound_scale", [(0, 1.0), (1, 30.0), (3, 30.0)])
def test_multifrontal_factors(method, seed, bound_scale):
    u = 0.01
    tree = assembly_tree(seed, bound_scale=bound_scale)
    A = tree["A"]
    fronts = multifrontal(tree, method, u)
    order, L, D = global_factors(tree, fronts)
    assert np.array_equal(np.sort(order), np.arange(A.shape[0]))
    res = np.abs(A[np.ix_(order, order)] - L @ D @ L.T).max() / np.abs(A).max()
    assert res <= 1e-11
    ev, ed = np.linalg.eigvalsh(A), np.linalg.eigvalsh(D)
    assert (ev > 0).sum() == (ed > 0).sum() and (ev < 0).sum() == (ed < 0).sum()
    if method in ("strict", "tpp"):
        assert np.abs(np.tril(L, -1)).max() <= (1 + 1e-12) / u
    # delayed variables reach the parent front, ahead of its own variables
    root = tree["postorder"][-1]
    for q in tree["postorder"]:
        fr = fronts[q]
        if q == root:
            assert fr["F"].nelim == fr["p"]
            continue
        par = fronts[tree["parent"][q]]
        delayed = fr["cvars"][:fr["ndelay"]]
        nd_par = par["p"] - tree["own"][tree["parent"][q]].size
        assert set(delayed.tolist()) <= set(par["vars"][:nd_par].tolist())
    if bound_scale > 1 and method != "restricted":
        assert sum(fronts[q]["ndelay"] for q in tree["postorder"]) > 0
