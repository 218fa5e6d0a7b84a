"""Scatter task: extend-add of a front's contribution into its parent, and
a multifrontal factorization over an assembly tree -- plain CPU oracle.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path; it shares no
code with the HIP library.

Section 1 lists Scatter as the fourth task on a supernode: S is added into
the fronts of other supernodes (multifrontal or supernodal techniques).  It
also says where delayed pivots go: a column that fails the pivot test at a
node is moved to a later supernode, and the final (root) supernode
eliminates everything.  In the multifrontal form used here:

* the front of node q is a dense symmetric matrix over the index list
  [variables delayed by q's children (child by child, in each child's
  position order)] + [q's own variables] + [q's boundary]; its first
  p = |delayed| + |own| columns are the supernode panel [A11; A21], the
  trailing block over the boundary is A22;
* the front holds the original entries of its own variables (own x own and
  boundary x own) and the extend-add of every child's contribution block;
  the boundary x boundary entries of the original matrix belong to an
  ancestor and are not assembled here;
* after Factor + Solve the contribution block is the trailing matrix over
  positions nelim..n-1: the delayed block and delayed columns as the panel
  holds them after the eliminations, and A22 - L21 D L21^T over the
  boundary (Form with the front's own trailing entries).
"""

import numpy as np

from .supernode import d_blocks, factor_supernode
from .threshold import PIV_2X2_FIRST


def boundary_block(F, A22):
    """A22 - L21 D11 L21^T: the boundary part of the contribution (Form,
    Section 1, applied to the front's own trailing entries)."""
    p = F.out.shape[1]
    L21 = F.out[p:, :F.nelim]
    D = d_blocks(F.piv, F.d, F.nelim)
    return A22 - (L21 @ D) @ L21.T


def contribution_block(F, S22):
    """The front's contribution to its parent over positions nelim..n-1
    (full symmetric): rows and columns of the delayed positions nelim..p-1
    come from the panel after the eliminations (the delayed block in the A11
    rows, lower triangle, and the delayed columns in the A21 rows); the
    boundary block is S22."""
    n, p = F.out.shape
    ne = F.nelim
    pd = p - ne
    C = np.zeros((n - ne, n - ne))
    Dd = np.tril(F.out[ne:p, ne:p])
    C[:pd, :pd] = Dd + np.tril(Dd, -1).T
    C[pd:, :pd] = F.out[p:, ne:p]
    C[:pd, pd:] = F.out[p:, ne:p].T
    C[pd:, pd:] = S22
    return C


def extend_add(Fp, C, pos):
    """Scatter (Section 1): Fp[pos[i], pos[j]] += C[i, j] for every i, j.

    pos maps the rows of the contribution block to rows of the parent
    front; it must be injective (each entry of the parent receives at most
    one entry of C)."""
    pos = np.asarray(pos)
    if np.unique(pos).size != pos.size:
        raise ValueError("extend-add map is not injective")
    Fp[np.ix_(pos, pos)] += C


def original_front(A, own, bound, ndelay):
    """The original entries of a front with index list [ndelay delayed
    variables] + own + bound: own x own and boundary x own (and their
    transposes); every other entry zero."""
    po = ndelay + own.size
    n = po + bound.size
    Fr = np.zeros((n, n))
    Fr[ndelay:po, ndelay:po] = A[np.ix_(own, own)]
    Fr[po:, ndelay:po] = A[np.ix_(bound, own)]
    Fr[ndelay:po, po:] = A[np.ix_(own, bound)]
    return Fr


def multifrontal(tree, method="relaxed", u=0.01, small=1e-20):
    """Multifrontal LDL^T of tree["A"] over the assembly tree (nodes in
    tree["postorder"], root last), every front factored with
    factor_supernode and the root with every column eliminated.

    Returns a dict per node q (fronts[q]): vars (the front's index list),
    p, assembled (the full symmetric front before its factorization), F (the
    SupernodeFactors), cvars (global variables of the contribution block) and
    C (the contribution block; None at the root).
    """
    A = tree["A"]
    root = tree["postorder"][-1]
    fronts = {}
    for q in tree["postorder"]:
        kids = tree["children"][q]
        delayed = [v for ch in kids for v in fronts[ch]["cvars"][:fronts[ch]["ndelay"]]]
        own, bound = tree["own"][q], tree["bound"][q]
        vars_ = np.concatenate([np.asarray(delayed, dtype=np.int64), own, bound])
        p = len(delayed) + own.size
        Fr = original_front(A, own, bound, len(delayed))
        where = {int(v): i for i, v in enumerate(vars_)}
        for ch in kids:
            fc = fronts[ch]
            extend_add(Fr, fc["C"], [where[int(v)] for v in fc["cvars"]])
        F = factor_supernode(Fr[:, :p].copy(), p, method, u, small, root=(q == root))
        rec = {"vars": vars_, "p": p, "assembled": Fr, "F": F, "cvars": None, "C": None, "ndelay": p - F.nelim}
        if q != root:
            S22 = boundary_block(F, Fr[p:, p:])
            rec["C"] = contribution_block(F, S22)
            rec["cvars"] = np.concatenate([vars_[F.perm[F.nelim:p]], vars_[p:]])
        fronts[q] = rec
    return fronts


def global_factors(tree, fronts):
    """The factorization P A P^T = L D L^T gathered from the fronts:
    order[k] = global variable eliminated k-th (postorder, each front's
    eliminated positions in order), L (N x N unit lower in that order) and
    D (block diagonal)."""
    N = tree["A"].shape[0]
    order = []
    for q in tree["postorder"]:
        fr = fronts[q]
        F = fr["F"]
        order.extend(int(fr["vars"][F.perm[k]]) for k in range(F.nelim))
    if len(order) != N:
        raise ValueError("not every variable was eliminated")
    rank = np.empty(N, dtype=np.int64)
    rank[np.asarray(order)] = np.arange(N)
    L = np.eye(N)
    D = np.zeros((N, N))
    for q in tree["postorder"]:
        fr = fronts[q]
        F, p, vars_ = fr["F"], fr["p"], fr["vars"]
        n = vars_.size
        # global variable at each final position of the front
        at = np.concatenate([vars_[F.perm], vars_[p:]])
        Dq = d_blocks(F.piv, F.d, F.nelim)
        for k in range(F.nelim):
            gk = rank[at[k]]
            for t in range(k + 1, n):
                if t == k + 1 and F.piv[k] == PIV_2X2_FIRST:
                    continue          # that slot holds D's off-diagonal
                L[rank[at[t]], gk] = F.out[t, k]
            for j in range(F.nelim):
                D[rank[at[j]], gk] = Dq[j, k]
    return np.asarray(order), L, D
