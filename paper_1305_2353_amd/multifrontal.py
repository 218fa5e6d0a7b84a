"""Multifrontal LDL^T over an assembly tree, level by level, from the C
interface's batched calls (Section 1: Factor, Solve, Form and Scatter on
every supernode; delayed pivots move to the parent, the root eliminates
everything).

The host keeps only the symbolic side: each front's index list (variables
delayed by its children, child by child in each child's position order,
then its own variables, then its boundary), the heights that group fronts
into levels, the buffer offsets of each batch and the extend-add maps.  All
arithmetic runs in the library:

    for each level (leaves first):
        a ctp Batch of the level's fronts (Form with CTP_FLAG_S_SUBTRACT, so
        each front's S buffer, holding its trailing block A22, ends as
        A22 - L21 D L21^T; the root level with CTP_FLAG_ROOT);
        the original entries of the fronts' own variables are copied in
        (own x own and boundary x own of the global matrix);
        every child's contribution is added by ctp_extend_add_batched, in
        rounds of at most one child per parent;
        ctp_supernode_batched;
        nelim and perm come back to the host (the parents' index lists
        depend on which variables were delayed).

Batches take the compressed and restricted rules (as ctp_supernode_batched).
"""

import ctypes

import numpy as np
import torch

from . import ctp


class Front:
    """One front after the factorization: its index list (global variables
    in the front's original order), panel width p, and where its outputs
    live (batch, index in the batch)."""

    def __init__(self, vars_, p, batch, index):
        self.vars = vars_
        self.p = p
        self.batch = batch
        self.index = index
        self.nelim = None
        self.perm = None
        self.assembled = None

    @property
    def n(self):
        return int(self.vars.size)

    def delayed(self):
        """Global variables of the delayed positions nelim..p-1, in order."""
        return self.vars[self.perm[self.nelim:self.p]]

    def outputs(self):
        """The front's panel (n x p, column-major view) and its perm, piv, d,
        nelim, status tensors."""
        out = self.batch.outputs(self.index)
        out["panel"] = self.batch.panel_view(self.index)
        return out


def _heights(parent, children, postorder):
    h = {}
    for q in postorder:
        h[q] = 1 + max((h[c] for c in children[q]), default=-1)
    return h


def multifrontal_factor(tree, A, method="relaxed", u=0.01, small=1e-20, keep_assembled=False):
    """Factor the global symmetric matrix A (N x N float64 device tensor)
    over tree (a dict with parent, children, own, bound, postorder -- the
    symbolic analysis).  Returns {node: Front}.  keep_assembled: keep a copy
    of every front as assembled (panel and trailing block) before its
    factorization, for checking."""
    if method not in ("relaxed", "strict", "restricted"):
        raise ctp.CtpError("the batched level takes the compressed and restricted rules")
    children, post = tree["children"], tree["postorder"]
    root = post[-1]
    height = _heights(tree["parent"], children, post)
    levels = [[q for q in post if height[q] == h] for h in range(height[root] + 1)]
    fronts = {}
    dev = A.device
    for level in levels:
        # index lists of the level's fronts
        infos = []
        for q in level:
            delayed = [fronts[c].delayed() for c in children[q]]
            delayed = np.concatenate(delayed) if delayed else np.zeros(0, dtype=np.int64)
            own, bound = np.asarray(tree["own"][q]), np.asarray(tree["bound"][q])
            vars_ = np.concatenate([delayed, own, bound]).astype(np.int64)
            infos.append((q, vars_, delayed.size + own.size, delayed.size))
        shapes = [(v.size, p) for _, v, p, _ in infos]
        flags = ctp.CTP_FLAG_S_SUBTRACT | (ctp.CTP_FLAG_ROOT if root in level else 0)
        opts = ctp.ctp_default_opts(method, u=u, small=small, flags=flags)
        batch = ctp.Batch(shapes, opts, form=[n > p for n, p in shapes], device=dev)
        batch.panels.zero_()
        if batch.S is not None:
            batch.S.zero_()
        for i, (q, vars_, p, nd) in enumerate(infos):
            own = torch.as_tensor(tree["own"][q], dtype=torch.long, device=dev)
            bound = torch.as_tensor(tree["bound"][q], dtype=torch.long, device=dev)
            panel = batch.panel_view(i)
            panel[nd:p, nd:p] = A[own][:, own]
            if bound.numel():
                panel[p:, nd:p] = A[bound][:, own]
            fronts[q] = Front(vars_, p, batch, i)
        _scatter_children(level, children, fronts, batch, dev)
        if keep_assembled:
            for q in level:
                fr = fronts[q]
                s = batch.s_view(fr.index)
                fr.assembled = (batch.panel_view(fr.index).clone(), s.clone() if s is not None else None)
        batch.run()
        nelim = batch.nelim.cpu().numpy()
        perm = batch.perm.cpu().numpy()
        for q in level:
            fr = fronts[q]
            nd = batch.node(fr.index)
            fr.nelim = int(nelim[fr.index])
            fr.perm = perm[nd.out_off:nd.out_off + nd.p].astype(np.int64)
    return fronts


def _scatter_children(level, children, fronts, batch, dev):
    """Extend-add every child of the level's fronts into them: one batched
    call per (child batch, round), round k taking the k-th child of each
    parent from that batch."""
    groups = {}
    for q in level:
        by_batch = {}
        for c in children[q]:
            by_batch.setdefault(id(fronts[c].batch), []).append(c)
        for key, cs in by_batch.items():
            for k, c in enumerate(cs):
                groups.setdefault((key, k), []).append((c, q))
    for (key, k), pairs in sorted(groups.items(), key=lambda kv: kv[0][1]):
        cb = fronts[pairs[0][0]].batch
        tasks = (ctp.CtpScatterTask * len(pairs))()
        maps, moff = [], 0
        for t, (c, q) in zip(tasks, pairs):
            fc, fq = fronts[c], fronts[q]
            cn, qn = cb.node(fc.index), batch.node(fq.index)
            where = {int(v): i for i, v in enumerate(fq.vars)}
            maps.append(np.array([where.get(int(v), -1) for v in fc.vars], dtype=np.int32))
            t.n, t.p, t.lda, t.lds = cn.n, cn.p, cn.lda, cn.lds
            t.np, t.pp, t.ldf, t.ld22 = qn.n, qn.p, qn.lda, qn.lds
            t.node = fc.index
            t.a_off, t.s_off, t.out_off = cn.a_off, cn.s_off, cn.out_off
            t.map_off = moff
            t.f_off, t.f22_off = qn.a_off, qn.s_off
            moff += cn.n
        tiles = ctp.ctp_scatter_plan(tasks)
        vmap = torch.as_tensor(np.concatenate(maps), device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        ctp.ctp_extend_add_batched(ctp.to_device_struct(tasks, dev), len(pairs), tiles, cb.panels, cb.S, cb.perm,
                                   cb.nelim, vmap, batch.panels, batch.S, status)
        if int(status.item()):
            raise ctp.CtpError("extend-add map out of range")
