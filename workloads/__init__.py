"""Seeded synthetic inputs shaped like the paper's timing workloads.

This module only draws random numbers and arranges them into matrices; it
holds none of the pivoting arithmetic.  Both the oracle-based checks and the
HIP path take their inputs from here, so that they see identical bits.

The paper times random dense supernodes (Section 7.1: p = 512 with n up to
100000, and n = 100000 with p up to 1024) without giving their
construction.  The recipes here are:

* supernode(n, p): A11 = tril(G) + tril(G,-1)^T with G ~ N(0,1)^(p x p),
  then a chosen number of diagonal entries (distinct, uniformly drawn)
  multiplied by a small factor so that some 1x1 candidates fail and 2x2
  pivots and delays occur; A21 ~ N(0,1)^((n-p) x p).  Draw order: G, the
  diagonal indices, A21.
* dense_indefinite(N): Q diag(lam) Q^T with Q the orthogonal factor of a
  Gaussian matrix (Householder QR, signs fixed by diag(R)) and lam half
  negative, half positive, |lam| ~ U[lo, 1], shuffled.
  dense_indefinite_torch(N) draws the same recipe with torch on a device
  (its own seeded stream, so a different matrix of the same law): the
  N = 16384 case would take minutes of CPU QR.
* batch of supernodes: n log-uniform, p uniform with p <= n/4.
* batch of dense systems (dense_indefinite_batch_torch): S independent
  draws of the dense_indefinite recipe on the device, one batched QR.

Every array is float64, row index first (n x p); the binding stores panels
column-major on the device.
"""

import numpy as np


def supernode(n, p, seed=0, n_small=0, small_scale=1e-8):
    """n x p supernode [A11; A21] (A11 stored as a full symmetric block)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((p, p))
    A11 = np.tril(G) + np.tril(G, -1).T
    if n_small:
        idx = rng.choice(p, n_small, replace=False)
        A11[idx, idx] *= small_scale
    A21 = rng.standard_normal((n - p, p))
    return np.vstack([A11, A21])


def small_supernode(seed=0):
    """n = 256, p = 32: four diagonal entries scaled by 1e-8."""
    return supernode(256, 32, seed, n_small=4, small_scale=1e-8)


def large_supernode(seed=0):
    """n = 100000, p = 512: 2% of the diagonal (10 entries) scaled by 1e-6."""
    return supernode(100000, 512, seed, n_small=int(0.02 * 512), small_scale=1e-6)


def dense_indefinite(N, seed=0, lam_lo=1e-3, nrhs=0):
    """Symmetric indefinite Q diag(lam) Q^T, half the eigenvalues negative.

    Returns (A, lam) or (A, lam, B) when nrhs > 0 with B ~ N(0,1)^(N x nrhs).
    """
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((N, N))
    Q, R = np.linalg.qr(Z)
    Q = Q * np.sign(np.diag(R))
    half = N // 2
    lam = np.concatenate([-rng.uniform(lam_lo, 1.0, half),
                          rng.uniform(lam_lo, 1.0, N - half)])
    rng.shuffle(lam)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    if nrhs:
        B = rng.standard_normal((N, nrhs))
        return A, lam, B
    return A, lam


def batch_shapes(count, seed=0, n_lo=64, n_hi=8192, p_lo=8, p_hi=256):
    """Shapes of a batch of independent supernodes: n log-uniform in
    [n_lo, n_hi], p uniform in [p_lo, min(p_hi, n // 4)]."""
    rng = np.random.default_rng(seed)
    ns, ps = [], []
    for _ in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        p = int(rng.integers(p_lo, min(p_hi, n // 4) + 1))
        ns.append(n)
        ps.append(p)
    return np.array(ns), np.array(ps)


def batch_panel(n, p, rng, small_prob=0.01, small_scale=1e-8):
    """One supernode of a batch, drawn from a shared generator: tril-reflected
    A11, each diagonal entry scaled with probability small_prob."""
    G = rng.standard_normal((p, p))
    A11 = np.tril(G) + np.tril(G, -1).T
    mask = rng.random(p) < small_prob
    A11[mask, mask] *= small_scale
    A21 = rng.standard_normal((n - p, p))
    return np.vstack([A11, A21])


def dense_indefinite_torch(N, seed=0, lam_lo=1e-3, nrhs=0, device="cuda"):
    """dense_indefinite's recipe drawn with torch on `device` (FP64).

    Returns (A, lam, B) as device tensors (B None when nrhs == 0); A is
    row-major N x N and symmetric, so it is its own column-major copy."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Z = torch.randn((N, N), dtype=torch.float64, device=device, generator=g)
    Q, R = torch.linalg.qr(Z)
    del Z
    Q = Q * torch.sign(torch.diagonal(R))
    del R
    half = N // 2
    u = torch.rand(N, dtype=torch.float64, device=device, generator=g) * (1.0 - lam_lo) + lam_lo
    lam = torch.cat([-u[:half], u[half:]])
    lam = lam[torch.randperm(N, device=device, generator=g)]
    A = (Q * lam) @ Q.T
    del Q
    A = 0.5 * (A + A.T)
    B = torch.randn((N, nrhs), dtype=torch.float64, device=device, generator=g) if nrhs else None
    return A, lam, B


def batch_panel_torch(n, p, gen, device="cuda", small_prob=0.01, small_scale=1e-8):
    """batch_panel's recipe drawn with torch on `device` from generator
    `gen` (FP64, n x p, row index first)."""
    import torch
    G = torch.randn((p, p), dtype=torch.float64, device=device, generator=gen)
    A11 = torch.tril(G) + torch.tril(G, -1).T
    mask = torch.rand(p, dtype=torch.float64, device=device, generator=gen) < small_prob
    a = torch.diagonal(A11).clone()
    d = torch.where(mask, a * small_scale, a)
    A11 = A11 - torch.diag(a) + torch.diag(d)
    A21 = torch.randn((n - p, p), dtype=torch.float64, device=device, generator=gen)
    return torch.cat([A11, A21])


def dense_indefinite_batch_torch(S, N, seed=0, lam_lo=1e-2, nrhs=4, device="cuda"):
    """S systems of dense_indefinite's recipe drawn with torch on `device`
    (FP64): Z (S, N, N) Gaussian, Q from one batched QR with the signs of
    diag(R), lam per system half -U[lam_lo, 1] and half U[lam_lo, 1]
    shuffled, A = Q diag(lam) Q^T symmetrised, B (S, N, nrhs) Gaussian.
    Returns (A, B), row-major device tensors."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Z = torch.randn((S, N, N), dtype=torch.float64, device=device, generator=g)
    Q, R = torch.linalg.qr(Z)
    del Z
    Q = Q * torch.sign(torch.diagonal(R, dim1=1, dim2=2)).unsqueeze(1)
    del R
    half = N // 2
    u = torch.rand((S, N), dtype=torch.float64, device=device, generator=g) * (1.0 - lam_lo) + lam_lo
    lam = torch.cat([-u[:, :half], u[:, half:]], dim=1)
    idx = torch.argsort(torch.rand((S, N), device=device, generator=g), dim=1)
    lam = torch.gather(lam, 1, idx)
    A = torch.bmm(Q * lam.unsqueeze(1), Q.transpose(1, 2).contiguous())
    del Q
    A = 0.5 * (A + A.transpose(1, 2))
    B = torch.randn((S, N, nrhs), dtype=torch.float64, device=device, generator=g)
    return A, B


def assembly_tree(seed=0, fanout=(3, 2), own_lo=16, own_hi=48, root_own=40, bound_frac=0.5,
                  small_prob=0.05, small_scale=1e-8, bound_scale=1.0):
    """A symmetric indefinite matrix with a known assembly tree.

    Tree: a root whose nodes at depth d have fanout[d] children each (the
    depth is len(fanout)).  Every non-root node owns own ~ U{own_lo..own_hi}
    variables, the root owns root_own; variables are numbered in postorder
    (a node's subtree before the node, children in order).  A node's
    boundary is a random subset of its parent's front variables (the
    parent's own variables and boundary), of size max(1, round(bound_frac *
    that set)).  Entries: A[own, own] symmetric with G ~ N(0,1) reflected
    from its lower triangle and each diagonal entry multiplied by
    small_scale with probability small_prob (so that pivots fail and are
    delayed); A[boundary, own] ~ bound_scale * N(0,1) and its transpose (a
    large bound_scale makes the threshold test fail against the boundary
    rows, so that every rule delays); zero elsewhere.

    Draw order: own sizes (breadth first), then per node top-down the
    boundary subset, then per node in postorder G, the small-diagonal mask,
    the boundary block.

    Returns a dict: A (N x N), parent (-1 for the root), children, own and
    bound (int arrays of global variables), postorder (node ids, root last).
    """
    rng = np.random.default_rng(seed)
    parent, children, depth = [-1], [[]], [0]
    frontier = [0]
    for d, f in enumerate(fanout):
        nxt = []
        for q in frontier:
            for _ in range(f):
                parent.append(q)
                children.append([])
                depth.append(d + 1)
                children[q].append(len(parent) - 1)
                nxt.append(len(parent) - 1)
        frontier = nxt
    nodes = len(parent)
    size = [root_own] + [int(rng.integers(own_lo, own_hi + 1)) for _ in range(1, nodes)]
    post = []

    def visit(q):
        for ch in children[q]:
            visit(ch)
        post.append(q)

    visit(0)
    own, start = [None] * nodes, 0
    for q in post:
        own[q] = np.arange(start, start + size[q])
        start += size[q]
    N = start
    bound = [np.zeros(0, dtype=np.int64) for _ in range(nodes)]
    for q in range(1, nodes):           # breadth first: a parent before its children
        pool = np.concatenate([own[parent[q]], bound[parent[q]]])
        k = max(1, int(round(bound_frac * pool.size)))
        bound[q] = np.sort(rng.choice(pool, k, replace=False))
    A = np.zeros((N, N))
    for q in post:
        o, b = own[q], bound[q]
        G = rng.standard_normal((o.size, o.size))
        B = np.tril(G) + np.tril(G, -1).T
        mask = rng.random(o.size) < small_prob
        B[mask, mask] *= small_scale
        A[np.ix_(o, o)] = B
        if b.size:
            E = bound_scale * rng.standard_normal((b.size, o.size))
            A[np.ix_(b, o)] = E
            A[np.ix_(o, b)] = E.T
    return {"A": A, "parent": parent, "children": children, "own": own, "bound": bound,
            "postorder": post}
