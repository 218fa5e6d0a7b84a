"""Scatter task on the GPU: ctp_extend_add and ctp_extend_add_batched
against the oracle's extend-add (oracle/multifrontal.py), through the C
interface.

Inputs are seeded random child panels, boundary blocks, permutations,
nelim and injective maps; the parent front starts from random values.  The
expected parent is the oracle's contribution_block scattered by its
extend_add into the same starting values: every parent entry gets at most
one add per child in both, so the comparison is bit for bit, entries the
child does not touch included.
"""

from types import SimpleNamespace

import numpy as np
import pytest
import torch

from gpu_helpers import require_gpu
from oracle.multifrontal import contribution_block, extend_add

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _announce(*args):
    print("case:", *args, flush=True)


def _child(rng, n, p, nelim, np_):
    panel = rng.standard_normal((n, p))
    S = rng.standard_normal((n - p, n - p))
    S = np.tril(S) + np.tril(S, -1).T
    perm = rng.permutation(p).astype(np.int32)
    vmap = rng.choice(np_, n, replace=False).astype(np.int32)
    return panel, S, perm, nelim, vmap


def _expected_add(Fp, child):
    panel, S, perm, nelim, vmap = child
    n, p = panel.shape
    A11 = np.tril(panel[:p, :p])
    out = panel.copy()
    out[:p, :p] = A11 + np.tril(A11, -1).T
    C = contribution_block(SimpleNamespace(out=out, nelim=nelim), S)
    pos = [int(vmap[perm[t]]) for t in range(nelim, p)] + [int(vmap[t]) for t in range(p, n)]
    extend_add(Fp, C, pos)


def _parent(rng, np_):
    F = rng.standard_normal((np_, np_))
    return np.tril(F) + np.tril(F, -1).T


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _colmajor(x):
    """Column-major device copy of a 2-D array (stride(0) == 1)."""
    return _dev(np.asarray(x).T).t()


def _gpu_parent(Fp, pp):
    f = _colmajor(Fp[:, :pp])
    f22 = _colmajor(Fp[pp:, pp:]) if pp < Fp.shape[0] else None
    return f, f22


def _lower_parent(f, f22, pp):
    """The parent's lower triangle as the GPU holds it (np x np, upper
    triangle zero)."""
    F = np.zeros((f.shape[0], f.shape[0]))
    F[:, :pp] = f.cpu().numpy()
    if f22 is not None:
        F[pp:, pp:] = f22.cpu().numpy()
    return np.tril(F)


CASES = [
    # (n, p, nelim, np, pp)
    (300, 80, 50, 500, 200),
    (129, 64, 0, 300, 64),       # every panel column delayed
    (200, 40, 40, 260, 100),     # nothing delayed: the boundary block only
    (70, 70, 30, 150, 150),      # n == p (no S); parent without a trailing block
    (65, 1, 0, 65, 1),
    (1, 1, 0, 1, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_extend_add_matches_oracle(case):
    from paper_1305_2353_amd import ctp
    n, p, nelim, np_, pp = case
    _announce("extend_add", case)
    rng = np.random.default_rng(n + 7 * p + nelim)
    Fp = _parent(rng, np_)
    children = [_child(rng, n, p, nelim, np_), _child(rng, n, p, max(nelim - 1, 0), np_)]
    f, f22 = _gpu_parent(Fp, pp)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for ch in children:
        panel, S, perm, ne, vmap = ch
        a = _colmajor(panel)
        s = _colmajor(S) if n > p else None
        ctp.ctp_extend_add(a, s, _dev(perm, torch.int32), _dev([ne], torch.int32), _dev(vmap, torch.int32), f, f22,
                           status)
        _expected_add(Fp, ch)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(_lower_parent(f, f22, pp), np.tril(Fp))


def test_extend_add_bad_map_is_flagged_and_skipped():
    from paper_1305_2353_amd import ctp
    _announce("extend_add bad map")
    rng = np.random.default_rng(3)
    n, p, nelim, np_, pp = 60, 20, 10, 90, 30
    Fp = _parent(rng, np_)
    panel, S, perm, ne, vmap = _child(rng, n, p, nelim, np_)
    bad = vmap.copy()
    bad[p + 5] = np_ + 3           # boundary row 5 of the child points past the parent
    f, f22 = _gpu_parent(Fp, pp)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctp.ctp_extend_add(_colmajor(panel), _colmajor(S), _dev(perm, torch.int32), _dev([ne], torch.int32),
                       _dev(bad, torch.int32), f, f22, status)
    torch.cuda.synchronize()
    assert int(status.item()) & ctp.CTP_STATUS_BAD_MAP
    # the expected parent: the same scatter without the entries of that row
    keep = [t for t in range(ne, n) if t != p + 5]
    A11 = np.tril(panel[:p, :p])
    out = panel.copy()
    out[:p, :p] = A11 + np.tril(A11, -1).T
    C = contribution_block(SimpleNamespace(out=out, nelim=ne), S)
    rows = [t - ne for t in keep]
    pos = [int(vmap[perm[t]]) if t < p else int(vmap[t]) for t in keep]
    extend_add(Fp, C[np.ix_(rows, rows)], pos)
    assert np.array_equal(_lower_parent(f, f22, pp), np.tril(Fp))


def test_extend_add_batched_rounds():
    """Five children into two parents: rounds of at most one child per
    parent, each round one batched launch, in stream order."""
    from paper_1305_2353_amd import ctp
    _announce("extend_add batched")
    rng = np.random.default_rng(11)
    parents = [(400, 150), (220, 220)]             # (np, pp)
    kids = [(0, 300, 60, 20), (1, 120, 30, 30), (0, 90, 90, 45), (0, 257, 128, 0), (1, 64, 16, 8)]
    Fps = [_parent(rng, np_) for np_, _ in parents]
    children = [_child(rng, n, p, ne, parents[par][0]) for par, n, p, ne in kids]
    # device buffers: child panels, S, perm, nelim, maps; parent panels, trailing blocks
    a_off, s_off, o_off, m_off, offs = 0, 0, 0, 0, []
    for (par, n, p, ne), ch in zip(kids, children):
        offs.append((a_off, s_off if n > p else -1, o_off, m_off))
        a_off += n * p
        s_off += (n - p) * (n - p)
        o_off += p
        m_off += n
    panels = np.zeros(a_off)
    Sbuf = np.zeros(max(s_off, 1))
    perms = np.zeros(o_off, dtype=np.int32)
    maps = np.zeros(m_off, dtype=np.int32)
    nelims = np.array([ne for _, _, _, ne in kids], dtype=np.int32)
    for (par, n, p, ne), ch, (ao, so, oo, mo) in zip(kids, children, offs):
        panel, S, perm, _, vmap = ch
        panels[ao:ao + n * p] = panel.T.ravel()
        if so >= 0:
            Sbuf[so:so + (n - p) ** 2] = S.T.ravel()
        perms[oo:oo + p] = perm
        maps[mo:mo + n] = vmap
    f_offs, g_offs, fbuf, gbuf = [], [], [], []
    fo = go = 0
    for (np_, pp), Fp in zip(parents, Fps):
        f_offs.append(fo)
        g_offs.append(go if pp < np_ else -1)
        fbuf.append(Fp[:, :pp].T.ravel())
        fo += np_ * pp
        if pp < np_:
            gbuf.append(Fp[pp:, pp:].T.ravel())
            go += (np_ - pp) ** 2
    d_panels, d_S = _dev(panels), _dev(Sbuf)
    d_perm, d_map, d_nelim = _dev(perms, torch.int32), _dev(maps, torch.int32), _dev(nelims, torch.int32)
    d_f, d_g = _dev(np.concatenate(fbuf)), _dev(np.concatenate(gbuf) if gbuf else np.zeros(1))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    # rounds: the k-th child of each parent
    order = {0: [0, 2, 3], 1: [1, 4]}
    for rnd in range(3):
        ids = [order[par][rnd] for par in order if rnd < len(order[par])]
        tasks = (ctp.CtpScatterTask * len(ids))()
        for t, k in zip(tasks, ids):
            par, n, p, ne = kids[k]
            np_, pp = parents[par]
            ao, so, oo, mo = offs[k]
            t.n, t.p, t.lda, t.lds = n, p, n, max(n - p, 1)
            t.np, t.pp, t.ldf, t.ld22 = np_, pp, np_, max(np_ - pp, 1)
            t.node, t.a_off, t.s_off, t.out_off, t.map_off = k, ao, so, oo, mo
            t.f_off, t.f22_off = f_offs[par], g_offs[par]
        tiles = ctp.ctp_scatter_plan(tasks)
        ctp.ctp_extend_add_batched(ctp.to_device_struct(tasks), len(ids), tiles, d_panels, d_S, d_perm, d_nelim,
                                   d_map, d_f, d_g, status)
        for k in ids:
            _expected_add(Fps[kids[k][0]], children[k])
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    fh, gh = d_f.cpu().numpy(), d_g.cpu().numpy()
    for (np_, pp), Fp, fo_, go_ in zip(parents, Fps, f_offs, g_offs):
        F = np.zeros((np_, np_))
        F[:, :pp] = fh[fo_:fo_ + np_ * pp].reshape(pp, np_).T
        if go_ >= 0:
            F[pp:, pp:] = gh[go_:go_ + (np_ - pp) ** 2].reshape(np_ - pp, np_ - pp).T
        assert np.array_equal(np.tril(F), np.tril(Fp))
