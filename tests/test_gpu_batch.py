"""Batched supernodes (ctp_supernode_batched): every node against the oracle
(decisions and A11 values bit for bit, L21 and S to the FP64 tolerance),
nodes without a Form, and replays of the batch captured in a HIP graph
checked against the eager result."""

import numpy as np
import pytest
import torch

from gpu_helpers import FP64_TOL, rel_err, require_gpu, schur_factors, schur_tol
from oracle.supernode import factor_supernode, schur_rows
from workloads import batch_panel, batch_shapes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _make(count, seed, n_hi=2000, method="relaxed", form=True, tile=0, tiled=False):
    from paper_1305_2353_amd import ctp
    ns, ps = batch_shapes(count, seed=seed, n_hi=n_hi)
    rng = np.random.default_rng(seed + 1)
    panels = [batch_panel(int(n), int(p), rng) for n, p in zip(ns, ps)]
    opts = ctp.ctp_default_opts(method)
    opts.tile = tile
    b = ctp.Batch(list(zip(ns, ps)), opts, form=form, tiled=tiled)
    for i, A in enumerate(panels):
        b.panel_view(i).copy_(torch.from_numpy(A).to("cuda"))
    return b, panels


def _check_node(b, i, A, method, check_s=True):
    n, p = A.shape
    ref = factor_supernode(A, p, method)
    if ref.trap.fragile_steps():
        return False
    f = b.outputs(i)
    assert int(f["nelim"].item()) == ref.nelim, i
    assert (f["perm"].cpu().numpy() == ref.perm).all(), i
    assert (f["piv"].cpu().numpy() == ref.piv).all(), i
    assert (f["d"].cpu().numpy() == ref.d).all(), i
    out = b.panel_view(i).cpu().numpy()
    assert (np.tril(out[:p]) == np.tril(ref.out[:p])).all(), i
    assert rel_err(out[p:], ref.out[p:]) <= FP64_TOL, i
    S = b.s_view(i)
    if check_s and S is not None and n > p:
        S_ref = schur_rows(ref, np.arange(n - p))
        assert rel_err(np.tril(S.cpu().numpy()), np.tril(S_ref)) <= FP64_TOL, (i, schur_tol(*schur_factors(ref, p), S_ref))
    return True


@pytest.mark.parametrize("method", ["relaxed", "strict", "restricted"])
def test_batch_matches_oracle(method):
    print("case: batch", method, flush=True)
    b, panels = _make(24, seed=3, method=method)
    b.run()
    torch.cuda.synchronize()
    checked = sum(_check_node(b, i, A, method) for i, A in enumerate(panels))
    assert checked >= 20


def test_batch_nodes_without_form():
    print("case: batch partial form", flush=True)
    from paper_1305_2353_amd import ctp
    ns, ps = batch_shapes(12, seed=8, n_hi=1500)
    rng = np.random.default_rng(9)
    panels = [batch_panel(int(n), int(p), rng) for n, p in zip(ns, ps)]
    form = [i % 3 != 1 for i in range(12)]
    b = ctp.Batch(list(zip(ns, ps)), ctp.ctp_default_opts("relaxed"), form=form)
    for i, A in enumerate(panels):
        b.panel_view(i).copy_(torch.from_numpy(A).to("cuda"))
    b.run()
    torch.cuda.synchronize()
    for i, A in enumerate(panels):
        assert (b.s_view(i) is None) == (not form[i])
        _check_node(b, i, A, "relaxed")


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("tiled", [False, True])
def test_batch_form_schedules_agree(tile, tiled):
    print("case: batch tile", tile, tiled, flush=True)
    b, panels = _make(10, seed=21, tile=tile, tiled=tiled)
    b.run()
    torch.cuda.synchronize()
    for i, A in enumerate(panels):
        _check_node(b, i, A, "relaxed")


def test_batch_graph_replays_match_eager():
    """The batch (with the restore of the pristine panels) captured once in
    a HIP graph and replayed several times, with eager work and
    synchronizations in between; every replay equals the eager run."""
    print("case: batch graph", flush=True)
    b, panels = _make(16, seed=31)
    pristine = b.panels.clone()
    b.S.zero_()          # the Form writes lower triangles only
    b.run()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in (("panels", b.panels), ("S", b.S), ("perm", b.perm), ("piv", b.piv),
                                      ("d", b.d), ("nelim", b.nelim))}
    b.panels.copy_(pristine)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.panels.copy_(pristine)
            b.run()
    torch.cuda.synchronize()
    for rep in range(3):
        b.S.zero_()
        b.perm.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in ref.items():
            assert torch.equal(getattr(b, k), v), (rep, k)
