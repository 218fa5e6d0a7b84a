"""The fused Factor + Solve + Form call and the batched tasks called one at a
time, through the C interface.

The fused call's Form is one persistent launch over the whole lower
triangle; it runs the same tile routine as ctp_schur, so its S must equal
ctp_schur's bit for bit (column-major or packed tiles), and the oracle's to
the Form tolerance.  Factor, Solve and Form of a batch called separately
must reproduce ctp_supernode_batched bit for bit."""

import numpy as np
import pytest
import torch

from gpu_helpers import FP64_TOL, assert_parity, rel_err, require_gpu, schur_factors, schur_tol
from oracle.supernode import factor_supernode, schur_rows
from workloads import batch_panel, supernode

pytestmark = pytest.mark.gpu

SC = 128


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _announce(*args):
    print("case:", *args, flush=True)


def _untile(buf, r):
    """Dense lower triangle from packed 128 x 128 tiles."""
    nt = (r + SC - 1) // SC
    out = np.zeros((r, r))
    t = 0
    for tm in range(nt):
        for tn in range(tm + 1):
            blk = buf[t * SC * SC:(t + 1) * SC * SC].reshape(SC, SC).T
            i1, j1 = min(r, (tm + 1) * SC), min(r, (tn + 1) * SC)
            out[tm * SC:i1, tn * SC:j1] = blk[:i1 - tm * SC, :j1 - tn * SC]
            t += 1
    return np.tril(out)


@pytest.mark.parametrize("method", ["relaxed", "strict", "tpp", "restricted"])
@pytest.mark.parametrize("shape", [(3000, 256), (1500, 48), (300, 200), (129, 128), (64, 64), (2049, 37)])
def test_fused_supernode_matches_steps_and_oracle(method, shape):
    from paper_1305_2353_amd import ctp
    n, p = shape
    r = n - p
    _announce("fused", method, shape)
    A = supernode(n, p, seed=5 * n + p, n_small=min(3, p))
    ref = factor_supernode(A, p, method)
    if ref.trap.fragile_steps():
        pytest.skip("near-tie decision in this draw")
    opts = ctp.ctp_default_opts(method)
    a = ctp.device_panel(A)
    work = ctp.workspace(n, p, opts)
    s = torch.full((r, r), 7.0, dtype=torch.float64, device="cuda").t() if r else None
    f = ctp.ctp_supernode(a, opts, work=work, s=s)
    torch.cuda.synchronize()
    g = {"out": a.cpu().numpy(), "perm": f["perm"].cpu().numpy(), "piv": f["piv"].cpu().numpy(),
         "d": f["d"].cpu().numpy(), "nelim": int(f["nelim"].item()), "status": int(f["status"].item())}
    assert_parity(g, ref, p, method, check_s=False)
    if r == 0:
        return
    S = s.cpu().numpy()
    # entries above the diagonal are left alone
    assert (np.triu(S, 1) == np.triu(np.full((r, r), 7.0), 1)).all()
    # the same bits as the Form call on the same workspace
    s2 = ctp.ctp_schur(a, f, 0, r, opts, work=work)
    torch.cuda.synchronize()
    assert (np.tril(S) == np.tril(s2.cpu().numpy())).all()
    # and the oracle
    S_ref = schur_rows(ref, np.arange(r))
    assert rel_err(np.tril(S), np.tril(S_ref)) <= FP64_TOL, schur_tol(*schur_factors(ref, p), S_ref)
    # packed tiles: the same values
    opts_t = ctp.ctp_default_opts(method, flags=ctp.CTP_FLAG_S_TILED)
    a2 = ctp.device_panel(A)
    work2 = ctp.workspace(n, p, opts_t)
    buf = torch.zeros(ctp.s_tiles(r) * SC * SC, dtype=torch.float64, device="cuda")
    ctp.ctp_supernode(a2, opts_t, work=work2, s=buf)
    torch.cuda.synchronize()
    assert (_untile(buf.cpu().numpy(), r) == np.tril(S)).all()
    assert torch.equal(a2, a)


@pytest.mark.parametrize("method", ["relaxed", "strict", "restricted"])
@pytest.mark.parametrize("tiled", [False, True])
def test_batched_tasks_one_at_a_time(method, tiled):
    from paper_1305_2353_amd import ctp
    _announce("batched tasks", method, tiled)
    rng = np.random.default_rng(17)
    shapes = [(700, 64), (129, 32), (2000, 200), (300, 75), (64, 16), (1000, 250), (40, 10)]
    panels = [batch_panel(n, p, rng) for n, p in shapes]
    form = [True, True, True, False, True, True, True]

    def make():
        b = ctp.Batch(shapes, ctp.ctp_default_opts(method), form=form, tiled=tiled)
        for i, P in enumerate(panels):
            b.panel_view(i).copy_(torch.as_tensor(P, device="cuda"))
        if b.S is not None:
            b.S.fill_(3.0)
        return b

    whole = make()
    whole.run()
    parts = make()
    parts.factor()
    parts.solve()
    parts.schur()
    torch.cuda.synchronize()
    assert torch.equal(whole.panels, parts.panels)
    assert torch.equal(whole.S, parts.S)
    for name in ("perm", "piv", "d", "nelim", "status"):
        assert torch.equal(getattr(whole, name), getattr(parts, name)), name
    # and each node against the oracle (decisions exact, S to its bound)
    for i, (P, (n, p)) in enumerate(zip(panels, shapes)):
        ref = factor_supernode(P, p, method)
        if ref.trap.fragile_steps():
            continue
        o = parts.outputs(i)
        assert int(o["nelim"].item()) == ref.nelim
        assert (o["perm"].cpu().numpy() == ref.perm).all()
        if form[i] and n > p:
            S = parts.s_view(i).cpu().numpy()
            S_ref = schur_rows(ref, np.arange(n - p))
            assert rel_err(np.tril(S), np.tril(S_ref)) <= FP64_TOL, (i, schur_tol(*schur_factors(ref, p), S_ref))
