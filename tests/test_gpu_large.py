"""GPU path at the full benchmark size (n = 100000, p = 512), in the launch
configuration the benchmark times (one factor, one solve, Form in 4096-row
blocks).  The oracle computes the whole Factor + Solve and sampled rows of
S; the compressed matrix is compared bit for bit."""

import numpy as np
import pytest
import torch

from gpu_helpers import FP64_TOL, rel_err, require_gpu, schur_row_tol
from oracle.supernode import compress_relaxed, compress_strict, d_blocks, factor_supernode, schur_rows
from workloads import large_supernode

pytestmark = pytest.mark.gpu

BLOCK = 4096


@pytest.fixture(scope="module")
def panel():
    require_gpu()
    return large_supernode(0)


@pytest.mark.parametrize("method", ["relaxed", "strict"])
def test_full_size_supernode(panel, method):
    from paper_1305_2353_amd import ctp
    A = panel
    n, p = A.shape
    r = n - p
    print("case: full size", method, n, p, flush=True)
    ref = factor_supernode(A, p, method)
    assert not ref.trap.fragile_steps()

    a = ctp.device_panel(A)
    C, crow, _ = ctp.ctp_compress(a, p, method)
    opts = ctp.ctp_default_opts(method)
    work = ctp.workspace(n, p, opts)
    f = ctp.ctp_factor_supernode(a, opts, work=work)
    ctp.ctp_solve_supernode(a, f, opts, work=work)
    torch.cuda.synchronize()

    # compression: exact
    C_ref = compress_strict(A[p:]) if method == "strict" else compress_relaxed(A[p:])[0]
    assert (C.cpu().numpy() == C_ref).all()
    # decisions and pivot-search outputs: exact
    assert int(f["nelim"].item()) == ref.nelim
    assert (f["perm"].cpu().numpy() == ref.perm).all()
    assert (f["piv"].cpu().numpy() == ref.piv).all()
    assert (f["d"].cpu().numpy() == ref.d).all()
    out = a.cpu().numpy()
    assert (np.tril(out[:p]) == np.tril(ref.out[:p])).all()
    # L21 and delayed columns
    assert rel_err(out[p:, :ref.nelim], ref.out[p:, :ref.nelim]) <= FP64_TOL
    assert rel_err(out[p:, ref.nelim:], ref.out[p:, ref.nelim:]) <= FP64_TOL

    # S: three of the 25 row blocks, launched as the benchmark launches them
    # (from the W the solve left in the workspace), checked on sampled rows
    # (first, last and random rows of the block).
    L21 = ref.out[p:, :ref.nelim]
    W = L21 @ d_blocks(ref.piv, ref.d, ref.nelim)
    S = torch.empty((r, BLOCK), dtype=torch.float64, device=a.device).t()
    rng = np.random.default_rng(5)
    nblk = -(-r // BLOCK)
    for b in (0, nblk // 2, nblk - 1):
        row0 = b * BLOCK
        nr = min(BLOCK, r - row0)
        ctp.ctp_schur(a, f, row0, nr, opts, s=S[:nr, :row0 + nr], work=work)
        torch.cuda.synchronize()
        loc = np.unique(np.concatenate([[0, nr - 1], rng.integers(0, nr, 6)]))
        rows = row0 + loc
        S_ref = schur_rows(ref, rows)
        got = S[torch.as_tensor(loc, device=a.device), :rows[-1] + 1].cpu().numpy()
        for q, i in enumerate(rows):
            assert rel_err(got[q, :i + 1], S_ref[q, :i + 1]) <= schur_row_tol(L21, W, i, S_ref[q, :i + 1]), (b, i)
