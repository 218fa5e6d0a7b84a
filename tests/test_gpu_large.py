"""GPU path at the full benchmark size (n = 100000, p = 512), in the launch
configuration the benchmark times (one factor, one solve, Form in 4096-row
blocks).

Strict and relaxed: the oracle computes the whole Factor + Solve and four
whole row blocks of S (the first, every eighth and the last); the compressed
matrix, the decisions and the A11 block are compared bit for bit, L21, the
delayed columns and each S block normwise against 1e-12.

Threshold partial pivoting: the oracle needs minutes on this panel, so its
result was stored by tests/golden/make_tpp_full.py (decisions and D exactly,
SHA-256 of the output panel, sampled rows); the GPU's panel must hash to the
same bytes.
"""

import hashlib
import json
import os

import numpy as np
import pytest
import torch

from gpu_helpers import FP64_TOL, rel_err, require_gpu, schur_tol
from oracle.supernode import compress_relaxed, compress_strict, d_blocks, factor_supernode, schur_block
from workloads import large_supernode

pytestmark = pytest.mark.gpu

BLOCK = 4096
HERE = os.path.dirname(os.path.abspath(__file__))


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
    del out

    # S: blocks 0, 8, 16 and the last of the 25 row blocks, launched as the
    # benchmark launches them (from the W the solve left in the workspace),
    # each compared whole, normwise: max |diff| / max(1, max |S block|).
    L21 = ref.out[p:, :ref.nelim]
    W = L21 @ d_blocks(ref.piv, ref.d, ref.nelim)
    S = torch.empty((r, BLOCK), dtype=torch.float64, device=a.device).t()
    nblk = -(-r // BLOCK)
    worst = 0.0
    for b in (0, 8, 16, nblk - 1):
        row0 = b * BLOCK
        nr = min(BLOCK, r - row0)
        ctp.ctp_schur(a, f, row0, nr, opts, s=S[:nr, :row0 + nr], work=work)
        torch.cuda.synchronize()
        got = np.tril(S[:nr, :row0 + nr].cpu().numpy(), row0)
        S_ref = schur_block(ref, row0, nr)
        err = rel_err(got, S_ref)
        # the forward-error bound of the arithmetic, as a diagnostic
        bound = schur_tol(L21[row0:row0 + nr], W[:row0 + nr], S_ref)
        print(f"S block {b}: normwise error {err:.2e} (forward-error bound {bound:.2e})", flush=True)
        worst = max(worst, err)
        del got, S_ref
    assert worst <= FP64_TOL, worst


def _hashes(out, p):
    low = np.ascontiguousarray(np.tril(out[:p]), dtype=np.float64)
    a21 = np.ascontiguousarray(out[p:], dtype=np.float64)
    return hashlib.sha256(low.tobytes()).hexdigest(), hashlib.sha256(a21.tobytes()).hexdigest()


def test_full_size_tpp(panel):
    from paper_1305_2353_amd import ctp
    with open(os.path.join(HERE, "golden", "tpp_n100000_p512.json")) as fh:
        gold = json.load(fh)
    A = panel
    n, p = A.shape
    assert (n, p) == (gold["n"], gold["p"]) and gold["fragile_steps"] == 0
    print("case: full size tpp", n, p, flush=True)
    a = ctp.device_panel(A)
    opts = ctp.ctp_default_opts("tpp")
    work = ctp.workspace(n, p, opts)
    f = ctp.ctp_factor_supernode(a, opts, work=work)
    ctp.ctp_solve_supernode(a, f, opts, work=work)
    torch.cuda.synchronize()
    assert int(f["nelim"].item()) == gold["nelim"]
    assert int(f["status"].item()) == gold["status"]
    assert (f["perm"].cpu().numpy() == np.array(gold["perm"])).all()
    assert (f["piv"].cpu().numpy() == np.array(gold["piv"])).all()
    assert (f["d"].cpu().numpy() == np.array([float.fromhex(x) for x in gold["d"]])).all()
    out = a.cpu().numpy()
    rows = np.array(gold["rows"])
    want = np.array([[float.fromhex(x) for x in row] for row in gold["row_values"]])
    assert (out[p + rows] == want).all(), np.abs(out[p + rows] - want).max()
    h11, h21 = _hashes(out, p)
    assert h11 == gold["sha256_a11_lower"]
    assert h21 == gold["sha256_a21"]
