"""Helpers for the GPU parity tests: run the HIP path through the C
interface and bring results back as numpy arrays."""

import numpy as np
import torch

from paper_1305_2353_amd import ctp

# Factors and Schur complement: relative agreement with the oracle,
# normwise per block (max |diff| / max(1, max |ref|)).
FP64_TOL = 1e-12


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctp.load()


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    if ref.size == 0:
        return 0.0
    return float(np.abs(x - ref).max() / max(1.0, np.abs(ref).max()))


def run_supernode(A, p, method, u=0.01, small=1e-20, schur=True, lda=None):
    """Factor + Solve (+ the whole S) of the n x p panel A on the GPU."""
    n = A.shape[0]
    a = ctp.device_panel(A, lda=lda)
    opts = ctp.ctp_default_opts(method, u=u, small=small)
    work = ctp.workspace(n, p, opts)
    f = ctp.ctp_supernode(a, opts, work=work)
    s = s_direct = None
    if schur and n > p:
        # from the W = L21 D that the solve left in the workspace ...
        s = ctp.ctp_schur(a, f, 0, n - p, opts, work=work)
        # ... and with W formed inside the Form kernel
        s_direct = ctp.ctp_schur(a, f, 0, n - p, opts)
    torch.cuda.synchronize()
    res = {
        "out": a.cpu().numpy(),
        "perm": f["perm"].cpu().numpy().astype(np.int64),
        "piv": f["piv"].cpu().numpy().astype(np.int64),
        "d": f["d"].cpu().numpy(),
        "nelim": int(f["nelim"].item()),
        "status": int(f["status"].item()),
    }
    if s is not None:
        res["S"] = s.cpu().numpy()
        res["S_direct"] = s_direct.cpu().numpy()
    return res


def assert_parity(g, ref, p, method, check_s=True):
    """GPU result g against the oracle's SupernodeFactors ref.

    Decisions (perm, piv, nelim) and the pivot-search outputs (D and the
    A11 rows of the panel) must match exactly: both sides apply the same
    IEEE operations in the same order.  L21, the delayed A21 columns and S
    agree to FP64_TOL.
    """
    from oracle.supernode import schur_rows
    assert g["nelim"] == ref.nelim, (method, g["nelim"], ref.nelim)
    assert (g["perm"] == ref.perm).all(), method
    assert (g["piv"] == ref.piv).all(), method
    assert (g["d"] == ref.d).all(), method
    assert (np.tril(g["out"][:p]) == np.tril(ref.out[:p])).all(), method
    n = ref.out.shape[0]
    if method == "tpp":
        # Listing 1 updates A21 with the same operations on both sides.
        assert (g["out"][p:] == ref.out[p:]).all(), method
    else:
        assert rel_err(g["out"][p:, :ref.nelim], ref.out[p:, :ref.nelim]) <= FP64_TOL, method
        assert rel_err(g["out"][p:, ref.nelim:], ref.out[p:, ref.nelim:]) <= FP64_TOL, method
    if check_s and n > p:
        S_ref = schur_rows(ref, np.arange(n - p))
        assert rel_err(np.tril(g["S"]), np.tril(S_ref)) <= FP64_TOL, method
        assert rel_err(np.tril(g["S_direct"]), np.tril(S_ref)) <= FP64_TOL, method
