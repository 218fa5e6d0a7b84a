"""Helpers for the GPU parity tests: run the HIP path through the C
interface and bring results back as numpy arrays."""

import numpy as np
import torch

from paper_1305_2353_amd import ctp

# Factors and Schur complement: relative agreement with the oracle,
# normwise per block (max |diff| / max(1, max |ref|)).
FP64_TOL = 1e-12


def schur_factors(ref, p):
    """L21 (eliminated columns) and W = L21 D of an oracle supernode."""
    from oracle.supernode import d_blocks
    L21 = ref.out[p:, :ref.nelim]
    return L21, L21 @ d_blocks(ref.piv, ref.d, ref.nelim)


def schur_tol(L21, W, S_ref, eps=2.0 ** -52):
    """schur_row_tol's bound for a whole lower triangle compared at once
    (the largest entry bound over the triangle, normalised by max |S|)."""
    K = L21.shape[1]
    mag = np.abs(L21) @ np.abs(W).T
    return 3 * max(K, 1) * eps * float(np.tril(mag).max(initial=0.0)) / max(1.0, float(np.abs(np.tril(S_ref)).max(initial=0.0)))


def rows_rel_err(got_rows, ref_rows, rows):
    """rel_err over sampled rows of S taken together (row i compared on
    columns 0..i): max |diff| / max(1, max |S|) over every sampled entry, the
    normwise measure of a block restricted to the sample."""
    diff = max((float(np.abs(got_rows[q][:i + 1] - ref_rows[q][:i + 1]).max(initial=0.0)) for q, i in enumerate(rows)),
               default=0.0)
    mag = max((float(np.abs(ref_rows[q][:i + 1]).max(initial=0.0)) for q, i in enumerate(rows)), default=0.0)
    return diff / max(1.0, mag)


def schur_row_tol(L21, W, i, s_row, eps=2.0 ** -52):
    """Tolerance for row i of S = L21 W^T (W = L21 D) against the oracle,
    normalised like rel_err.  S(i, j) is an inner product of length nelim
    of computed rows: its rounding is bounded by nelim eps
    sum_k |L21(i, k)| |W(j, k)|, and the solve's rounding in L21(i, :) and
    in W(j, :) contributes a term of the same form each, hence three times
    that sum, maximised over the row's columns j <= i and divided by
    max(1, max |S(i, :)|)."""
    K = L21.shape[1]
    mag = np.abs(W[:i + 1]) @ np.abs(L21[i])
    return 3 * max(K, 1) * eps * float(mag.max(initial=0.0)) / max(1.0, float(np.abs(s_row).max(initial=0.0)))


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctp.load()


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    if ref.size == 0:
        return 0.0
    return float(np.abs(x - ref).max() / max(1.0, np.abs(ref).max()))


def run_supernode(A, p, method, u=0.01, small=1e-20, schur=True, lda=None, flags=0):
    """Factor + Solve (+ the whole S) of the n x p panel A on the GPU."""
    n = A.shape[0]
    a = ctp.device_panel(A, lda=lda)
    opts = ctp.ctp_default_opts(method, u=u, small=small, flags=flags)
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
    (normwise over the triangle) agree to FP64_TOL.
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
        # the FP64 bar, normwise over the triangle; the forward-error bound
        # of the arithmetic goes into the message
        bound = schur_tol(*schur_factors(ref, p), S_ref)
        for key in ("S", "S_direct"):
            err = rel_err(np.tril(g[key]), np.tril(S_ref))
            assert err <= FP64_TOL, (method, key, err, bound)
