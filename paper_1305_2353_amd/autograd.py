"""torch.autograd.Function for x = A^-1 b with A symmetric indefinite,
factorized by the dense driver (ctp_ldlt_dense, compressed pivoting per
panel) and differentiated with the stored factors, pivots frozen:

    forward:   P A P^T = L D L^T,   x = A^-1 b
    backward:  bbar = A^-1 xbar,    Abar = -(bbar x^T + x bbar^T) / 2

(ctp_ldlt_adjoint).  Abar is the gradient for symmetric perturbations of A
(the factorization reads only its lower triangle): the directional
derivative along a symmetric E is <Abar, E>.  Every step runs in the HIP
library; this module only arranges tensors and keeps the factors between
forward and backward.
"""

import torch

from . import ctp


def _colmajor(t):
    """Column-major float64 copy of a 2-D CUDA tensor."""
    return t.t().contiguous().t() if t.stride(0) != 1 or t.dim() != 2 else t.clone()


class LDLTSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, b, pw=256, method="relaxed"):
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("A must be N x N")
        one = b.dim() == 1
        B = b.reshape(b.shape[0], -1)
        N, nrhs = B.shape
        pw = min(pw, max(N, 1))
        opts = ctp.ctp_default_opts(method)
        a = _colmajor(A.detach().to(torch.float64))
        work = ctp.dense_workspace(N, pw, opts, nrhs, device=A.device)
        f = ctp.ctp_ldlt_dense(a, pw, opts, work)
        x = _colmajor(B.detach().to(torch.float64))
        ctp.ctp_ldlt_solve(a, f, x, opts, work)
        ctx.state = (a, f, x, opts, work, one)
        return x[:, 0].clone() if one else x.clone()

    @staticmethod
    def backward(ctx, gx):
        a, f, x, opts, work, one = ctx.state
        xb = _colmajor(gx.reshape(x.shape[0], -1).to(torch.float64))
        bbar, abar = ctp.ctp_ldlt_adjoint(a, f, x, xb, opts, work)
        gb = bbar[:, 0].clone() if one else bbar.clone()
        return abar.contiguous(), gb, None, None


class LDLTSolveBatched(torch.autograd.Function):
    """The same for a batch of systems (S, N, N): every panel step runs for
    all systems at once (ctp_ldlt_dense_batched), and the solves and
    adjoints are batched launches."""

    @staticmethod
    def forward(ctx, A, b, pw=256, method="relaxed"):
        if A.dim() != 3 or A.shape[1] != A.shape[2]:
            raise ValueError("A must be S x N x N")
        one = b.dim() == 2
        B = b.reshape(b.shape[0], b.shape[1], -1)
        S, N, nrhs = B.shape
        pw = min(pw, max(N, 1))
        opts = ctp.ctp_default_opts(method)
        a = ctp.batch_colmajor(A)
        work = ctp.dense_batched_workspace(S, N, pw, opts, device=A.device)
        f = ctp.ctp_ldlt_dense_batched(a, pw, opts, work)
        x = ctp.batch_colmajor(B)
        ctp.ctp_ldlt_solve_batched(a, f, x, opts, work)
        ctx.state = (a, f, x, opts, work, one)
        return x[:, :, 0].clone() if one else x.clone()

    @staticmethod
    def backward(ctx, gx):
        a, f, x, opts, work, one = ctx.state
        xb = ctp.batch_colmajor(gx.reshape(x.shape[0], x.shape[1], -1))
        bbar, abar = ctp.ctp_ldlt_adjoint_batched(a, f, x, xb, opts, work)
        gb = bbar[:, :, 0].clone() if one else bbar.clone()
        return abar.contiguous(), gb, None, None


def ldlt_solve(A, b, pw=256, method="relaxed"):
    """x = A^-1 b, differentiable in A (symmetric directions) and b.
    A: (N, N) or a batch (S, N, N); b: (N,), (N, k) or the matching batch
    ((S, N) or (S, N, k)).  A batch is factorized, solved and differentiated
    with batched launches (strict, relaxed or restricted rule)."""
    if A.dim() == 3:
        return LDLTSolveBatched.apply(A, b, pw, method)
    return LDLTSolve.apply(A, b, pw, method)
