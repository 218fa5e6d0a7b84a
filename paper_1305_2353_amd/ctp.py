"""Python binding of libctp.so (ctypes): the C entry points under the same
names, with torch tensors for device memory and the current torch stream.

Only argument marshalling happens here; every step of the computation runs
in the HIP library.  If the library has not been built, or there is no GPU,
the calls raise -- there is no CPU fallback.

Panels are column-major, as in the C interface: a float64 CUDA tensor `a`
of shape (n, p) with a.stride(0) == 1 and lda = a.stride(1) >= n (see
`device_panel`).  Integer outputs are int32 tensors.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctp.so")

CTP_TPP, CTP_STRICT, CTP_RELAXED, CTP_RESTRICTED = 0, 1, 2, 3
METHOD_IDS = {"tpp": CTP_TPP, "strict": CTP_STRICT, "relaxed": CTP_RELAXED,
              "restricted": CTP_RESTRICTED}
CTP_PIV_ZERO, CTP_PIV_1X1, CTP_PIV_2X2_FIRST, CTP_PIV_2X2_SECOND, CTP_PIV_DELAYED = 0, 1, 2, -2, -1
CTP_STATUS_ZERO_PIVOT, CTP_STATUS_NONFINITE, CTP_STATUS_RELAXED_RESCAN = 1, 2, 4
CTP_STATUS_ROOT_FALLBACK = 8
CTP_STATUS_BAD_MAP = 16
CTP_FLAG_ROOT = 1
CTP_FLAG_ONE_WG = 2
CTP_FLAG_S_TILED = 4
SC_TILE = 128
CTP_FLAG_S_SUBTRACT = 8
CTP_ERR_PANEL_TOO_WIDE = -900
CTP_ERR_SCRATCH_TOO_SMALL = -901
CTP_NOALLOC_SCRATCH_BYTES = 64 << 20
PREC_IDS = {"fp64": 0, "fp32": 1, "bf16": 2}
CTP_MAX_P = 512

# Every symbol declared in include/ctp.h.
EXPORTED = ("ctp_default_opts", "ctp_version", "ctp_workspace_size", "ctp_compress",
            "ctp_factor_supernode", "ctp_solve_supernode", "ctp_supernode", "ctp_supernode_noalloc",
            "ctp_schur", "ctp_dense_workspace_size", "ctp_ldlt_dense", "ctp_ldlt_solve", "ctp_ldlt_refine",
            "ctp_ldlt_adjoint", "ctp_batch_plan", "ctp_supernode_batched", "ctp_factor_supernode_batched",
            "ctp_solve_supernode_batched", "ctp_schur_batched",
            "ctp_dense_batched_workspace_size", "ctp_ldlt_dense_batched", "ctp_ldlt_solve_batched",
            "ctp_ldlt_adjoint_batched", "ctp_extend_add", "ctp_scatter_plan", "ctp_extend_add_batched")


class CtpOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("u", ctypes.c_double), ("small", ctypes.c_double),
                ("prec", ctypes.c_int), ("tile", ctypes.c_int), ("flags", ctypes.c_uint)]


class CtpNode(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("lda", ctypes.c_int), ("lds", ctypes.c_int),
                ("a_off", ctypes.c_longlong), ("s_off", ctypes.c_longlong), ("out_off", ctypes.c_longlong),
                ("work_off", ctypes.c_longlong), ("tile_off", ctypes.c_longlong)]


class CtpBatchInfo(ctypes.Structure):
    _fields_ = [("work_bytes", ctypes.c_size_t), ("tiles", ctypes.c_longlong), ("count", ctypes.c_int),
                ("max_p", ctypes.c_int), ("max_r", ctypes.c_int), ("max_chunks", ctypes.c_int),
                ("form_workgroups", ctypes.c_int)]


class CtpScatterTask(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("lda", ctypes.c_int), ("lds", ctypes.c_int),
                ("np", ctypes.c_int), ("pp", ctypes.c_int), ("ldf", ctypes.c_int), ("ld22", ctypes.c_int),
                ("node", ctypes.c_int), ("a_off", ctypes.c_longlong), ("s_off", ctypes.c_longlong),
                ("out_off", ctypes.c_longlong), ("map_off", ctypes.c_longlong), ("f_off", ctypes.c_longlong),
                ("f22_off", ctypes.c_longlong), ("tile_off", ctypes.c_longlong)]


class CtpError(RuntimeError):
    pass


_lib = None


def load(path=LIB_PATH):
    """Load libctp.so and declare the C signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CtpError(f"{path} is missing: build it with `python -m paper_1305_2353_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, D, SZ, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_longlong
    OPT = ctypes.POINTER(CtpOpts)
    sig = {
        "ctp_default_opts": (None, [OPT]),
        "ctp_version": (ctypes.c_char_p, []),
        "ctp_workspace_size": (I, [I, I, OPT, ctypes.POINTER(SZ)]),
        "ctp_compress": (I, [I, I, P, I, I, P, I, P, P, P, SZ, P]),
        "ctp_factor_supernode": (I, [I, I, P, I, OPT, P, P, P, P, P, P, SZ, P]),
        "ctp_solve_supernode": (I, [I, I, P, I, P, P, P, P, OPT, P, SZ, P]),
        "ctp_supernode": (I, [I, I, P, I, OPT, P, P, P, P, P, P, I, P, SZ, P]),
        "ctp_supernode_noalloc": (I, [I, I, P, I, OPT, P, P, P, P, P, P, I, P]),
        "ctp_schur": (I, [I, I, P, I, P, P, P, I, I, P, I, OPT, P, SZ, P]),
        "ctp_dense_workspace_size": (I, [I, I, OPT, I, ctypes.POINTER(SZ)]),
        "ctp_ldlt_dense": (I, [I, I, P, I, OPT, P, P, P, P, ctypes.POINTER(I), P, SZ, P]),
        "ctp_ldlt_solve": (I, [I, I, P, I, P, P, P, P, I, OPT, I, P, SZ, P]),
        "ctp_ldlt_refine": (I, [I, I, P, I, P, I, P, P, P, P, I, P, I, OPT, I, D, I,
                                ctypes.POINTER(I), ctypes.POINTER(D), P, SZ, P]),
        "ctp_ldlt_adjoint": (I, [I, I, P, I, P, P, P, P, I, P, I, P, I, OPT, I, P, SZ, P]),
        "ctp_batch_plan": (I, [I, P, OPT, ctypes.POINTER(CtpBatchInfo)]),
        "ctp_supernode_batched": (I, [I, P, ctypes.POINTER(CtpBatchInfo), P, P, P, P, P, P, P, OPT, P, SZ, P]),
        "ctp_factor_supernode_batched": (I, [I, P, ctypes.POINTER(CtpBatchInfo), P, P, P, P, P, P, OPT, P, SZ,
                                             P]),
        "ctp_solve_supernode_batched": (I, [I, P, ctypes.POINTER(CtpBatchInfo), P, P, P, P, P, OPT, P, SZ, P]),
        "ctp_schur_batched": (I, [I, P, ctypes.POINTER(CtpBatchInfo), P, P, P, P, P, OPT, P, SZ, P]),
        "ctp_dense_batched_workspace_size": (I, [I, I, I, OPT, ctypes.POINTER(SZ)]),
        "ctp_ldlt_dense_batched": (I, [I, I, I, P, I, LL, OPT, P, P, P, P, ctypes.POINTER(I), P, SZ, P]),
        "ctp_ldlt_solve_batched": (I, [I, I, I, P, I, LL, P, P, P, P, I, LL, OPT, I, P, SZ, P]),
        "ctp_ldlt_adjoint_batched": (I, [I, I, I, P, I, LL, P, P, P, P, I, LL, P, I, LL, P, I, LL, OPT, I, P,
                                         SZ, P]),
        "ctp_extend_add": (I, [I, I, P, I, P, I, P, P, P, I, I, P, I, P, I, P, P]),
        "ctp_scatter_plan": (I, [I, P, ctypes.POINTER(LL)]),
        "ctp_extend_add_batched": (I, [I, P, LL, P, P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, name):
    if rc != 0:
        raise CtpError(f"{name} returned {rc}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _panel_args(a):
    if a.dtype != torch.float64 or not a.is_cuda or a.dim() != 2:
        raise CtpError("panel must be a 2-D float64 CUDA tensor")
    n, p = a.shape
    if a.stride(0) != 1 and not (p <= 1):
        raise CtpError("panel must be column-major (stride(0) == 1)")
    lda = a.stride(1) if p > 1 else max(n, 1)
    return n, p, max(lda, 1)


def device_panel(A, lda=None, device="cuda"):
    """Column-major float64 device copy of the n x p array A."""
    A = torch.as_tensor(A, dtype=torch.float64)
    n, p = A.shape
    lda = lda or n
    buf = torch.zeros((p, lda), dtype=torch.float64, device=device)
    buf[:, :n] = A.T.to(device)
    return buf.t()[:n, :] if lda != n else buf.t()


def ctp_default_opts(method="relaxed", u=0.01, small=1e-20, prec="fp64", flags=0):
    o = CtpOpts()
    load().ctp_default_opts(ctypes.byref(o))
    o.method = METHOD_IDS[method] if isinstance(method, str) else int(method)
    o.u = u
    o.small = small
    o.prec = PREC_IDS[prec] if isinstance(prec, str) else int(prec)
    o.flags = flags
    return o


def ctp_version():
    return load().ctp_version().decode()


def ctp_workspace_size(n, p, opts):
    out = ctypes.c_size_t(0)
    _check(load().ctp_workspace_size(n, p, ctypes.byref(opts), ctypes.byref(out)),
           "ctp_workspace_size")
    return out.value


def workspace(n, p, opts, device="cuda"):
    return torch.empty(max(ctp_workspace_size(n, p, opts), 1), dtype=torch.uint8, device=device)


def ctp_compress(a, p_cols, method, work=None):
    """Compressed matrix of A21 = a[p:, :]: returns (C, crow, status)."""
    n, p, lda = _panel_args(a)
    assert p == p_cols
    mid = METHOD_IDS[method] if isinstance(method, str) else int(method)
    opts = ctp_default_opts(mid)
    work = work if work is not None else workspace(n, p, opts, a.device)
    c = torch.empty((p, p), dtype=torch.float64, device=a.device)   # row-major (p, p) = C^T
    crow = torch.empty(max(p, 1), dtype=torch.int32, device=a.device)
    status = torch.zeros(1, dtype=torch.int32, device=a.device)
    _check(load().ctp_compress(n, p, _ptr(a), lda, mid, _ptr(c), max(p, 1), _ptr(crow), _ptr(status),
                               _ptr(work), work.numel(), _stream()), "ctp_compress")
    return c.t(), crow[:p], status


def _outputs(p, device):
    return (torch.empty(max(p, 1), dtype=torch.int32, device=device),
            torch.empty(max(p, 1), dtype=torch.int32, device=device),
            torch.empty(max(2 * p, 1), dtype=torch.float64, device=device),
            torch.zeros(1, dtype=torch.int32, device=device),
            torch.zeros(1, dtype=torch.int32, device=device))


def ctp_factor_supernode(a, opts, work=None, outs=None):
    """Factor task in place on the column-major panel a.  Returns a dict of
    device tensors perm, piv, d, nelim, status."""
    n, p, lda = _panel_args(a)
    work = work if work is not None else workspace(n, p, opts, a.device)
    perm, piv, d, nelim, status = outs if outs is not None else _outputs(p, a.device)
    _check(load().ctp_factor_supernode(n, p, _ptr(a), lda, ctypes.byref(opts), _ptr(perm), _ptr(piv),
                                       _ptr(d), _ptr(nelim), _ptr(status), _ptr(work), work.numel(),
                                       _stream()), "ctp_factor_supernode")
    return {"perm": perm[:p], "piv": piv[:p], "d": d[:2 * p], "nelim": nelim, "status": status}


def ctp_solve_supernode(a, f, opts, work=None):
    n, p, lda = _panel_args(a)
    work = work if work is not None else workspace(n, p, opts, a.device)
    _check(load().ctp_solve_supernode(n, p, _ptr(a), lda, _ptr(f["perm"]), _ptr(f["piv"]), _ptr(f["d"]),
                                      _ptr(f["nelim"]), ctypes.byref(opts), _ptr(work), work.numel(),
                                      _stream()),
           "ctp_solve_supernode")


def _s_args(s, r, opts):
    """Pointer and leading dimension of an S argument of ctp_supernode: a
    column-major (r x r) float64 tensor, or with CTP_FLAG_S_TILED a flat
    buffer of s_tiles(r) * 16384 doubles; None for no Form."""
    if s is None:
        return ctypes.c_void_p(0), max(r, 1)
    if s.dtype != torch.float64 or not s.is_cuda:
        raise CtpError("S must be a float64 CUDA tensor")
    if opts.flags & CTP_FLAG_S_TILED:
        if s.numel() < s_tiles(r) * SC_TILE * SC_TILE:
            raise CtpError("tiled S buffer too small")
        return _ptr(s), SC_TILE
    if s.dim() != 2 or tuple(s.shape) != (r, r) or (r > 1 and s.stride(0) != 1):
        raise CtpError("S must be a column-major (n-p) x (n-p) tensor")
    return _ptr(s), max(s.stride(1) if r > 1 else 1, r, 1)


def s_tiles(r):
    """Number of 128 x 128 tiles of the lower triangle of an order-r S."""
    nt = (r + SC_TILE - 1) // SC_TILE
    return nt * (nt + 1) // 2


def ctp_supernode(a, opts, work=None, outs=None, s=None):
    """Factor + Solve in place, and with s the whole lower triangle of S
    (Form) into s; returns the factor dict."""
    n, p, lda = _panel_args(a)
    work = work if work is not None else workspace(n, p, opts, a.device)
    perm, piv, d, nelim, status = outs if outs is not None else _outputs(p, a.device)
    sp, lds = _s_args(s, n - p, opts)
    _check(load().ctp_supernode(n, p, _ptr(a), lda, ctypes.byref(opts), _ptr(perm), _ptr(piv), _ptr(d),
                                _ptr(nelim), _ptr(status), sp, lds, _ptr(work), work.numel(), _stream()),
           "ctp_supernode")
    return {"perm": perm[:p], "piv": piv[:p], "d": d[:2 * p], "nelim": nelim, "status": status}


def ctp_supernode_noalloc(a, opts, outs=None, s=None):
    """ctp_supernode with the library's static device scratch instead of a
    caller workspace (no allocation inside the call)."""
    n, p, lda = _panel_args(a)
    perm, piv, d, nelim, status = outs if outs is not None else _outputs(p, a.device)
    sp, lds = _s_args(s, n - p, opts)
    _check(load().ctp_supernode_noalloc(n, p, _ptr(a), lda, ctypes.byref(opts), _ptr(perm), _ptr(piv), _ptr(d),
                                        _ptr(nelim), _ptr(status), sp, lds, _stream()), "ctp_supernode_noalloc")
    return {"perm": perm[:p], "piv": piv[:p], "d": d[:2 * p], "nelim": nelim, "status": status}


def ctp_schur(a, f, row0, nrows, opts, s=None, work=None):
    """Rows row0..row0+nrows-1 of the lower triangle of S.  s: column-major
    (nrows x (row0+nrows)) float64 CUDA tensor (allocated if None).  work:
    the workspace filled by ctp_solve_supernode / ctp_supernode for this
    panel (W = L21 D is read from it), or None to form W inside the kernel."""
    n, p, lda = _panel_args(a)
    if s is None:
        s = torch.zeros((row0 + nrows, max(nrows, 1)), dtype=torch.float64, device=a.device).t()[:nrows]
    lds = s.stride(1) if s.dim() == 2 and s.shape[1] > 1 else max(nrows, 1)
    lwork = work.numel() if work is not None else 0
    _check(load().ctp_schur(n, p, _ptr(a), lda, _ptr(f["piv"]), _ptr(f["d"]), _ptr(f["nelim"]), row0, nrows,
                            _ptr(s), lds, ctypes.byref(opts), _ptr(work), lwork, _stream()), "ctp_schur")
    return s


# ---------------------------------------------------------------------------
# dense LDL^T by supernode panels
# ---------------------------------------------------------------------------

def ctp_dense_workspace_size(N, pw, opts, nrhs_max=16):
    out = ctypes.c_size_t(0)
    _check(load().ctp_dense_workspace_size(N, pw, ctypes.byref(opts), nrhs_max, ctypes.byref(out)),
           "ctp_dense_workspace_size")
    return out.value


def dense_workspace(N, pw, opts, nrhs_max=16, device="cuda"):
    return torch.empty(max(ctp_dense_workspace_size(N, pw, opts, nrhs_max), 1), dtype=torch.uint8,
                       device=device)


def _square_args(a):
    n, m, lda = _panel_args(a)
    if n != m:
        raise CtpError("square matrix expected")
    return n, lda


def ctp_ldlt_dense(a, pw, opts, work):
    """P A P^T = L D L^T in place on the column-major N x N tensor a (lower
    triangle read).  Returns perm, piv, d, status (device) and npanels."""
    N, lda = _square_args(a)
    perm = torch.empty(max(N, 1), dtype=torch.int32, device=a.device)
    piv = torch.empty(max(N, 1), dtype=torch.int32, device=a.device)
    d = torch.zeros(max(2 * N, 1), dtype=torch.float64, device=a.device)
    status = torch.zeros(1, dtype=torch.int32, device=a.device)
    npan = ctypes.c_int(0)
    _check(load().ctp_ldlt_dense(N, pw, _ptr(a), lda, ctypes.byref(opts), _ptr(perm), _ptr(piv), _ptr(d),
                                 _ptr(status), ctypes.byref(npan), _ptr(work), work.numel(), _stream()),
           "ctp_ldlt_dense")
    return {"perm": perm[:N], "piv": piv[:N], "d": d[:2 * N], "status": status, "npanels": npan.value,
            "pw": pw}


def ctp_ldlt_solve(a, f, b, opts, work):
    """b <- A^-1 b in place (b: column-major N x nrhs float64 CUDA tensor)."""
    N, lda = _square_args(a)
    nb, nrhs, ldb = _panel_args(b)
    assert nb == N
    _check(load().ctp_ldlt_solve(N, nrhs, _ptr(a), lda, _ptr(f["perm"]), _ptr(f["piv"]), _ptr(f["d"]), _ptr(b),
                                 ldb, ctypes.byref(opts), f["pw"], _ptr(work), work.numel(), _stream()),
           "ctp_ldlt_solve")
    return b


def ctp_ldlt_refine(a0, a, f, b, opts, work, tol=1e-14, max_steps=10, x=None):
    """FP64 iterative refinement; a0 holds the original matrix (both
    triangles).  Returns (x, steps, backward-error history)."""
    N, lda = _square_args(a)
    _, lda0 = _square_args(a0)
    nb, nrhs, ldb = _panel_args(b)
    if x is None:
        x = device_panel(torch.zeros(N, nrhs, dtype=torch.float64), device=a.device)
    _, _, ldx = _panel_args(x)
    steps = ctypes.c_int(0)
    hist = (ctypes.c_double * (max_steps + 1))()
    _check(load().ctp_ldlt_refine(N, nrhs, _ptr(a0), lda0, _ptr(a), lda, _ptr(f["perm"]), _ptr(f["piv"]),
                                  _ptr(f["d"]), _ptr(b), ldb, _ptr(x), ldx, ctypes.byref(opts), f["pw"], tol,
                                  max_steps, ctypes.byref(steps), hist, _ptr(work), work.numel(), _stream()),
           "ctp_ldlt_refine")
    return x, steps.value, list(hist)[:steps.value + 1]


def ctp_ldlt_adjoint(a, f, x, xbar, opts, work, abar=None):
    """bbar = A^-1 xbar (in place of xbar) and Abar = -sym(bbar x^T) (full
    N x N, column-major), from the factors of ctp_ldlt_dense."""
    N, lda = _square_args(a)
    _, nrhs, ldx = _panel_args(x)
    _, _, ldxb = _panel_args(xbar)
    if abar is None:
        abar = torch.empty((N, N), dtype=torch.float64, device=a.device).t()
    _, ldg = _square_args(abar)
    _check(load().ctp_ldlt_adjoint(N, nrhs, _ptr(a), lda, _ptr(f["perm"]), _ptr(f["piv"]), _ptr(f["d"]), _ptr(x),
                                   ldx, _ptr(xbar), ldxb, _ptr(abar), ldg, ctypes.byref(opts), f["pw"], _ptr(work),
                                   work.numel(), _stream()), "ctp_ldlt_adjoint")
    return xbar, abar


# ---------------------------------------------------------------------------
# batches of dense systems
# ---------------------------------------------------------------------------

def batch_colmajor(t):
    """(count, N, M) float64 CUDA copy with every system column-major."""
    return t.detach().to(torch.float64).transpose(1, 2).contiguous().transpose(1, 2)


def _batch_args(t, what):
    if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 3:
        raise CtpError(f"{what} must be a 3-D float64 CUDA tensor (count, rows, cols)")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise CtpError(f"{what}: every system must be column-major (stride(1) == 1)")
    count, n, m = t.shape
    ld = t.stride(2) if m > 1 else max(n, 1)
    return count, n, m, max(ld, 1), t.stride(0)


def ctp_dense_batched_workspace_size(count, N, pw, opts):
    out = ctypes.c_size_t(0)
    _check(load().ctp_dense_batched_workspace_size(count, N, pw, ctypes.byref(opts), ctypes.byref(out)),
           "ctp_dense_batched_workspace_size")
    return out.value


def dense_batched_workspace(count, N, pw, opts, device="cuda"):
    return torch.empty(max(ctp_dense_batched_workspace_size(count, N, pw, opts), 1), dtype=torch.uint8,
                       device=device)


def ctp_ldlt_dense_batched(a, pw, opts, work):
    """P A P^T = L D L^T in place for every system of a (count, N, N), each
    column-major (lower triangles read).  Returns perm, piv (count, N), d
    (count, 2N), status (count,) on the device and the number of steps."""
    count, N, M, lda, stride = _batch_args(a, "a")
    if N != M:
        raise CtpError("square systems expected")
    dev = a.device
    perm = torch.empty((count, max(N, 1)), dtype=torch.int32, device=dev)
    piv = torch.empty((count, max(N, 1)), dtype=torch.int32, device=dev)
    d = torch.zeros((count, max(2 * N, 1)), dtype=torch.float64, device=dev)
    status = torch.zeros(max(count, 1), dtype=torch.int32, device=dev)
    nsteps = ctypes.c_int(0)
    _check(load().ctp_ldlt_dense_batched(count, N, pw, _ptr(a), lda, stride, ctypes.byref(opts), _ptr(perm),
                                         _ptr(piv), _ptr(d), _ptr(status), ctypes.byref(nsteps), _ptr(work),
                                         work.numel(), _stream()), "ctp_ldlt_dense_batched")
    return {"perm": perm[:, :N], "piv": piv[:, :N], "d": d[:, :2 * N], "status": status[:count],
            "nsteps": nsteps.value, "pw": pw, "_perm": perm, "_piv": piv, "_d": d}


def ctp_ldlt_solve_batched(a, f, b, opts, work):
    """b <- A^-1 b in place for every system (b: (count, N, nrhs), each
    column-major)."""
    count, N, _, lda, stride = _batch_args(a, "a")
    cb, nb, nrhs, ldb, bstride = _batch_args(b, "b")
    assert cb == count and nb == N
    _check(load().ctp_ldlt_solve_batched(count, N, nrhs, _ptr(a), lda, stride, _ptr(f["_perm"]), _ptr(f["_piv"]),
                                         _ptr(f["_d"]), _ptr(b), ldb, bstride, ctypes.byref(opts), f["pw"],
                                         _ptr(work), work.numel(), _stream()), "ctp_ldlt_solve_batched")
    return b


def ctp_ldlt_adjoint_batched(a, f, x, xbar, opts, work, abar=None):
    """For every system: bbar = A^-1 xbar (in place of xbar) and Abar =
    -sym(bbar x^T), returned as (count, N, N) column-major per system."""
    count, N, _, lda, stride = _batch_args(a, "a")
    _, _, nrhs, ldx, xstride = _batch_args(x, "x")
    _, _, _, ldxb, xbstride = _batch_args(xbar, "xbar")
    if abar is None:
        abar = torch.empty((count, N, N), dtype=torch.float64, device=a.device).transpose(1, 2)
    _, _, _, ldg, gstride = _batch_args(abar, "abar")
    _check(load().ctp_ldlt_adjoint_batched(count, N, nrhs, _ptr(a), lda, stride, _ptr(f["_perm"]), _ptr(f["_piv"]),
                                           _ptr(f["_d"]), _ptr(x), ldx, xstride, _ptr(xbar), ldxb, xbstride,
                                           _ptr(abar), ldg, gstride, ctypes.byref(opts), f["pw"], _ptr(work),
                                           work.numel(), _stream()), "ctp_ldlt_adjoint_batched")
    return xbar, abar


# ---------------------------------------------------------------------------
# batches of supernodes
# ---------------------------------------------------------------------------

class Batch:
    """A batch of supernodes laid out in one panel buffer (each panel
    column-major with lda = n), one S buffer (lds = n - p) and concatenated
    outputs, planned once; run() enqueues ctp_supernode_batched.

    shapes: list of (n, p).  form: which nodes get S (bool or list).
    tiled: store each S as its lower 128 x 128 tiles (CTP_FLAG_S_TILED)."""

    def __init__(self, shapes, opts, form=True, device="cuda", tiled=False):
        self.shapes = [(int(n), int(p)) for n, p in shapes]
        self.tiled = tiled
        if tiled:
            opts.flags |= CTP_FLAG_S_TILED
        self.opts = opts
        count = len(self.shapes)
        forms = [bool(form)] * count if isinstance(form, bool) else [bool(f) for f in form]
        nodes = (CtpNode * count)()
        a_off = s_off = out_off = 0
        for i, (n, p) in enumerate(self.shapes):
            r = n - p
            nd = nodes[i]
            nd.n, nd.p, nd.lda, nd.lds = n, p, n, max(r, 1)
            nd.a_off, nd.out_off = a_off, out_off
            nd.s_off = s_off if forms[i] else -1
            a_off += n * p
            out_off += p
            if forms[i]:
                if tiled:
                    nt = (r + SC_TILE - 1) // SC_TILE
                    s_off += nt * (nt + 1) // 2 * SC_TILE * SC_TILE
                else:
                    s_off += max(r, 1) * r
        self.info = CtpBatchInfo()
        _check(load().ctp_batch_plan(count, ctypes.cast(nodes, ctypes.c_void_p), ctypes.byref(opts),
                                     ctypes.byref(self.info)), "ctp_batch_plan")
        self.nodes_host = nodes
        raw = bytes(memoryview(nodes).cast("B"))
        self.nodes = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.count = count
        self.panels = torch.empty(max(a_off, 1), dtype=torch.float64, device=device)
        self.S = torch.empty(max(s_off, 1), dtype=torch.float64, device=device) if s_off else None
        self.perm = torch.empty(max(out_off, 1), dtype=torch.int32, device=device)
        self.piv = torch.empty(max(out_off, 1), dtype=torch.int32, device=device)
        self.d = torch.empty(max(2 * out_off, 1), dtype=torch.float64, device=device)
        self.nelim = torch.zeros(max(count, 1), dtype=torch.int32, device=device)
        self.status = torch.zeros(max(count, 1), dtype=torch.int32, device=device)
        self.work = torch.empty(max(self.info.work_bytes, 1), dtype=torch.uint8, device=device)

    def node(self, i):
        return self.nodes_host[i]

    def panel_view(self, i):
        nd = self.nodes_host[i]
        return self.panels[nd.a_off:nd.a_off + nd.n * nd.p].view(nd.p, nd.n).t()

    def s_view(self, i):
        """S of node i as an (r x r) tensor (tiled storage is assembled into
        a dense lower triangle; entries above the diagonal are zero there)."""
        nd = self.nodes_host[i]
        r = nd.n - nd.p
        if nd.s_off < 0 or self.S is None:
            return None
        if not self.tiled:
            return self.S[nd.s_off:nd.s_off + nd.lds * r].view(r, nd.lds).t()[:r]
        T = SC_TILE
        nt = (r + T - 1) // T
        out = torch.zeros((r, r), dtype=torch.float64, device=self.S.device)
        t = 0
        for tm in range(nt):
            for tn in range(tm + 1):
                blk = self.S[nd.s_off + t * T * T:nd.s_off + (t + 1) * T * T].view(T, T).t()
                i1, j1 = min(r, (tm + 1) * T), min(r, (tn + 1) * T)
                out[tm * T:i1, tn * T:j1] = blk[:i1 - tm * T, :j1 - tn * T]
                t += 1
        return torch.tril(out)

    def outputs(self, i):
        nd = self.nodes_host[i]
        o = nd.out_off
        return {"perm": self.perm[o:o + nd.p], "piv": self.piv[o:o + nd.p], "d": self.d[2 * o:2 * o + 2 * nd.p],
                "nelim": self.nelim[i:i + 1], "status": self.status[i:i + 1]}

    def run(self):
        _check(load().ctp_supernode_batched(self.count, _ptr(self.nodes), ctypes.byref(self.info), _ptr(self.panels),
                                            _ptr(self.S), _ptr(self.perm), _ptr(self.piv), _ptr(self.d),
                                            _ptr(self.nelim), _ptr(self.status), ctypes.byref(self.opts),
                                            _ptr(self.work), self.work.numel(), _stream()),
               "ctp_supernode_batched")

    def factor(self):
        """Factor task of every node (ctp_factor_supernode_batched)."""
        _check(load().ctp_factor_supernode_batched(self.count, _ptr(self.nodes), ctypes.byref(self.info),
                                                   _ptr(self.panels), _ptr(self.perm), _ptr(self.piv), _ptr(self.d),
                                                   _ptr(self.nelim), _ptr(self.status), ctypes.byref(self.opts),
                                                   _ptr(self.work), self.work.numel(), _stream()),
               "ctp_factor_supernode_batched")

    def solve(self):
        """Solve task of every node (ctp_solve_supernode_batched)."""
        _check(load().ctp_solve_supernode_batched(self.count, _ptr(self.nodes), ctypes.byref(self.info),
                                                  _ptr(self.panels), _ptr(self.perm), _ptr(self.piv), _ptr(self.d),
                                                  _ptr(self.nelim), ctypes.byref(self.opts), _ptr(self.work),
                                                  self.work.numel(), _stream()), "ctp_solve_supernode_batched")

    def schur(self):
        """Form task of every node with S (ctp_schur_batched)."""
        _check(load().ctp_schur_batched(self.count, _ptr(self.nodes), ctypes.byref(self.info), _ptr(self.panels),
                                        _ptr(self.piv), _ptr(self.d), _ptr(self.nelim), _ptr(self.S),
                                        ctypes.byref(self.opts), _ptr(self.work), self.work.numel(), _stream()),
               "ctp_schur_batched")


# ---------------------------------------------------------------------------
# Scatter (extend-add into the parent front)
# ---------------------------------------------------------------------------

def _colmajor(t, what):
    if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
        raise CtpError(f"{what} must be a 2-D float64 CUDA tensor")
    rows, cols = t.shape
    if cols > 1 and t.stride(0) != 1:
        raise CtpError(f"{what} must be column-major (stride(0) == 1)")
    return max(t.stride(1) if cols > 1 else rows, rows, 1)


def ctp_extend_add(a, s, perm, nelim, vmap, f, f22=None, status=None):
    """Add a factored front's contribution block into its parent front
    (ctp_extend_add).  a: the child's n x p panel after Factor + Solve; s:
    its (n-p) x (n-p) boundary block A22 - L21 D L21^T (None when n == p);
    perm, nelim: the child's factorization outputs (int32 device tensors);
    vmap: n int32 (child original local index -> parent row); f: the
    parent's np x pp panel; f22: its (np-pp) x (np-pp) trailing block (None
    when pp == np); status: optional int32 device word."""
    n, p = a.shape
    lda = _colmajor(a, "panel")
    lds = _colmajor(s, "s") if s is not None else 1
    np_, pp = f.shape
    ldf = _colmajor(f, "parent panel")
    ld22 = _colmajor(f22, "parent trailing block") if f22 is not None else 1
    _check(load().ctp_extend_add(n, p, _ptr(a), lda, _ptr(s), lds, _ptr(perm), _ptr(nelim), _ptr(vmap), np_, pp,
                                 _ptr(f), ldf, _ptr(f22), ld22, _ptr(status), _stream()), "ctp_extend_add")


def ctp_scatter_plan(tasks):
    """Plan a ctypes array of CtpScatterTask in place; returns the tiles."""
    tiles = ctypes.c_longlong(0)
    _check(load().ctp_scatter_plan(len(tasks), ctypes.cast(tasks, ctypes.c_void_p), ctypes.byref(tiles)),
           "ctp_scatter_plan")
    return tiles.value


def ctp_extend_add_batched(tasks_dev, count, tiles, panels, s, perm, nelim, vmap, fpanels, f22, status=None):
    """ctp_extend_add_batched on a device copy of a planned task array."""
    _check(load().ctp_extend_add_batched(count, _ptr(tasks_dev), tiles, _ptr(panels), _ptr(s), _ptr(perm),
                                         _ptr(nelim), _ptr(vmap), _ptr(fpanels), _ptr(f22), _ptr(status),
                                         _stream()), "ctp_extend_add_batched")


def to_device_struct(arr, device="cuda"):
    """A ctypes structure array copied to device memory (uint8 tensor)."""
    raw = bytes(memoryview(arr).cast("B"))
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
