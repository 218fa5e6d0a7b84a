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
CTP_MAX_P = 512

# Every symbol declared in include/ctp.h.
EXPORTED = ("ctp_default_opts", "ctp_version", "ctp_workspace_size", "ctp_compress",
            "ctp_factor_supernode", "ctp_solve_supernode", "ctp_supernode", "ctp_schur")


class CtpOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("u", ctypes.c_double), ("small", ctypes.c_double),
                ("prec", ctypes.c_int), ("tile", ctypes.c_int), ("flags", ctypes.c_uint)]


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
    P, I, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    OPT = ctypes.POINTER(CtpOpts)
    sig = {
        "ctp_default_opts": (None, [OPT]),
        "ctp_version": (ctypes.c_char_p, []),
        "ctp_workspace_size": (I, [I, I, OPT, ctypes.POINTER(SZ)]),
        "ctp_compress": (I, [I, I, P, I, I, P, I, P, P, P, SZ, P]),
        "ctp_factor_supernode": (I, [I, I, P, I, OPT, P, P, P, P, P, P, SZ, P]),
        "ctp_solve_supernode": (I, [I, I, P, I, P, P, P, P, OPT, P, SZ, P]),
        "ctp_supernode": (I, [I, I, P, I, OPT, P, P, P, P, P, P, SZ, P]),
        "ctp_schur": (I, [I, I, P, I, P, P, P, I, I, P, I, OPT, P, SZ, P]),
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


def ctp_default_opts(method="relaxed", u=0.01, small=1e-20):
    o = CtpOpts()
    load().ctp_default_opts(ctypes.byref(o))
    o.method = METHOD_IDS[method] if isinstance(method, str) else int(method)
    o.u = u
    o.small = small
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


def ctp_supernode(a, opts, work=None, outs=None):
    """Factor + Solve in place; returns the factor dict."""
    n, p, lda = _panel_args(a)
    work = work if work is not None else workspace(n, p, opts, a.device)
    perm, piv, d, nelim, status = outs if outs is not None else _outputs(p, a.device)
    _check(load().ctp_supernode(n, p, _ptr(a), lda, ctypes.byref(opts), _ptr(perm), _ptr(piv), _ptr(d),
                                _ptr(nelim), _ptr(status), _ptr(work), work.numel(), _stream()),
           "ctp_supernode")
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
