"""Roofline probes (libctp_probe.so): the matrix-core and HBM peaks measured
on the machine at hand, beside the datasheet figures the roofline fractions
are quoted against.

    mfma_peak("fp64" | "fp32" | "bf16") -> TFLOP/s of a register-only loop
        of the matrix-core instruction the library's kernels use;
    copy_bandwidth(bytes) -> GB/s (read + written) of a 16-byte stream copy.

Timing with HIP events on the current stream (the launchers only launch).
"""

import ctypes
import os

from .ctp import CtpError

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctp_probe.so")
KINDS = {"fp64": 0, "fp32": 1, "bf16": 2}
_lib = None


def load(path=LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CtpError(f"{path} is missing: build it with `python -m paper_1305_2353_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, SZ, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_longlong
    lib.ctp_probe_mfma_flop.restype, lib.ctp_probe_mfma_flop.argtypes = LL, [I]
    lib.ctp_probe_mfma.restype, lib.ctp_probe_mfma.argtypes = I, [I, I, I, P, P]
    lib.ctp_probe_nacc.restype, lib.ctp_probe_nacc.argtypes = I, []
    lib.ctp_probe_copy.restype, lib.ctp_probe_copy.argtypes = I, [P, P, SZ, I, I, P]
    _lib = lib
    return lib


def _timed(launch, reps):
    import torch
    launch()                                     # warm-up
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        launch()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def mfma_peak(dtype="fp64", grid=2048, iters=4096, reps=3):
    """TFLOP/s of the matrix-core loop: grid x 4 waves, each iters x NACC
    instructions (best of reps launches)."""
    import torch
    lib = load()
    kind = KINDS[dtype]
    out = torch.empty(grid * 4, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def launch():
        rc = lib.ctp_probe_mfma(kind, grid, iters, ctypes.c_void_p(out.data_ptr()), stream)
        if rc:
            raise CtpError(f"ctp_probe_mfma returned {rc}")

    ms = _timed(launch, reps)
    flop = float(lib.ctp_probe_mfma_flop(kind)) * lib.ctp_probe_nacc() * iters * grid * 4
    return flop / (ms * 1e-3) / 1e12


def copy_bandwidth(nbytes=1 << 31, grids=(2048, 4096, 8192), reps=3):
    """GB/s (bytes read + bytes written) of a device-to-device copy: the
    best over a few grid sizes, with plain and with non-temporal accesses."""
    import torch
    lib = load()
    n = nbytes // 16 * 16
    src = torch.empty(n // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    best = 0.0
    for nt in (0, 1):
        for grid in grids:
            def launch():
                rc = lib.ctp_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, grid, nt,
                                        stream)
                if rc:
                    raise CtpError(f"ctp_probe_copy returned {rc}")

            ms = _timed(launch, reps)
            best = max(best, 2.0 * n / (ms * 1e-3) / 1e9)
    if not torch.equal(src[:4096], dst[:4096]):
        raise CtpError("probe copy produced wrong data")
    return best
