"""Compressed threshold pivoting for symmetric indefinite supernodes on
AMD Instinct MI355X (gfx950).

The computation lives in the HIP library libctp.so (csrc/, C interface in
include/ctp.h); `paper_1305_2353_amd.ctp` is its Python binding.
"""

__all__ = ["ctp", "build"]
