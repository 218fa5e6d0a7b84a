"""The allocation-free entry point (ctp_supernode_noalloc) against the
entry point it varies (ctp_supernode with a caller workspace), through the C
interface: two calls in a row on the library's static scratch, the second
with a smaller panel, each bit for bit equal to ctp_supernode on the same
input; and the size limit."""

import numpy as np
import pytest
import torch

from gpu_helpers import require_gpu
from workloads import supernode

pytestmark = pytest.mark.gpu


def _run(A, p, method, noalloc, tiled=False):
    from paper_1305_2353_amd import ctp
    n = A.shape[0]
    r = n - p
    flags = ctp.CTP_FLAG_S_TILED if tiled else 0
    opts = ctp.ctp_default_opts(method, flags=flags)
    a = ctp.device_panel(A)
    if tiled:
        s = torch.full((ctp.s_tiles(r) * 128 * 128,), 5.0, dtype=torch.float64, device="cuda")
    else:
        s = torch.full((r, r), 5.0, dtype=torch.float64, device="cuda").t()
    if noalloc:
        f = ctp.ctp_supernode_noalloc(a, opts, s=s)
    else:
        f = ctp.ctp_supernode(a, opts, work=ctp.workspace(n, p, opts), s=s)
    torch.cuda.synchronize()
    return {"a": a.cpu(), "s": s.cpu(), **{k: v.cpu() for k, v in f.items()}}


@pytest.mark.parametrize("method", ["relaxed", "strict", "tpp"])
def test_noalloc_matches_workspace_call_twice(method):
    require_gpu()
    # first call: a larger panel; second: a smaller one that reuses the scratch
    for (n, p, seed, tiled) in [(9000, 300, 1, False), (700, 60, 2, True)]:
        print("case: noalloc", method, n, p, tiled, flush=True)
        A = supernode(n, p, seed=seed, n_small=3)
        want = _run(A, p, method, noalloc=False, tiled=tiled)
        got = _run(A, p, method, noalloc=True, tiled=tiled)
        for k in want:
            assert torch.equal(got[k], want[k]), (method, n, p, k)


def test_noalloc_rejects_a_panel_beyond_its_scratch():
    require_gpu()
    from paper_1305_2353_amd import ctp
    A = supernode(20000, 512, seed=3)
    a = ctp.device_panel(A)
    with pytest.raises(ctp.CtpError, match=str(ctp.CTP_ERR_SCRATCH_TOO_SMALL)):
        ctp.ctp_supernode_noalloc(a, ctp.ctp_default_opts("relaxed"))
