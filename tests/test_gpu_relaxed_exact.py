"""Relaxed compression (Section 4.2) on panels of at most 16384 A21 rows,
where every column j gets the exact list of its j+1 best rows: C and the
rows behind it bit for bit against the oracle's column walk, on the inputs
that stress the lists.

* A21 dominated by a rank-one term: every column ranks the rows alike, so
  column j's pick is the last entry of its list (the top-8 lists of taller
  panels are exhausted from the ninth column on and need rescans);
* many equal magnitudes (small integers, an all-zero A21): the order between
  equal values is decided by the row, the last digits of the selection key;
* list sizes: lists kept in LDS for the walk and lists too large for it
  (p = 512), the widest panel the compression accepts (p = 1024, whose last
  list fills the final sort), fewer rows than columns, and 16384 rows against
  16385 (the first height that falls back to top-8 lists and rescans).
"""

import numpy as np
import pytest
import torch

from oracle.supernode import compress_relaxed
from workloads import supernode

pytestmark = pytest.mark.gpu

ST_RESCAN = 4
EXACT_ROWS = 16384


def _announce(*args):
    print("case:", *args, flush=True)


def _panel(n, p, kind, seed):
    A = supernode(n, p, seed=seed, n_small=min(3, p))
    rng = np.random.default_rng(seed + 1)
    if kind == "rank1":
        A[p:] += 100.0 * np.outer(rng.standard_normal(n - p), rng.standard_normal(p))
    elif kind == "ints":
        A[p:] = rng.integers(-2, 3, size=(n - p, p)).astype(np.float64)
    elif kind == "zeros":
        A[p:] = 0.0
    elif kind == "neg_zero":
        A[p:] = -0.0
        A[p + 5, :] = 1.0
    return A


CASES = [
    (16384 + 256, 256, "rank1"),    # the tallest exact panel, lists in LDS
    (16385 + 256, 256, "rank1"),    # one row more: top-8 lists and rescans
    (8000 + 512, 512, "rank1"),     # lists too large for LDS
    (3000, 1024, "rank1"),          # the widest panel: 1024-entry last list
    (5064, 64, "ints"),             # ties everywhere
    (600, 40, "zeros"),             # all ties
    (300, 32, "neg_zero"),          # -0 and +0 compare equal
    (300, 256, "rank1"),            # 44 rows for 256 columns
    (12000, 130, "plain"),
]


@pytest.mark.parametrize("case", CASES)
def test_relaxed_exact_lists(case):
    from paper_1305_2353_amd import ctp
    n, p, kind = case
    _announce("relaxed exact", case)
    A = _panel(n, p, kind, seed=n + p)
    a = ctp.device_panel(A)
    C, crow, status = ctp.ctp_compress(a, p, "relaxed")
    torch.cuda.synchronize()
    ref, rows = compress_relaxed(A[p:])
    assert (crow.cpu().numpy() == rows).all()
    got = np.ascontiguousarray(C.cpu().numpy())
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))   # signs of zeros included
    st = int(status.item()) if hasattr(status, "item") else int(status)
    rescan = kind == "rank1" and n - p > EXACT_ROWS
    assert bool(st & ST_RESCAN) == rescan, st
