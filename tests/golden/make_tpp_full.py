"""Write the oracle's threshold-partial-pivoting result for the n = 100000,
p = 512 supernode (workloads.large_supernode(0), u = 0.01, small = 1e-20)
to tpp_n100000_p512.json.

    python tests/golden/make_tpp_full.py

The oracle needs several minutes for this panel (every one of the 512
eliminations updates all 99488 rows of A21), too long for a test, so its
result is stored once: the decisions and D exactly (hexadecimal floats), the
SHA-256 of the lower triangle of the A11 rows and of the A21 rows of the
output panel (row-major float64 bytes), and 16 sampled A21 rows in full.
Only oracle/ and workloads/ are called.
"""

import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.supernode import factor_supernode  # noqa: E402
from workloads import large_supernode  # noqa: E402

OUT = os.path.join(HERE, "tpp_n100000_p512.json")


def panel_hashes(out, p):
    low = np.ascontiguousarray(np.tril(out[:p]), dtype=np.float64)
    a21 = np.ascontiguousarray(out[p:], dtype=np.float64)
    return hashlib.sha256(low.tobytes()).hexdigest(), hashlib.sha256(a21.tobytes()).hexdigest()


def main():
    A = large_supernode(0)
    n, p = A.shape
    F = factor_supernode(A, p, "tpp", u=0.01, small=1e-20)
    h11, h21 = panel_hashes(F.out, p)
    rows = sorted(set([0, n - p - 1] + list(np.random.default_rng(7).integers(0, n - p, 14))))
    rec = {
        "workload": "workloads.large_supernode(0): n=100000, p=512, TPP, u=0.01, small=1e-20",
        "n": n, "p": p, "nelim": int(F.nelim), "status": int(F.status),
        "fragile_steps": len(F.trap.fragile_steps()),
        "perm": [int(x) for x in F.perm],
        "piv": [int(x) for x in F.piv],
        "d": [float(x).hex() for x in F.d],
        "sha256_a11_lower": h11,
        "sha256_a21": h21,
        "rows": [int(r) for r in rows],
        "row_values": [[float(x).hex() for x in F.out[p + r]] for r in rows],
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT}: nelim {F.nelim}")


if __name__ == "__main__":
    main()
