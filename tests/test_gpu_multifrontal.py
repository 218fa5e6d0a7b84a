"""Multi-level multifrontal factorization on the GPU (Section 1: Factor,
Solve, Form and Scatter chained over an assembly tree, delayed pivots
passed to the parent) against the oracle's multifrontal factorization of
the same synthetic matrix (oracle/multifrontal.py).

Per front: the same index list, nelim and pivot order (decisions exact
where no decision of the oracle is a near tie), the assembled front and the
factored panel within 1e-12 normwise; globally, the GPU factors reproduce
P A P^T and have the inertia of A.
"""

from types import SimpleNamespace

import numpy as np
import pytest
import torch

from gpu_helpers import rel_err, require_gpu
from oracle.multifrontal import global_factors, multifrontal
from workloads import assembly_tree

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _announce(*args):
    print("case:", *args, flush=True)


def _fragile(fronts):
    return any(fr["F"].trap.fragile_steps() for fr in fronts.values())


CASES = [("relaxed", 0, (3, 2), 30.0), ("strict", 0, (3, 2), 30.0), ("relaxed", 1, (4,), 1.0),
         ("strict", 1, (4,), 1.0), ("restricted", 1, (4,), 1.0), ("relaxed", 2, (2, 2, 2), 30.0),
         ("strict", 2, (2, 2, 2), 30.0), ("restricted", 3, (3, 2), 1.0)]


# Restricted pivoting tests its pivots against A11 alone (Section 3.2): with
# boundary rows scaled up its L grows without bound and the factors carry
# that growth times the rounding, so it runs on unscaled trees only.
@pytest.mark.parametrize("method,seed,fanout,bound_scale", CASES)
def test_multifrontal_matches_oracle(method, seed, fanout, bound_scale):
    from paper_1305_2353_amd.multifrontal import multifrontal_factor
    _announce("multifrontal", method, seed, fanout, bound_scale)
    tree = assembly_tree(seed, fanout=fanout, bound_scale=bound_scale)
    A = tree["A"]
    ref = multifrontal(tree, method)
    if _fragile(ref):
        pytest.skip("near-tie decision in this draw")
    fronts = multifrontal_factor(tree, torch.as_tensor(A, device="cuda"), method, keep_assembled=True)
    torch.cuda.synchronize()
    gpu_fronts = {}
    for q in tree["postorder"]:
        fr, rf = fronts[q], ref[q]
        F = rf["F"]
        assert np.array_equal(fr.vars, rf["vars"]), q
        assert fr.p == rf["p"], q
        assert fr.nelim == F.nelim, q
        assert np.array_equal(fr.perm, F.perm), q
        # the front as assembled (panel lower part and trailing block)
        panel0, s0 = fr.assembled
        p = fr.p
        P0 = panel0.cpu().numpy()
        assert rel_err(np.tril(P0[:p]), np.tril(rf["assembled"][:p, :p])) <= TOL, q
        if fr.n > p:
            assert rel_err(P0[p:], rf["assembled"][p:, :p]) <= TOL, q
            assert rel_err(np.tril(s0.cpu().numpy()), np.tril(rf["assembled"][p:, p:])) <= TOL, q
        out = fr.outputs()
        panel = out["panel"].cpu().numpy()
        piv = out["piv"].cpu().numpy()
        d = out["d"].cpu().numpy()
        assert np.array_equal(piv, F.piv), q
        assert rel_err(d, F.d) <= TOL, q
        assert rel_err(np.tril(panel[:p]), np.tril(F.out[:p])) <= TOL, q
        if fr.n > p:
            assert rel_err(panel[p:], F.out[p:]) <= TOL, q
        gpu_fronts[q] = {"vars": fr.vars, "p": p,
                         "F": SimpleNamespace(out=panel, perm=fr.perm, piv=piv, d=d, nelim=fr.nelim)}
    # the GPU's own factors, gathered: P A P^T = L D L^T and the inertia of A
    order, L, D = global_factors(tree, gpu_fronts)
    res = np.abs(A[np.ix_(order, order)] - L @ D @ L.T).max() / np.abs(A).max()
    assert res <= 1e-11
    ev, ed = np.linalg.eigvalsh(A), np.linalg.eigvalsh(D)
    assert (ev > 0).sum() == (ed > 0).sum() and (ev < 0).sum() == (ed < 0).sum()
