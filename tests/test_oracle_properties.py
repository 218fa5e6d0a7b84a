"""The oracle against what the mathematics fixes.

* Brute force: the factors rebuild P A11 P^T and A21 P^T.
* Closed forms given the decisions (Schur complements from the original
  data by dense solves) for L21, the delayed blocks and S.
* Sylvester's law of inertia: D has the eigenvalue signs of the
  eliminated block.
* Theorem 5.1 / eq. (5.1): |l| <= 1/u for TPP and strict, and the growth
  bounds per 1x1 and 2x2 pivot; Lemma 5.1: the strict C bounds the real A21.
* Special cases where the methods must coincide.
* Exact rational arithmetic agrees with the float run at robust decisions.
* Decision replay: every logged test input equals the Schur complement of
  the original data at that point.
"""

from fractions import Fraction as Fr

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle.supernode import (closed_forms, compress_relaxed, compress_strict, d_blocks,
                              factor_supernode, schur_rows, unit_lower_L11)
from oracle.threshold import (PIV_2X2_FIRST, PIV_ZERO, R_ABS, R_NORMAL,
                              factor_trapezoid)
from workloads import small_supernode, supernode

METHODS = ["tpp", "strict", "relaxed", "restricted"]
CASES = [(256, 32, 0, 4), (96, 24, 1, 3), (64, 16, 2, 5), (40, 12, 3, 2), (24, 24, 4, 3),
         (300, 48, 5, 6), (33, 7, 6, 1)]


def _panel(n, p, seed, nsmall):
    return supernode(n, p, seed, n_small=nsmall, small_scale=1e-8)


def _factors(F, p):
    L = unit_lower_L11(F.out, F.piv, F.nelim)
    D = d_blocks(F.piv, F.d, F.nelim)
    return L, D


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", CASES)
def test_brute_force_reconstruction(method, case):
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    F = factor_supernode(A, p, method)
    L, D = _factors(F, p)
    ne = F.nelim
    A11 = np.tril(A[:p]) + np.tril(A[:p], -1).T
    B = A11[np.ix_(F.perm, F.perm)]
    G = A[p:][:, F.perm]
    scale = np.abs(A).max()
    LE, Ld = L[:ne, :ne], L[ne:, :ne]
    L21 = F.out[p:, :ne]
    # eliminated block and L_dE
    assert np.abs(B[:ne, :ne] - LE @ D @ LE.T).max(initial=0) <= 1e-12 * scale
    assert np.abs(B[ne:, :ne] - Ld @ D @ LE.T).max(initial=0) <= 1e-12 * scale
    # delayed block of A11 (lower triangle)
    Bdd = B[ne:, ne:] - Ld @ D @ Ld.T
    assert np.abs(np.tril(F.out[ne:p, ne:p] - Bdd)).max(initial=0) <= 1e-11 * scale
    # A21 rows
    assert np.abs(G[:, :ne] - L21 @ D @ LE.T).max(initial=0) <= 1e-11 * scale
    assert np.abs(F.out[p:, ne:] - (G[:, ne:] - L21 @ D @ Ld.T)).max(initial=0) <= 1e-11 * scale


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", CASES[:5])
def test_closed_forms_and_schur(method, case):
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    F = factor_supernode(A, p, method)
    assert PIV_ZERO not in F.piv
    cf = closed_forms(A, p, F.perm, F.piv, F.nelim)
    scale = max(1.0, np.abs(cf["S"]).max(initial=0))
    S = schur_rows(F, np.arange(n - p))
    assert np.abs(np.tril(S) - np.tril(cf["S"])).max(initial=0) <= 1e-10 * scale
    assert np.abs(F.out[p:, F.nelim:] - cf["Gd_prime"]).max(initial=0) <= 1e-10 * scale
    ne = F.nelim
    assert np.abs(np.tril(F.out[ne:p, ne:p] - cf["Bdd_prime"])).max(initial=0) <= 1e-10 * scale
    # W = L21 D
    D = d_blocks(F.piv, F.d, ne)
    assert np.abs(F.W - F.out[p:, :ne] @ D).max(initial=0) <= 1e-11 * max(1.0, np.abs(F.W).max(initial=0))


def _inertia_of_D(F):
    D = d_blocks(F.piv, F.d, F.nelim)
    ev = []
    k = 0
    while k < F.nelim:
        if F.piv[k] == PIV_2X2_FIRST:
            ev.extend(np.linalg.eigvalsh(D[k:k + 2, k:k + 2]))
            k += 2
        else:
            ev.append(D[k, k])
            k += 1
    ev = np.array(ev)
    return int((ev > 0).sum()), int((ev < 0).sum()), int((ev == 0).sum())


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", CASES)
def test_inertia_matches_eigenvalues(method, case):
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    F = factor_supernode(A, p, method)
    A11 = np.tril(A[:p]) + np.tril(A[:p], -1).T
    B = A11[np.ix_(F.perm, F.perm)][:F.nelim, :F.nelim]
    ev = np.linalg.eigvalsh(B) if F.nelim else np.zeros(0)
    tol = 1e-12 * max(1.0, np.abs(B).max()) if F.nelim else 0
    assert _inertia_of_D(F) == (int((ev > tol).sum()), int((ev < -tol).sum()),
                                int((np.abs(ev) <= tol).sum()))


@pytest.mark.parametrize("method", ["tpp", "strict"])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("u", [0.01, 0.1, 0.5])
def test_l_bounded_by_inverse_threshold(method, case, u):
    # Theorem 5.1 (strict) and the threshold tests (TPP): every L entry,
    # A21 rows included, is at most 1/u in magnitude.
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    F = factor_supernode(A, p, method, u=u)
    L, _ = _factors(F, p)
    L21 = F.out[p:, :F.nelim]
    bound = (1 / u) * (1 + 1e-12)
    assert np.abs(np.tril(L, -1)).max(initial=0) <= bound
    assert np.abs(L21).max(initial=0) <= bound


def test_relaxed_l_can_exceed_bound_somewhere():
    # Relaxed pivoting only tests the rows kept in C; on panels with many
    # rows the worst L21 entry is typically larger than the C rows allow.
    worst = 0.0
    for seed in range(6):
        A = _panel(400, 24, seed, 3)
        F = factor_supernode(A, 24, "relaxed", u=0.5)
        worst = max(worst, np.abs(F.out[24:, :F.nelim]).max(initial=0))
    assert worst > 2.0


def _shadow_states(A, p, F, u):
    """Trapezoid [A11; A21] after each accepted decision of F, obtained by
    applying F's decisions to the real panel with the ordinary update."""
    dec = [d for d in F.log if d.kind in ("1x1", "2x2")]
    states = []
    for q in range(len(dec) + 1):
        forced = [(d.kind,) + tuple(d.cols) for d in dec[:q]]
        T = factor_trapezoid(A[:p], A[p:], u, 1e-20, R_NORMAL, forced)
        states.append((T, dec[q - 1].kind if q else None))
    return states


@pytest.mark.parametrize("method", ["tpp", "strict"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_growth_bound_per_pivot(method, seed):
    # eq. (5.1): mu_{q+1} <= mu_q (1 + 1/u) for a 1x1 pivot and
    # mu_{q+2} <= mu_q (1 + 2/u) for a 2x2 pivot, mu over the uneliminated
    # trapezoid (A11 lower part and all A21 rows).
    u = 0.5
    n, p = 60, 12
    A = _panel(n, p, seed, 3)
    F = factor_supernode(A, p, method, u=u)
    prev = None
    for T, kind in _shadow_states(A, p, F, u):
        k = T.nelim
        mu = max(np.abs(np.tril(T.T[k:, k:])).max(initial=0), np.abs(T.R[:, k:]).max(initial=0))
        if prev is not None:
            factor = (1 + 1 / u) if kind == "1x1" else (1 + 2 / u)
            assert mu <= prev * factor * (1 + 1e-12)
        prev = mu


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_lemma_5_1_strict_c_bounds_a21(seed):
    # |a^(q)(i,k)| <= c^(q)(j,k) for i in J_j after every elimination q,
    # with the real A21 updated by the strict run's decisions.
    u = 0.1
    n, p = 80, 10
    A = _panel(n, p, seed, 2)
    A21 = A[p:]
    J = np.argmax(np.abs(A21), axis=1)
    F = factor_supernode(A, p, "strict", u=u)
    dec = [d for d in F.log if d.kind in ("1x1", "2x2")]
    for q in range(len(dec) + 1):
        forced = [(d.kind,) + tuple(d.cols) for d in dec[:q]]
        real = factor_trapezoid(A[:p], A21, u, 1e-20, R_NORMAL, forced)
        comp = factor_trapezoid(A[:p], compress_strict(A21), u, 1e-20, R_ABS, forced)
        assert (real.perm == comp.perm).all()
        bound = comp.R[J]          # row j of C for each A21 row
        assert (np.abs(real.R) <= bound * (1 + 1e-12) + 1e-300).all()


@pytest.mark.parametrize("case", [(32, 32, 0, 4), (16, 16, 1, 2), (9, 9, 2, 1)])
def test_all_methods_agree_without_a21(case):
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    ref = factor_supernode(A, p, "tpp")
    for method in METHODS[1:]:
        F = factor_supernode(A, p, method)
        assert (F.perm == ref.perm).all() and (F.piv == ref.piv).all()
        assert (F.out == ref.out).all()


@pytest.mark.parametrize("seed", range(4))
def test_all_methods_agree_when_a21_is_zero(seed):
    A = _panel(70, 14, seed, 3)
    A[14:] = 0
    ref = factor_supernode(A, 14, "tpp")
    for method in METHODS[1:]:
        F = factor_supernode(A, 14, method)
        assert (F.perm == ref.perm).all() and (F.piv == ref.piv).all()
        assert (np.tril(F.out[:14]) == np.tril(ref.out[:14])).all()


@pytest.mark.parametrize("case", [(40, 20, 0), (30, 20, 1), (21, 20, 2), (48, 24, 3)])
def test_relaxed_equals_tpp_when_c_holds_every_row(case):
    # n - p <= p: C holds every A21 row (plus zero rows), and both tests
    # only use maxima, so relaxed and TPP make the same decisions with the
    # same arithmetic on A11.
    n, p, seed = case
    A = _panel(n, p, seed, 3)
    T = factor_supernode(A, p, "tpp")
    R = factor_supernode(A, p, "relaxed")
    assert (T.perm == R.perm).all() and (T.piv == R.piv).all()
    assert (np.tril(T.out[:p]) == np.tril(R.out[:p])).all()
    assert np.abs(T.out[p:] - R.out[p:]).max(initial=0) <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("seed", range(6))
def test_strict_equals_tpp_for_one_column(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((30, 1))
    if seed % 2:
        A[0, 0] *= 1e-3
    T = factor_supernode(A, 1, "tpp")
    S = factor_supernode(A, 1, "strict")
    assert T.nelim == S.nelim and (T.piv == S.piv).all()


@pytest.mark.parametrize("seed", range(4))
def test_restricted_is_compressed_with_zero_c(seed):
    A = _panel(50, 10, seed, 3)
    F = factor_supernode(A, 10, "restricted")
    Z = factor_trapezoid(A[:10], np.zeros((10, 10)), 0.01, 1e-20, R_NORMAL)
    assert (F.perm == Z.perm).all() and (F.piv == Z.piv).all()
    assert (np.tril(F.out[:10]) == np.tril(Z.T)).all()


@pytest.mark.parametrize("seed", range(20))
def test_strict_acceptance_implies_tpp_acceptance(seed):
    # At the first decision the state is the same for both; C bounds A21
    # (Lemma 5.1, q = 0) and both tests are monotone in the column maxima.
    A = _panel(60, 8, seed, 2)
    S = factor_supernode(A, 8, "strict")
    T = factor_supernode(A, 8, "tpp")
    if S.log[0].kind in ("1x1", "2x2"):
        assert T.log[0].kind == S.log[0].kind and T.log[0].cols == S.log[0].cols


def _int_panel(n, p, seed):
    rng = np.random.default_rng(seed)
    G = rng.integers(-6, 7, size=(p, p))
    A11 = np.tril(G) + np.tril(G, -1).T
    A21 = rng.integers(-9, 10, size=(n - p, p))
    return np.vstack([A11, A21])


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_agrees_with_float(method, seed):
    n, p = 18 + seed, 6
    Ai = _int_panel(n, p, seed)
    Fx = factor_supernode(np.array([[Fr(int(x)) for x in r] for r in Ai], dtype=object),
                          p, method, u=Fr(1, 100), small=Fr(1, 10**20))
    Ff = factor_supernode(Ai.astype(float), p, method)
    robust_prefix = len(Ff.log) if not Ff.trap.fragile_steps() else Ff.trap.fragile_steps()[0]
    kinds_x = [(d.kind, d.cols) for d in Fx.log[:robust_prefix]]
    kinds_f = [(d.kind, d.cols) for d in Ff.log[:robust_prefix]]
    assert kinds_x == kinds_f
    if not Ff.trap.fragile_steps():
        assert (Fx.perm == Ff.perm).all() and Fx.nelim == Ff.nelim
        ex = np.array(Fx.out, dtype=float)
        assert np.abs(ex - Ff.out).max(initial=0) <= 1e-10 * max(1.0, np.abs(ex).max())


def _replay_rows(method, F, A, p):
    n = A.shape[0]
    if method == "tpp":
        return list(range(p, n))
    if method == "relaxed":
        return [p + int(r) for r in F.crow if r >= 0]
    return []


@pytest.mark.parametrize("method", ["tpp", "relaxed", "restricted", "strict"])
@pytest.mark.parametrize("case", [(80, 16, 0, 3), (120, 20, 1, 4), (256, 32, 0, 4)])
def test_decision_replay_from_schur_complements(method, case):
    """Every logged test input (pivot entries and column maxima) equals the
    Schur complement of the original data with respect to the columns
    eliminated before that decision."""
    n, p, seed, nsmall = case
    A = _panel(n, p, seed, nsmall)
    F = factor_supernode(A, p, method)
    M = np.vstack([np.tril(A[:p]) + np.tril(A[:p], -1).T, A[p:]])   # n x p
    rrows = _replay_rows(method, F, A, p)
    elim = []
    checked = 0
    for dec in F.log:
        if dec.kind == "pass":
            continue
        if elim:
            E = np.array(elim)
            X = np.linalg.solve(M[E][:, E], M[E])             # A_EE^-1 A_E*
            S = M - M[:, E] @ X                               # n x p Schur complement
        else:
            S = M.copy()
        unelim = [c for c in range(p) if c not in elim]
        m = dec.cols[-1]

        def colmax(c, excl):
            vals = [abs(S[i, c]) for i in unelim if i not in excl] + [abs(S[i, c]) for i in rrows]
            return max(vals, default=0.0)

        tol = 1e-9
        v = dec.vals
        if "maxm" in v:
            assert abs(v["a_mm"] - S[m, m]) <= tol * max(1, abs(S[m, m]))
            if method != "strict":
                assert abs(v["maxm"] - colmax(m, {m})) <= tol * max(1, v["maxm"])
            else:
                assert v["maxm"] >= colmax(m, {m}) * (1 - 1e-12)
        if "maxt" in v:
            t = v["t"]
            assert abs(v["a_tt"] - S[t, t]) <= tol * max(1, abs(S[t, t]))
            assert abs(v["a_tm"] - S[m, t]) <= tol * max(1, abs(S[m, t]))
            if method != "strict":
                assert abs(v["maxt"] - colmax(t, {t, m})) <= tol * max(1, v["maxt"])
                assert abs(v["maxm2"] - colmax(m, {t, m})) <= tol * max(1, v["maxm2"])
        checked += 1
        if dec.kind == "1x1":
            elim.append(m)
        elif dec.kind == "2x2":
            elim.extend(dec.cols)
    assert checked >= p // 2


@settings(max_examples=40, deadline=None)
@given(p=st.integers(1, 14), extra=st.integers(0, 30), seed=st.integers(0, 10**6),
       method=st.sampled_from(METHODS), nsmall=st.integers(0, 3))
def test_property_factors_are_consistent(p, extra, seed, method, nsmall):
    n = p + extra
    A = supernode(n, p, seed, n_small=min(nsmall, p), small_scale=1e-8)
    F = factor_supernode(A, p, method)
    assert 0 <= F.nelim <= p
    assert sorted(F.perm) == list(range(p))
    L, D = _factors(F, p)
    ne = F.nelim
    A11 = np.tril(A[:p]) + np.tril(A[:p], -1).T
    B = A11[np.ix_(F.perm, F.perm)]
    scale = np.abs(A).max()
    assert np.abs(B[:ne, :ne] - L[:ne, :ne] @ D @ L[:ne, :ne].T).max(initial=0) <= 1e-11 * scale
    if method in ("tpp", "strict"):
        assert np.abs(F.out[p:, :ne]).max(initial=0) <= 100 * (1 + 1e-12)
