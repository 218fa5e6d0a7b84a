"""Threshold pivoting on a trapezoid [A11; R] -- plain CPU oracle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library.

What it computes (Hogg & Scott, "Compressed threshold pivoting for sparse
symmetric indefinite systems", arXiv 1305.2353):

* The threshold partial pivoting kernel of Section 2 (Listing 1 with the
  1x1 test of eq. (2.1) and the 2x2 test of eq. (2.2)), applied to a
  trapezoid whose top is the symmetric p x p block A11 and whose bottom is a
  rectangular block R of r rows:
    - TPP:         R = A21 itself (every row is scanned and updated),
    - strict:      R = the compressed matrix C of eq. (4.2), updated with the
                   absolute-value formula eq. (4.4) (Section 4.1),
    - relaxed:     R = the relaxed compressed matrix of Section 4.2, updated
                   with the ordinary formula eq. (4.3),
    - restricted:  R is empty (Section 3.2: only A11 is tested).
* A decision log with the relative margin of every test, so that callers can
  tell decisions that rounding cannot flip from near-ties.

Readings of the paper taken here (where it is silent, garbled or
self-contradictory; each one is labelled and listed in the design notes):

* Loop control.  The candidate m starts at the second column and moves on by
  two after a 2x2 pivot and by one after a 1x1 pivot, as in Listing 1.  A
  candidate that fails both tests moves m on by one.  When m runs past the
  last column a new pass starts at the first uneliminated column, whose first
  candidate has no partner and so is tried as a 1x1; a pass that eliminates
  nothing ends the loop.  The first pass always gets such a second pass.
  With p = 1 the single column is the first candidate.
* The determinant test rejects the pair when |det| <= max(small, |det0|/2,
  |det1|/2); the text explains that the opposite inequality is what makes the
  pivot acceptable, so the listing's comparison sign is read as inverted.
* The 2x2 magnitude used for scaling is max(|a_tt|, |a_tm|, |a_mm|) (the
  listing repeats a_tt).
* The 2x2 stability test is eq. (2.2): |D^-1| (maxt, maxm)^T <= (1/u, 1/u)^T
  with D = [[a_tt, a_tm], [a_tm, a_mm]], the form the proof of Theorem 5.1
  relies on.
* The column maxima cover every uneliminated A11 index of the symmetric
  column (entries left and below the diagonal) and every row of R.
* "Permute m to position nelim+1" is a symmetric interchange of rows and
  columns of A11 and an interchange of columns of R.  For a 2x2 pivot t goes
  to nelim+1 first, then m to nelim+2.
* The zero-pivot test looks at the whole uneliminated symmetric column, the
  diagonal and R.  A zero pivot gets D = 0, a zero column of L and no update.
* Ties: the partner t is the lowest index among equal magnitudes.
* The strict 1x1 update is c(:,j) += c(:,k) |a(j,k)| / |a(k,k)| (the
  unscaled form in the proof of Lemma 5.1); the strict 2x2 update is
  c(:,j) += (c(:,k), c(:,k+1)) |D^-1| (|a(j,k)|, |a(j,k+1)|)^T, the bound used
  in the proof of Theorem 5.1.  In both cases the pivot columns of C are
  replaced by the bound c |D^-1| on the corresponding rows of L.

Arithmetic.  Every value is produced by IEEE double (or exact Fraction) basic
operations written out one by one -- each product rounded before each sum --
so that the sequence of operations applied to any one entry is fixed by this
text and nothing else:

    1x1 pivot d:   l_i = w_i / d;           a_ij <- a_ij - l_i * w_j
    2x2 pivot D:   s = 1 / max|D|;  det = (a22*s)*a11 - (a21*s)*a21;
                   f = s / det;  Dinv = [[f*a22, -(f*a21)], [-(f*a21), f*a11]]
                   l_i1 = w_i1*Dinv11 + w_i2*Dinv21,  l_i2 = w_i1*Dinv12 + w_i2*Dinv22
                   a_ij <- a_ij - (l_i1*w_j1 + l_i2*w_j2)

Storage.  A11 is held as a full square (its lower triangle reflected at the
start).  Each elimination updates the whole trailing square with the plain
outer product above, both triangles independently, so entry (i, j) always
receives l_i * w_j; the two triangles may therefore differ in the last bit.
The symmetric interchanges are plain row-and-column swaps of the square.
Reads follow the paper's notation: a column is read down the square (entries
above and below the diagonal of column m), the partner search reads row m
left of the diagonal, and pivot blocks use the diagonal and the entry below
it.  The factors are the lower triangle.

Numbers may be numpy float64 arrays or numpy object arrays of
fractions.Fraction (exact rational mode); the code is the same for both.
"""

from dataclasses import dataclass, field

import numpy as np

# Pivot-type codes stored per final position.
PIV_ZERO = 0        # zero pivot (column treated as zero, D = 0)
PIV_1X1 = 1         # 1x1 pivot
PIV_2X2_FIRST = 2   # first column of a 2x2 pivot
PIV_2X2_SECOND = -2  # second column of a 2x2 pivot
PIV_DELAYED = -1    # not eliminated (delayed to a later supernode)

# Status bits (the same meaning as the library's device status word).
ST_ZERO_PIVOT = 1      # a zero pivot was recorded
ST_NONFINITE = 2       # a NaN or an infinity was read by a pivot test
ST_ROOT_FALLBACK = 8   # a root panel eliminated a column regardless of u

# Update rules for the bottom block R.
R_NORMAL = "normal"   # eq. (4.3): TPP, relaxed
R_ABS = "abs"         # eq. (4.4): strict

# Margin below which a decision is reported as fragile (a near tie that a
# rounding difference could flip).
FRAGILE = 1e-9


def _zero_like(a):
    """Additive zero of the element type of array a (float or Fraction)."""
    if a.dtype == object:
        from fractions import Fraction
        return Fraction(0)
    return np.float64(0.0)


def _absmax(x, zero):
    """max |x| over the entries of x, or zero for an empty x."""
    if x.size == 0:
        return zero
    return np.max(np.abs(x))


def _finite(x):
    """True when every entry of x (a scalar or an array) is a finite number;
    exact rationals always are."""
    x = np.asarray(x)
    if x.dtype == object:
        return True
    return bool(np.isfinite(x).all())


def _ratio_margin(value, bound):
    """Relative margin value/bound - 1 as a float (inf when bound is 0)."""
    value, bound = float(value), float(bound)
    if bound == 0.0:
        return float("inf") if value > 0 else 0.0
    return value / bound - 1.0


@dataclass
class Decision:
    """One step of the pivot search, with the margins that decided it.

    kind: 'zero', '2x2', '1x1', 'reject' (both tests failed) or 'pass'
    (a new pass starts).  cols are original column ids; pos the positions.
    margins: name -> signed relative margin; |margin| < FRAGILE means that a
    rounding-level change to the data could have changed the outcome.
    """
    kind: str
    cols: tuple
    pos: tuple
    nelim: int
    margins: dict = field(default_factory=dict)
    vals: dict = field(default_factory=dict)

    def fragile(self, tol=FRAGILE):
        return any(abs(v) < tol for v in self.margins.values())


@dataclass
class TrapezoidFactors:
    """Result of threshold pivoting on [A11; R] (final positions).

    T:     p x p square; its lower triangle holds the factors: for eliminated column k,
           T[k,k] = D(k,k), T[k+1,k] = D(k+1,k) when k starts a 2x2 pivot,
           other entries below the diagonal are L; the delayed block holds the
           updated A11 entries.  Upper triangle: working values.
    R:     r x p, eliminated columns hold L rows of R (TPP / relaxed) or the
           bound on them (strict); delayed columns hold the updated R.
    perm:  perm[k] = original column at final position k.
    piv:   pivot-type code per position.
    d:     length 2p; d[2k] = D(k,k), d[2k+1] = D(k+1,k) for the first column
           of a 2x2 pivot, else 0.
    nelim: number of eliminated columns.
    log:   list of Decision.
    status: OR of the ST_* bits.
    """
    T: np.ndarray
    R: np.ndarray
    perm: np.ndarray
    piv: np.ndarray
    d: np.ndarray
    nelim: int
    log: list
    status: int = 0

    def fragile_steps(self, tol=FRAGILE):
        return [i for i, dec in enumerate(self.log) if dec.fragile(tol)]


def symmetric_from_lower(A11):
    """Full symmetric matrix whose lower triangle is that of A11."""
    low = np.tril(A11)
    return low + np.tril(A11, -1).T


def accept_2x2(a_tt, a_tm, a_mm, maxt, maxm, u, small):
    """2x2 acceptance test for the pair (t, m) (Section 2, eq. (2.2)).

    Returns (accepted, margins).  margins['det'] is the relative margin of
    the non-singularity/cancellation test and margins['stab'] that of the
    stability test 1 - u * max(|D^-1| (maxt, maxm)^T).
    """
    margins = {}
    big = max(abs(a_tt), abs(a_tm), abs(a_mm))
    if big < small:
        margins["small"] = _ratio_margin(big, small)
        return False, margins
    s = 1 / big
    det1 = (a_tm * s) * a_tm
    det0 = (a_mm * s) * a_tt
    det = det0 - det1
    bound = max(small, abs(det0) / 2, abs(det1) / 2)
    margins["det"] = _ratio_margin(abs(det), bound)
    if abs(det) <= bound:
        return False, margins
    if max(maxt, maxm) < small:
        margins["colsmall"] = _ratio_margin(max(maxt, maxm), small)
        return True, margins
    f = s / abs(det)
    # |D^-1| (maxt, maxm)^T, D = [[a_tt, a_tm], [a_tm, a_mm]].
    g_t = (f * abs(a_mm)) * maxt + (f * abs(a_tm)) * maxm
    g_m = (f * abs(a_tm)) * maxt + (f * abs(a_tt)) * maxm
    inv_u = 1 / u
    margins["stab_t"] = -_ratio_margin(g_t, inv_u)
    margins["stab_m"] = -_ratio_margin(g_m, inv_u)
    return (g_t <= inv_u) and (g_m <= inv_u), margins


def reject_2x2_early(a_tt, a_tm, a_mm, maxm, u, small):
    """The 2x2 test of eq. (2.2) decided without maxt, where its outcome is
    already fixed: True when the pair is certainly rejected.  (The paper
    evaluates the test with both maxima; skipping column t where the
    outcome cannot depend on it changes no decision, only which entries the
    search reads.)

    The acceptance test (accept_2x2) fails whatever maxt >= 0 is when the
    scaled determinant fails its test, or when the term of a component of
    |D^-1| (maxt, maxm)^T that does not involve maxt already exceeds 1/u:
    the other term is nonnegative, and the rounded sum of nonnegative terms
    is at least each of them.  With maxm below small the small-column branch
    of the test may accept, so nothing is decided there.  The search then
    does not read column t at all (so its entries do not reach the
    non-finite status bit).
    """
    big = max(abs(a_tt), abs(a_tm), abs(a_mm))
    if big < small:
        return True
    s = 1 / big
    det1 = (a_tm * s) * a_tm
    det0 = (a_mm * s) * a_tt
    det = det0 - det1
    bound = max(small, abs(det0) / 2, abs(det1) / 2)
    if abs(det) <= bound:
        return True
    if not maxm >= small:
        return False
    f = s / abs(det)
    inv_u = 1 / u
    return (f * abs(a_tm)) * maxm > inv_u or (f * abs(a_tt)) * maxm > inv_u


def det_ok(a_tt, a_tm, a_mm, small):
    """The non-singularity part of the 2x2 test alone (Section 2; reading
    C2/C3): scaled determinant clear of cancellation and of small."""
    big = max(abs(a_tt), abs(a_tm), abs(a_mm))
    if big < small:
        return False
    s = 1 / big
    det1 = (a_tm * s) * a_tm
    det0 = (a_mm * s) * a_tt
    det = det0 - det1
    return abs(det) > max(small, abs(det0) / 2, abs(det1) / 2)


def accept_1x1(a_mm, maxm, u):
    """1x1 acceptance test |a_mm| >= u * maxm (Section 2, eq. (2.1))."""
    bound = u * maxm
    return abs(a_mm) >= bound, {"one": _ratio_margin(abs(a_mm), bound)}


def _swap(T, R, perm, a, b):
    """Symmetric interchange of positions a and b (rows and columns of the
    symmetric A11, columns of R)."""
    if a == b:
        return
    T[[a, b], :] = T[[b, a], :]
    T[:, [a, b]] = T[:, [b, a]]
    R[:, [a, b]] = R[:, [b, a]]
    perm[[a, b]] = perm[[b, a]]


def _eliminate_1x1(T, R, k, r_update):
    """Apply the 1x1 pivot at position k to the trailing trapezoid."""
    d = T[k, k]
    w = T[k + 1:, k].copy()             # column below the pivot (A11 rows)
    l = w / d
    T[k + 1:, k + 1:] = T[k + 1:, k + 1:] - np.outer(l, w)
    T[k + 1:, k] = l
    if r_update == R_NORMAL:
        wr = R[:, k].copy()
        lr = wr / d
        R[:, k + 1:] = R[:, k + 1:] - np.outer(lr, w)
        R[:, k] = lr
    else:
        # Strict compressed update (Section 4.1, eq. (4.4), Lemma 5.1): every
        # row of C bounds the magnitudes of the A21 rows it stands for.
        chat = R[:, k] / abs(d)
        R[:, k + 1:] = R[:, k + 1:] + np.outer(chat, np.abs(w))
        R[:, k] = chat


def _eliminate_2x2(T, R, k, r_update):
    """Apply the 2x2 pivot at positions (k, k+1) to the trailing trapezoid."""
    a11, a21, a22 = T[k, k], T[k + 1, k], T[k + 1, k + 1]
    s = 1 / max(abs(a11), abs(a21), abs(a22))
    det = (a22 * s) * a11 - (a21 * s) * a21
    f = s / det
    i11, i21, i22 = f * a22, -(f * a21), f * a11
    w1 = T[k + 2:, k].copy()
    w2 = T[k + 2:, k + 1].copy()
    l1 = w1 * i11 + w2 * i21
    l2 = w1 * i21 + w2 * i22
    T[k + 2:, k + 2:] = T[k + 2:, k + 2:] - (np.outer(l1, w1) + np.outer(l2, w2))
    T[k + 2:, k] = l1
    T[k + 2:, k + 1] = l2
    if r_update == R_NORMAL:
        r1 = R[:, k].copy()
        r2 = R[:, k + 1].copy()
        lr1 = r1 * i11 + r2 * i21
        lr2 = r1 * i21 + r2 * i22
        R[:, k + 2:] = R[:, k + 2:] - (np.outer(lr1, w1) + np.outer(lr2, w2))
        R[:, k] = lr1
        R[:, k + 1] = lr2
    else:
        # Strict 2x2 bound (proof of Theorem 5.1): (c1, c2) |D^-1| bounds the
        # L entries of the represented rows, and the trailing bound grows by
        # that times (|a(j,k)|, |a(j,k+1)|).
        c1 = R[:, k].copy()
        c2 = R[:, k + 1].copy()
        j11, j21, j22 = abs(i11), abs(i21), abs(i22)
        ch1 = c1 * j11 + c2 * j21
        ch2 = c1 * j21 + c2 * j22
        R[:, k + 2:] = R[:, k + 2:] + (np.outer(ch1, np.abs(w1)) + np.outer(ch2, np.abs(w2)))
        R[:, k] = ch1
        R[:, k + 1] = ch2


def _col_values(T, R, nelim, m, exclude):
    """Entries of the uneliminated symmetric column m of A11 (rows nelim..p-1
    except those in exclude) followed by column m of R."""
    p = T.shape[0]
    rows = [i for i in range(nelim, p) if i not in exclude]
    top = T[rows, m] if rows else T[:0, m]
    return np.concatenate([top, R[:, m]])


def factor_trapezoid(A11, R, u=0.01, small=1e-20, r_update=R_NORMAL, forced=None, root=False):
    """Threshold pivoting (Section 2, Listing 1) on the trapezoid [A11; R].

    A11: p x p, only its lower triangle is read.  R: r x p (may have r = 0).
    forced: optional list of decisions to apply instead of testing, each
    ('1x1', col), ('2x2', col_t, col_m) or ('zero', col) with original
    column ids; the loop stops when the list is used up.  (Used to replay a
    pivot order stated in the paper.)
    root: the last panel of a factorization, where every column must be
    eliminated (Section 1 says all pivots are eliminated in the final
    supernode; the paper gives no mechanism).  When a pass makes no progress
    the column at position nelim is eliminated regardless of u: as a 1x1 if
    |a(k,k)| >= small, else as a 2x2 with column k+1 if its determinant
    passes the nonsingularity test, else as a zero pivot.  Then the normal
    loop resumes with a new pass.  Each such step is logged as 'fallback'.
    """
    p = A11.shape[0]
    T = symmetric_from_lower(A11)
    R = R.copy()
    zero = _zero_like(T)
    perm = np.arange(p)
    piv = np.full(p, PIV_DELAYED, dtype=np.int64)
    d = np.full(2 * p, zero, dtype=T.dtype) if p else np.zeros(0, dtype=T.dtype)
    log = []
    nelim = 0
    status = 0

    def record_zero(m):
        nonlocal nelim, status
        status |= ST_ZERO_PIVOT
        _swap(T, R, perm, m, nelim)
        k = nelim
        piv[k] = PIV_ZERO
        d[2 * k] = zero
        T[k, k] = zero
        T[k + 1:, k] = zero
        R[:, k] = zero
        nelim += 1

    def record_1x1(m):
        nonlocal nelim
        _swap(T, R, perm, m, nelim)
        k = nelim
        piv[k] = PIV_1X1
        d[2 * k] = T[k, k]
        _eliminate_1x1(T, R, k, r_update)
        nelim += 1

    def record_2x2(t, m):
        nonlocal nelim
        _swap(T, R, perm, t, nelim)
        _swap(T, R, perm, m, nelim + 1)
        k = nelim
        piv[k], piv[k + 1] = PIV_2X2_FIRST, PIV_2X2_SECOND
        d[2 * k], d[2 * k + 1], d[2 * k + 2] = T[k, k], T[k + 1, k], T[k + 1, k + 1]
        _eliminate_2x2(T, R, k, r_update)
        nelim += 2

    if forced is not None:
        for dec in forced:
            pos = [int(np.nonzero(perm == c)[0][0]) for c in dec[1:]]
            if dec[0] == "1x1":
                log.append(Decision("1x1", tuple(dec[1:]), tuple(pos), nelim))
                record_1x1(pos[0])
            elif dec[0] == "2x2":
                log.append(Decision("2x2", tuple(dec[1:]), tuple(pos), nelim))
                t, m = pos
                # t goes first; if m sits at nelim it is moved by that swap.
                _swap(T, R, perm, t, nelim)
                m = int(np.nonzero(perm == dec[2])[0][0])
                _swap(T, R, perm, m, nelim + 1)
                k = nelim
                piv[k], piv[k + 1] = PIV_2X2_FIRST, PIV_2X2_SECOND
                d[2 * k], d[2 * k + 1], d[2 * k + 2] = T[k, k], T[k + 1, k], T[k + 1, k + 1]
                _eliminate_2x2(T, R, k, r_update)
                nelim += 2
            elif dec[0] == "zero":
                log.append(Decision("zero", tuple(dec[1:]), tuple(pos), nelim))
                record_zero(pos[0])
            else:
                raise ValueError(dec)
        return TrapezoidFactors(T, R, perm, piv, d, nelim, log, status)

    def fallback_step():
        nonlocal status
        status |= ST_ROOT_FALLBACK
        k = nelim
        if abs(T[k, k]) >= small:
            log.append(Decision("fallback", (int(perm[k]),), (k,), nelim))
            record_1x1(k)
            return
        if k + 1 < p and det_ok(T[k, k], T[k + 1, k], T[k + 1, k + 1], small):
            log.append(Decision("fallback", (int(perm[k]), int(perm[k + 1])), (k, k + 1), nelim))
            record_2x2(k, k + 1)
            return
        log.append(Decision("fallback", (int(perm[k]),), (k,), nelim))
        record_zero(k)

    m = 1 if p >= 2 else 0
    progress = True
    while nelim < p:
        if m >= p:
            if not progress:
                if not root:
                    break
                fallback_step()
                m = nelim
                continue
            progress = False
            m = nelim
            log.append(Decision("pass", (), (m,), nelim))
            continue
        # Zero column: everything in the uneliminated column is below small.
        colm = _col_values(T, R, nelim, m, {m})
        if not (_finite(T[m, m]) and _finite(colm)):
            status |= ST_NONFINITE
        colmax = max(abs(T[m, m]), _absmax(colm, zero))
        if colmax < small:
            log.append(Decision("zero", (int(perm[m]),), (m,), nelim,
                                {"zero": -_ratio_margin(colmax, small)}))
            record_zero(m)
            m += 1
            progress = True
            continue
        if m > nelim:
            # Partner t: largest |a(m, j)| over the pending columns nelim..m-1.
            row = np.abs(T[m, nelim:m])
            t = nelim + int(np.argmax(row))
            maxm = _absmax(_col_values(T, R, nelim, m, {t, m}), zero)
            # column t is read only when the test needs maxt
            early = _finite(row) and reject_2x2_early(T[t, t], T[m, t], T[m, m], maxm, u, small)
            if not (_finite(row) and _finite(T[t, t]) and (early or _finite(_col_values(T, R, nelim, t, {t})))):
                status |= ST_NONFINITE
            margins = {}
            if row.size > 1:
                srt = sorted((float(v) for v in row), reverse=True)
                margins["t_gap"] = _ratio_margin(srt[0], srt[1]) if srt[1] > 0 else float("inf")
            maxt = _absmax(_col_values(T, R, nelim, t, {t, m}), zero)
            ok, mg = accept_2x2(T[t, t], T[m, t], T[m, m], maxt, maxm, u, small)
            assert not (early and ok), "an early rejection must agree with the full test"
            margins.update(mg)
            vals2 = {"t": int(perm[t]), "a_tt": T[t, t], "a_tm": T[m, t],
                     "a_mm": T[m, m], "maxt": maxt, "maxm2": maxm}
            if ok:
                log.append(Decision("2x2", (int(perm[t]), int(perm[m])), (t, m), nelim,
                                    margins, vals2))
                record_2x2(t, m)
                m += 2
                progress = True
                continue
            tried2 = margins
        else:
            tried2, vals2 = {}, {}
        maxm = _absmax(_col_values(T, R, nelim, m, {m}), zero)
        ok, mg = accept_1x1(T[m, m], maxm, u)
        vals = {**vals2, "a_mm": T[m, m], "maxm": maxm}
        if ok:
            log.append(Decision("1x1", (int(perm[m]),), (m,), nelim, {**tried2, **mg}, vals))
            record_1x1(m)
            m += 1
            progress = True
            continue
        log.append(Decision("reject", (int(perm[m]),), (m,), nelim, {**tried2, **mg}, vals))
        m += 1
    return TrapezoidFactors(T, R, perm, piv, d, nelim, log, status)
