// The threshold tests of the pivot loop (Section 2, eqs. (2.1) and (2.2)),
// the 2x2 pivot inverse, and the column-maximum bookkeeping, shared by the
// pivot searches.  Every expression keeps the oracle's operation order; the
// including file turns contraction off, so each product and sum rounds on
// its own.
#pragma once

#include "common.h"

namespace ctp {

// true for NaN and +-infinity
CTP_DEV bool nonfinite(double x) { return !(fabs(x) <= 1.7976931348623157e308); }

// The two largest |a| of a column (values only: when the largest value
// occurs twice, excluding either row leaves it, so no row numbers are
// needed), and whether a NaN or an infinity was met.
struct Top2 {
  double v1, v2;
  bool bad;
};

CTP_DEV Top2 top2_empty() { return Top2{-1.0, -1.0, false}; }

// x = |a| or NaN; a NaN never enters the maxima
CTP_DEV void top2_insert(Top2& t, double x) {
  t.bad |= nonfinite(x);
  x = fmax(x, -1.0);
  t.v2 = fmax(t.v2, fmin(t.v1, x));
  t.v1 = fmax(t.v1, x);
}

CTP_DEV void top2_merge(Top2& t, double o1, double o2) {
  t.v2 = fmax(fmax(t.v2, o2), fmin(t.v1, o1));
  t.v1 = fmax(t.v1, o1);
}

CTP_DEV double top2_max(const Top2& t) { return t.v1 > 0.0 ? t.v1 : 0.0; }

// largest value once one entry of value x is taken out (0 when none is left)
CTP_DEV double top2_excluding(const Top2& t, double x) {
  const double v = x == t.v1 ? t.v2 : t.v1;
  return v > 0.0 ? v : 0.0;
}

// ties of the partner search go to the lowest index
CTP_DEV bool pv_better(double va, int ia, double vb, int ib) { return va > vb || (va == vb && ia < ib); }

// Non-singularity part of the 2x2 test alone (Section 2): the scaled
// determinant is clear of cancellation and of small.
CTP_DEV bool det_ok(double att, double atm, double amm, double small) {
  const double big = fmax(fmax(fabs(att), fabs(atm)), fabs(amm));
  if (big < small) return false;
  const double s = 1.0 / big;
  const double det1 = (atm * s) * atm;
  const double det0 = (amm * s) * att;
  const double det = det0 - det1;
  return fabs(det) > fmax(fmax(small, fabs(det0) / 2.0), fabs(det1) / 2.0);
}

// The whole 2x2 test of the pivot (t, m) (Section 2): the determinant test
// above, then eq. (2.2), |D^-1| (maxt, maxm)^T <= 1/u, with maxt the
// largest entry of column t and maxm that of column m, both over the rows
// other than t and m.
CTP_DEV bool accept_2x2(double att, double atm, double amm, double maxt, double maxm, double small, double inv_u) {
  const double big = fmax(fmax(fabs(att), fabs(atm)), fabs(amm));
  if (big < small) return false;
  const double s = 1.0 / big;
  const double det1 = (atm * s) * atm;
  const double det0 = (amm * s) * att;
  const double det = det0 - det1;
  const double bound = fmax(fmax(small, fabs(det0) / 2.0), fabs(det1) / 2.0);
  if (!(fabs(det) > bound)) return false;
  if (fmax(maxt, maxm) < small) return true;
  const double f = s / fabs(det);
  const double gt = (f * fabs(amm)) * maxt + (f * fabs(atm)) * maxm;
  const double gm = (f * fabs(atm)) * maxt + (f * fabs(att)) * maxm;
  return (gt <= inv_u) && (gm <= inv_u);
}

// The 2x2 test above decided before column t's maximum is known, where its
// outcome cannot depend on it: true when the pair is rejected for every
// maxt >= 0 (the determinant test fails, or a term of |D^-1| (maxt, maxm)
// without maxt already exceeds 1/u: the rounded sum with a nonnegative term
// is at least that term).  With maxm below small the small-column branch
// may still accept, so nothing is decided.  The same comparisons as
// accept_2x2, so an early rejection is one that accept_2x2 would give.
CTP_DEV bool reject_2x2_early(double att, double atm, double amm, double maxm, double small, double inv_u) {
  const double big = fmax(fmax(fabs(att), fabs(atm)), fabs(amm));
  if (big < small) return true;
  const double s = 1.0 / big;
  const double det1 = (atm * s) * atm;
  const double det0 = (amm * s) * att;
  const double det = det0 - det1;
  const double bound = fmax(fmax(small, fabs(det0) / 2.0), fabs(det1) / 2.0);
  if (!(fabs(det) > bound)) return true;
  if (!(maxm >= small)) return false;
  const double f = s / fabs(det);
  return (f * fabs(atm)) * maxm > inv_u || (f * fabs(att)) * maxm > inv_u;
}

// D^-1 of the 2x2 pivot [d1 d21; d21 d2] (scaled by the largest entry).
CTP_DEV void inverse_2x2(double d1, double d21, double d2, double& i11, double& i21, double& i22) {
  const double s = 1.0 / fmax(fmax(fabs(d1), fabs(d21)), fabs(d2));
  const double det = (d2 * s) * d1 - (d21 * s) * d21;
  const double f = s / det;
  i11 = f * d2;
  i21 = -(f * d21);
  i22 = f * d1;
}

}  // namespace ctp
