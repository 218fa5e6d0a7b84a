// Threshold pivot search on a trapezoid [A11; R] (Section 2: tests (2.1) and
// (2.2); run on the compressed trapezoid of Section 4, Fig. 4.1 (c), or for
// TPP on the whole panel).
//
// R is the compressed matrix C (strict: absolute-value update (4.4); relaxed:
// ordinary update (4.3)), the real A21 (TPP) or empty (restricted pivoting).
//
// Readings of the paper (the same as the oracle's):
//  * candidate m starts at the second column, advances by 2 after a 2x2
//    pivot, by 1 after a 1x1 pivot or a double failure; past the last column
//    a new pass starts at the first uneliminated column (tried alone as a
//    1x1) if the pass eliminated anything (the first pass always gets one);
//  * the determinant test rejects when |det| <= max(small, |det0|/2,
//    |det1|/2); the 2x2 scale uses max(|a_tt|, |a_tm|, |a_mm|);
//  * the 2x2 stability test is |D^-1| (maxt, maxm)^T <= 1/u (eq. (2.2));
//  * column maxima run over the whole uneliminated column of the square and
//    every row of R; the partner search reads row m left of the diagonal;
//  * interchanges are symmetric row-and-column swaps (t to position nelim,
//    then m to nelim+1 for a 2x2 pivot);
//  * zero pivot: every entry of the column below `small`: D = 0, zero L
//    column, no update;  ties go to the lowest index.
//
// Arithmetic: contraction is off in this file; every update is a rounded
// product followed by a rounded sum, in the oracle's order:
//      1x1:  l_i = w_i / d;  a_ij = a_ij - l_i * w_j
//      2x2:  s = 1/max|D|, det = (a22*s)*a11 - (a21*s)*a21, f = s/det,
//            Dinv = [[f*a22, -(f*a21)], [., f*a11]],
//            l_i1 = w_i1*Dinv11 + w_i2*Dinv21, l_i2 = w_i1*Dinv12 + w_i2*Dinv22,
//            a_ij = a_ij - (l_i1*w_j1 + l_i2*w_j2)
// A11 is kept as a full square in the panel's A11 block (the lower triangle
// is reflected first); entry (i, j) of the trailing square always receives
// l_i * w_j, so every value is reproducible bit for bit.
//
// Organisation (batched, delayed updates):
//  * decide kernel (one workgroup): runs the pivot loop.  Trailing entries
//    are read lazily as "stored value minus the pending updates" of up to
//    NSLOT eliminated columns whose multipliers (l) and pivot-column values
//    (w) sit in LDS.  Because every pending update of entry (i, j) is
//    l_i * w_j with vectors permuted along with the rows, lazy reads commute
//    with the interchanges and give exactly the right-looking values.  The
//    launch stops when the batch is full (or the loop ends), saving its
//    state in the workspace.
//  * apply kernel (many workgroups): applies the batch to the trailing
//    square and to R, entry by entry in the same order.
//  The host enqueues init, then a fixed number of decide/apply pairs
//  (enough for p eliminations); pairs after the end of the loop exit at
//  once, so the launch sequence does not depend on the data.

#include "common.h"

#pragma clang fp contract(off)

namespace ctp {

constexpr int PIV_THREADS = 1024;
constexpr int PIV_WAVES = PIV_THREADS / 64;
constexpr int NSLOT = PIV_NSLOT;   // pending eliminated columns per batch
constexpr int RCACHE = 1024;       // R rows whose multipliers are cached in LDS
constexpr int APPLY_TILE = 64;

struct PivState {
  int nelim, m, progress, done;
  int nslot, status, pad0, pad1;
  int slot_k[NSLOT];      // position of the pivot column behind each slot
  int slot_kind[NSLOT];   // 1: 1x1, 2: first column of a 2x2, 3: second column
};

struct PivotArgs {
  int p;
  double* T;     // A11 as a full square, column-major, lda
  int lda;
  int r;
  double* R;     // bottom block, column-major, ldr (may be null when r == 0)
  int ldr;
  int abs_update;   // 1: strict rule for R
  int root;         // 1: eliminate every column (fallback when a pass stalls)
  double u, small;
  int* perm;
  int* piv;
  double* d;
  int* nelim_out;
  int* status;
  PivState* st;
  double* wbuf;  // NSLOT x p: the batch's w vectors for the apply kernel
};

static_assert(sizeof(PivState) <= PIV_STATE_BYTES, "pivot state does not fit its workspace slot");

// ---------------------------------------------------------------------------
// init: reflect A11, reset the state and the outputs
// ---------------------------------------------------------------------------

CTP_DEV void pivot_init_body(const PivotArgs& g, size_t tid, size_t stride) {
  const int p = g.p;
  for (size_t q = tid; q < (size_t)p * p; q += stride) {
    const int i = (int)(q % p), j = (int)(q / p);
    if (i < j) CM(g.T, i, j, g.lda) = CM(g.T, j, i, g.lda);
  }
  for (size_t k = tid; k < (size_t)p; k += stride) {
    g.perm[k] = (int)k;
    g.piv[k] = PIV_DELAYED;
    g.d[2 * k] = 0.0;
    g.d[2 * k + 1] = 0.0;
  }
  if (tid == 0) {
    PivState* st = g.st;
    st->nelim = 0;
    st->m = p >= 2 ? 1 : 0;
    st->progress = 1;
    st->done = p == 0;
    st->nslot = 0;
    st->status = 0;
    *g.nelim_out = 0;
  }
}

__global__ void pivot_init_kernel(PivotArgs g) {
  pivot_init_body(g, (size_t)blockIdx.x * blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x);
}

// ---------------------------------------------------------------------------
// decide: the pivot loop on lazily updated values
// ---------------------------------------------------------------------------

struct DecideShared {
  double red_v[PIV_WAVES];
  double red_v2[PIV_WAVES];
  int red_i[PIV_WAVES];
  int nelim, m, progress, done, nslot, action, status;
  int kind[NSLOT];
  int sk[NSLOT];
};

// LDS of the decide kernel.  Dynamic part: multipliers of A11 rows
// lA[NSLOT][p], pivot-column values wc[NSLOT][p] (both by position) and
// multipliers of the first rc rows of R, lR[NSLOT][rc].
extern __shared__ double pv_dyn[];
__shared__ DecideShared pv_sh;
__shared__ double pv_d[2 * CTP_MAX_P];
__shared__ int pv_perm[CTP_MAX_P];
__shared__ int pv_piv[CTP_MAX_P];

CTP_DEV double& lA(int p, int s, int i) { return pv_dyn[s * p + i]; }
CTP_DEV double& wc(int p, int s, int j) { return pv_dyn[NSLOT * p + s * p + j]; }
CTP_DEV double& lR(int p, int rc, int s, int i) { return pv_dyn[2 * NSLOT * p + s * rc + i]; }

CTP_DEV double lazy_a(const PivotArgs& g, int i, int j) {
  double v = CM(g.T, i, j, g.lda);
  const int p = g.p;
  const int ns = pv_sh.nslot;
  for (int s = 0; s < ns; ++s) {
    if (pv_sh.kind[s] == 1) {
      const double prod = lA(p, s, i) * wc(p, s, j);
      v = v - prod;
    } else {
      const double upd = lA(p, s, i) * wc(p, s, j) + lA(p, s + 1, i) * wc(p, s + 1, j);
      v = v - upd;
      ++s;
    }
  }
  return v;
}

CTP_DEV double r_mult(const PivotArgs& g, int rc, int s, int i) {
  return i < rc ? lR(g.p, rc, s, i) : CM(g.R, i, pv_sh.sk[s], g.ldr);
}

CTP_DEV double lazy_r(const PivotArgs& g, int rc, int i, int j) {
  double v = CM(g.R, i, j, g.ldr);
  const int p = g.p;
  const int ns = pv_sh.nslot;
  for (int s = 0; s < ns; ++s) {
    if (pv_sh.kind[s] == 1) {
      const double lr = r_mult(g, rc, s, i);
      const double w = wc(p, s, j);
      if (g.abs_update) {
        const double prod = lr * fabs(w);
        v = v + prod;
      } else {
        const double prod = lr * w;
        v = v - prod;
      }
    } else {
      const double l1 = r_mult(g, rc, s, i), l2 = r_mult(g, rc, s + 1, i);
      const double w1 = wc(p, s, j), w2 = wc(p, s + 1, j);
      if (g.abs_update) {
        const double upd = l1 * fabs(w1) + l2 * fabs(w2);
        v = v + upd;
      } else {
        const double upd = l1 * w1 + l2 * w2;
        v = v - upd;
      }
      ++s;
    }
  }
  return v;
}

CTP_DEV double block_max(double v) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  if (lane == 0) pv_sh.red_v[wave] = v;
  __syncthreads();
  double r = pv_sh.red_v[0];
  for (int w = 1; w < PIV_WAVES; ++w) r = fmax(r, pv_sh.red_v[w]);
  __syncthreads();
  return r;
}

CTP_DEV void block_max2(double& v1, double& v2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v1 = wave_max(v1);
  v2 = wave_max(v2);
  if (lane == 0) { pv_sh.red_v[wave] = v1; pv_sh.red_v2[wave] = v2; }
  __syncthreads();
  double r1 = pv_sh.red_v[0], r2 = pv_sh.red_v2[0];
  for (int w = 1; w < PIV_WAVES; ++w) { r1 = fmax(r1, pv_sh.red_v[w]); r2 = fmax(r2, pv_sh.red_v2[w]); }
  __syncthreads();
  v1 = r1;
  v2 = r2;
}

CTP_DEV int block_argmax(double v, int idx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  if (lane == 0) { pv_sh.red_v[wave] = v; pv_sh.red_i[wave] = idx; }
  __syncthreads();
  double bv = pv_sh.red_v[0];
  int bi = pv_sh.red_i[0];
  for (int w = 1; w < PIV_WAVES; ++w) {
    double ov = pv_sh.red_v[w];
    int oi = pv_sh.red_i[w];
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  __syncthreads();
  return bi;
}

// max |a(i, col)| over uneliminated rows i in [nelim, p) \ {x1, x2} of the
// square and all rows of R: this thread's partial.
CTP_DEV double col_partial(const PivotArgs& g, int rc, int nelim, int col, int x1, int x2) {
  double v = 0.0;
  for (int i = nelim + threadIdx.x; i < g.p; i += PIV_THREADS)
    if (i != x1 && i != x2) v = fmax(v, fabs(lazy_a(g, i, col)));
  for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) v = fmax(v, fabs(lazy_r(g, rc, i, col)));
  return v;
}

// Symmetric interchange of positions a and b: rows then columns of the
// square (stored values, L rows of eliminated columns), the rows of the
// pending multiplier / pivot-column vectors, the columns of R, perm.
CTP_DEV void sym_swap(const PivotArgs& g, int a, int b) {
  if (a == b) return;
  const int p = g.p;
  for (int j = threadIdx.x; j < p; j += PIV_THREADS) {
    const double x = CM(g.T, a, j, g.lda), y = CM(g.T, b, j, g.lda);
    CM(g.T, a, j, g.lda) = y;
    CM(g.T, b, j, g.lda) = x;
  }
  const int ns = pv_sh.nslot;
  for (int s = threadIdx.x; s < ns; s += PIV_THREADS) {
    double x = lA(p, s, a);
    lA(p, s, a) = lA(p, s, b);
    lA(p, s, b) = x;
    x = wc(p, s, a);
    wc(p, s, a) = wc(p, s, b);
    wc(p, s, b) = x;
  }
  if (threadIdx.x == 0) {
    const int t = pv_perm[a];
    pv_perm[a] = pv_perm[b];
    pv_perm[b] = t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < p; i += PIV_THREADS) {
    const double x = CM(g.T, i, a, g.lda), y = CM(g.T, i, b, g.lda);
    CM(g.T, i, a, g.lda) = y;
    CM(g.T, i, b, g.lda) = x;
  }
  for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) {
    const double x = CM(g.R, i, a, g.ldr), y = CM(g.R, i, b, g.ldr);
    CM(g.R, i, a, g.ldr) = y;
    CM(g.R, i, b, g.ldr) = x;
  }
  __syncthreads();
}

enum { ACT_NONE = 0, ACT_ZERO, ACT_2X2, ACT_1X1, ACT_REJECT, ACT_PASS, ACT_STOP, ACT_FALLBACK };

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

CTP_DEV void pivot_decide_body(const PivotArgs& g) {
  DecideShared& sh = pv_sh;
  const int p = g.p;
  const int rc = min(g.r, RCACHE);

  PivState* st = g.st;
  if (threadIdx.x == 0) {
    sh.nelim = st->nelim;
    sh.m = st->m;
    sh.progress = st->progress;
    sh.done = st->done;
    sh.status = 0;
    sh.nslot = 0;
  }
  __syncthreads();
  if (sh.done) {
    // the previous apply consumed the last batch
    if (threadIdx.x == 0) st->nslot = 0;
    return;
  }
  for (int k = threadIdx.x; k < p; k += PIV_THREADS) {
    pv_perm[k] = g.perm[k];
    pv_piv[k] = g.piv[k];
    pv_d[2 * k] = g.d[2 * k];
    pv_d[2 * k + 1] = g.d[2 * k + 1];
  }
  __syncthreads();

  const double inv_u = 1.0 / g.u;
  bool batch_full = false;
  while (true) {
    const int nelim = sh.nelim;
    const int m = sh.m;
    if (nelim >= p || batch_full) break;
    int action = ACT_NONE;
    int t = -1;
    int mc = m;        // position the action applies to
    bool fb = false;   // root fallback step
    if (m >= p) {
      __syncthreads();
      if (threadIdx.x == 0) {
        if (!sh.progress) sh.action = g.root ? ACT_FALLBACK : ACT_STOP;
        else { sh.action = ACT_PASS; sh.progress = 0; sh.m = nelim; }
      }
      __syncthreads();
      if (sh.action == ACT_STOP) break;
      if (sh.action == ACT_PASS) continue;
      // A pass without progress in the last panel: eliminate the column at
      // nelim regardless of u (1x1 unless below small, else a 2x2 with the
      // next column if its determinant is safely nonzero, else zero).
      fb = true;
      const int k = nelim;
      const double akk = lazy_a(g, k, k);
      if (fabs(akk) >= g.small) {
        action = ACT_1X1;
        mc = k;
      } else if (k + 1 < p && det_ok(akk, lazy_a(g, k + 1, k), lazy_a(g, k + 1, k + 1), g.small)) {
        action = ACT_2X2;
        t = k;
        mc = k + 1;
      } else {
        action = ACT_ZERO;
        mc = k;
      }
      if (threadIdx.x == 0) sh.status |= ST_ROOT_FALLBACK;
    } else {
      double maxm = block_max(col_partial(g, rc, nelim, m, m, m));
      const double amm = lazy_a(g, m, m);
      const double colmax = fmax(fabs(amm), maxm);
      if (threadIdx.x == 0 && !isfinite(colmax)) sh.status |= ST_NONFINITE;
      if (colmax < g.small) {
        action = ACT_ZERO;
      } else if (m > nelim) {
        double v = -1.0;
        int idx = 0x7fffffff;
        for (int j = nelim + threadIdx.x; j < m; j += PIV_THREADS) {
          double x = fabs(lazy_a(g, m, j));
          if (x != x) x = -0.5;   // NaN: loses to any number, keeps t a valid index
          if (x > v) { v = x; idx = j; }
        }
        t = block_argmax(v, idx);
        double maxt = col_partial(g, rc, nelim, t, t, m);
        double maxm2 = col_partial(g, rc, nelim, m, t, m);
        block_max2(maxt, maxm2);
        const double att = lazy_a(g, t, t), atm = lazy_a(g, m, t);
        const double big = fmax(fmax(fabs(att), fabs(atm)), fabs(amm));
        bool ok = false;
        if (!(big < g.small)) {
          const double s = 1.0 / big;
          const double det1 = (atm * s) * atm;
          const double det0 = (amm * s) * att;
          const double det = det0 - det1;
          const double bound = fmax(fmax(g.small, fabs(det0) / 2.0), fabs(det1) / 2.0);
          if (fabs(det) > bound) {
            if (fmax(maxt, maxm2) < g.small) {
              ok = true;
            } else {
              const double f = s / fabs(det);
              const double gt = (f * fabs(amm)) * maxt + (f * fabs(atm)) * maxm2;
              const double gm = (f * fabs(atm)) * maxt + (f * fabs(att)) * maxm2;
              ok = (gt <= inv_u) && (gm <= inv_u);
            }
          }
        }
        if (ok) action = ACT_2X2;
      }
      if (action == ACT_NONE) {
        const double bound = g.u * maxm;
        action = (fabs(amm) >= bound) ? ACT_1X1 : ACT_REJECT;
      }
    }
    // after an elimination: the next candidate and the progress flag (a
    // fallback step restarts the pass and does not count as progress)
    const int next1 = fb ? nelim + 1 : m + 1;
    const int next2 = fb ? nelim + 2 : m + 2;
    const int prog = fb ? 0 : 1;
    // Every thread has read the values behind the decision before any
    // thread starts the interchanges and writes below: without this wait a
    // fast wave can swap rows that a slow wave is still reading, and the
    // waves then disagree on the action.
    __syncthreads();

    if (action == ACT_ZERO) {
      sym_swap(g, mc, nelim);
      const int k = nelim;
      for (int i = k + 1 + threadIdx.x; i < p; i += PIV_THREADS) CM(g.T, i, k, g.lda) = 0.0;
      for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) CM(g.R, i, k, g.ldr) = 0.0;
      __syncthreads();
      if (threadIdx.x == 0) {
        CM(g.T, k, k, g.lda) = 0.0;
        pv_piv[k] = PIV_ZERO;
        pv_d[2 * k] = 0.0;
        pv_d[2 * k + 1] = 0.0;
        sh.nelim = nelim + 1;
        sh.m = next1;
        sh.progress = prog;
        sh.status |= ST_ZERO_PIVOT;
      }
    } else if (action == ACT_2X2) {
      sym_swap(g, t, nelim);
      sym_swap(g, mc, nelim + 1);
      const int k = nelim;
      const int s0 = sh.nslot;
      const double a11 = lazy_a(g, k, k), a21 = lazy_a(g, k + 1, k);
      const double a22 = lazy_a(g, k + 1, k + 1);
      const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
      const double det = (a22 * s) * a11 - (a21 * s) * a21;
      const double f = s / det;
      const double i11 = f * a22, i21 = -(f * a21), i22 = f * a11;
      for (int i = k + 2 + threadIdx.x; i < p; i += PIV_THREADS) {
        const double w1 = lazy_a(g, i, k), w2 = lazy_a(g, i, k + 1);
        const double l1 = w1 * i11 + w2 * i21;
        const double l2 = w1 * i21 + w2 * i22;
        CM(g.T, i, k, g.lda) = l1;
        CM(g.T, i, k + 1, g.lda) = l2;
        lA(p, s0, i) = l1;
        lA(p, s0 + 1, i) = l2;
        wc(p, s0, i) = w1;
        wc(p, s0 + 1, i) = w2;
      }
      const double j11 = fabs(i11), j21 = fabs(i21), j22 = fabs(i22);
      for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) {
        const double x1 = lazy_r(g, rc, i, k), x2 = lazy_r(g, rc, i, k + 1);
        double l1, l2;
        if (g.abs_update) {
          l1 = x1 * j11 + x2 * j21;
          l2 = x1 * j21 + x2 * j22;
        } else {
          l1 = x1 * i11 + x2 * i21;
          l2 = x1 * i21 + x2 * i22;
        }
        CM(g.R, i, k, g.ldr) = l1;
        CM(g.R, i, k + 1, g.ldr) = l2;
        if (i < rc) {
          lR(p, rc, s0, i) = l1;
          lR(p, rc, s0 + 1, i) = l2;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        CM(g.T, k, k, g.lda) = a11;
        CM(g.T, k + 1, k, g.lda) = a21;
        CM(g.T, k + 1, k + 1, g.lda) = a22;
        pv_piv[k] = PIV_2X2_FIRST;
        pv_piv[k + 1] = PIV_2X2_SECOND;
        pv_d[2 * k] = a11;
        pv_d[2 * k + 1] = a21;
        pv_d[2 * k + 2] = a22;
        pv_d[2 * k + 3] = 0.0;
        sh.kind[s0] = 2;
        sh.kind[s0 + 1] = 3;
        sh.sk[s0] = k;
        sh.sk[s0 + 1] = k + 1;
        sh.nslot = s0 + 2;
        sh.nelim = nelim + 2;
        sh.m = next2;
        sh.progress = prog;
      }
    } else if (action == ACT_1X1) {
      sym_swap(g, mc, nelim);
      const int k = nelim;
      const int s0 = sh.nslot;
      const double dk = lazy_a(g, k, k);
      for (int i = k + 1 + threadIdx.x; i < p; i += PIV_THREADS) {
        const double w = lazy_a(g, i, k);
        const double l = w / dk;
        CM(g.T, i, k, g.lda) = l;
        lA(p, s0, i) = l;
        wc(p, s0, i) = w;
      }
      const double adk = fabs(dk);
      for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) {
        const double x = lazy_r(g, rc, i, k);
        const double l = g.abs_update ? x / adk : x / dk;
        CM(g.R, i, k, g.ldr) = l;
        if (i < rc) lR(p, rc, s0, i) = l;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        CM(g.T, k, k, g.lda) = dk;
        pv_piv[k] = PIV_1X1;
        pv_d[2 * k] = dk;
        pv_d[2 * k + 1] = 0.0;
        sh.kind[s0] = 1;
        sh.sk[s0] = k;
        sh.nslot = s0 + 1;
        sh.nelim = nelim + 1;
        sh.m = next1;
        sh.progress = prog;
      }
    } else {
      __syncthreads();
      if (threadIdx.x == 0) sh.m = m + 1;
    }
    __syncthreads();
    batch_full = sh.nslot >= NSLOT - 1;
  }
  __syncthreads();

  // Save the batch for the apply kernel and the loop state for the next launch.
  const int nslot = sh.nslot;
  for (int q = threadIdx.x; q < nslot * p; q += PIV_THREADS) g.wbuf[q] = pv_dyn[NSLOT * p + q];
  for (int k = threadIdx.x; k < p; k += PIV_THREADS) {
    g.perm[k] = pv_perm[k];
    g.piv[k] = pv_piv[k];
    g.d[2 * k] = pv_d[2 * k];
    g.d[2 * k + 1] = pv_d[2 * k + 1];
  }
  if (threadIdx.x == 0) {
    const bool finished = sh.nelim >= p || !batch_full;
    st->nelim = sh.nelim;
    st->m = sh.m;
    st->progress = sh.progress;
    st->done = finished;
    st->nslot = nslot;
    for (int s = 0; s < NSLOT; ++s) {
      st->slot_k[s] = sh.sk[s];
      st->slot_kind[s] = s < nslot ? sh.kind[s] : 0;
    }
    *g.nelim_out = sh.nelim;
    if (sh.status) atomicOr(g.status, sh.status);
  }
}

__global__ __launch_bounds__(PIV_THREADS) void pivot_decide_kernel(PivotArgs g) { pivot_decide_body(g); }

// ---------------------------------------------------------------------------
// apply: materialise the pending batch on the trailing square and on R
// ---------------------------------------------------------------------------

// One 64 x 64 tile b of the trailing square (tiles_a of them) or of R,
// thread t of 256: 4 consecutive rows x 4 columns.
CTP_DEV void pivot_apply_tile(const PivotArgs& g, int b, int t, int nslot, int nelim, const int* kind,
                              const int* sk) {
  const int p = g.p;
  const int nt = p - nelim;
  const int tw = (nt + APPLY_TILE - 1) / APPLY_TILE;
  const int tiles_a = tw * tw;
  bool in_r;
  int i0, j0;
  if (b < tiles_a) {
    in_r = false;
    i0 = nelim + (b % tw) * APPLY_TILE;
    j0 = nelim + (b / tw) * APPLY_TILE;
  } else {
    const int q = b - tiles_a;
    in_r = true;
    i0 = (q % ((g.r + APPLY_TILE - 1) / APPLY_TILE)) * APPLY_TILE;
    j0 = nelim + (q / ((g.r + APPLY_TILE - 1) / APPLY_TILE)) * APPLY_TILE;
  }
  const int rows_end = in_r ? g.r : p;
  double* X = in_r ? g.R : g.T;
  const int ldx = in_r ? g.ldr : g.lda;
  // thread: 4 consecutive rows x 4 columns (16 threads cover 64 rows)
  const int ib = i0 + (t % 16) * 4;
  const int jb = j0 + (t / 16) * 4;
  double v[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = ib + e, j = jb + c;
      v[c][e] = (i < rows_end && j < p) ? CM(X, i, j, ldx) : 0.0;
    }
  const bool absu = in_r && g.abs_update;
  for (int s = 0; s < nslot; ++s) {
    const int two = kind[s] == 2;
    double l1[4], l2[4], w1[4], w2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = min(ib + e, rows_end - 1);
      l1[e] = CM(X, i, sk[s], ldx);
      l2[e] = two ? CM(X, i, sk[s + 1], ldx) : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = min(jb + c, p - 1);
      w1[c] = g.wbuf[s * p + j];
      w2[c] = two ? g.wbuf[(s + 1) * p + j] : 0.0;
      if (absu) { w1[c] = fabs(w1[c]); w2[c] = fabs(w2[c]); }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (two) {
          const double upd = l1[e] * w1[c] + l2[e] * w2[c];
          v[c][e] = absu ? v[c][e] + upd : v[c][e] - upd;
        } else {
          const double prod = l1[e] * w1[c];
          v[c][e] = absu ? v[c][e] + prod : v[c][e] - prod;
        }
      }
    s += two;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = ib + e, j = jb + c;
      if (i < rows_end && j < p) CM(X, i, j, ldx) = v[c][e];
    }
}

CTP_DEV int pivot_apply_tiles(const PivotArgs& g, int nelim) {
  const int nt = g.p - nelim;
  if (nt <= 0) return 0;
  const int tw = (nt + APPLY_TILE - 1) / APPLY_TILE;
  return tw * tw + ((g.r + APPLY_TILE - 1) / APPLY_TILE) * tw;
}

__global__ __launch_bounds__(256) void pivot_apply_kernel(PivotArgs g) {
  __shared__ int kind[NSLOT], sk[NSLOT];
  __shared__ int s_nslot, s_nelim;
  const PivState* st = g.st;
  if (threadIdx.x == 0) {
    s_nslot = st->nslot;
    s_nelim = st->nelim;
  }
  if (threadIdx.x < NSLOT) {
    kind[threadIdx.x] = st->slot_kind[threadIdx.x];
    sk[threadIdx.x] = st->slot_k[threadIdx.x];
  }
  __syncthreads();
  const int nslot = s_nslot;
  if (nslot == 0) return;
  if ((int)blockIdx.x >= pivot_apply_tiles(g, s_nelim)) return;
  pivot_apply_tile(g, blockIdx.x, threadIdx.x, nslot, s_nelim, kind, sk);
}

// ---------------------------------------------------------------------------
// the whole search in one workgroup: decide, then the same workgroup
// applies the batch (four tiles at a time) -- for trapezoids small enough
// that one CU can sweep them, e.g. a compressed trapezoid with p <= 256.
// Same arithmetic, in the same order, as the decide / apply launches.
// ---------------------------------------------------------------------------

__shared__ int pw_kind[NSLOT], pw_sk[NSLOT], pw_info[3];

CTP_DEV void pivot_factor_wg_body(const PivotArgs& g) {
  pivot_init_body(g, threadIdx.x, PIV_THREADS);
  __syncthreads();
  const int rounds = g.p / (NSLOT - 1) + 2;
  for (int q = 0; q < rounds; ++q) {
    pivot_decide_body(g);
    __syncthreads();
    if (threadIdx.x == 0) {
      pw_info[0] = g.st->nslot;
      pw_info[1] = g.st->nelim;
      pw_info[2] = g.st->done;
    }
    if (threadIdx.x < NSLOT) {
      pw_kind[threadIdx.x] = g.st->slot_kind[threadIdx.x];
      pw_sk[threadIdx.x] = g.st->slot_k[threadIdx.x];
    }
    __syncthreads();
    const int nslot = pw_info[0], nelim = pw_info[1], done = pw_info[2];
    if (nslot > 0) {
      const int tiles = pivot_apply_tiles(g, nelim);
      for (int b = threadIdx.x / 256; b < tiles; b += PIV_THREADS / 256)
        pivot_apply_tile(g, b, threadIdx.x % 256, nslot, nelim, pw_kind, pw_sk);
    }
    __syncthreads();
    if (done || nslot == 0) break;
  }
}

__global__ __launch_bounds__(PIV_THREADS) void pivot_factor_wg_kernel(PivotArgs g) { pivot_factor_wg_body(g); }

// one workgroup per supernode of a batch
__global__ __launch_bounds__(PIV_THREADS) void pivot_factor_batch_kernel(const PivotArgs* __restrict__ args,
                                                                          int count) {
  if ((int)blockIdx.x >= count) return;
  const PivotArgs g = args[blockIdx.x];
  pivot_factor_wg_body(g);
}

size_t pivot_lds_bytes(int p, int r);

// ---------------------------------------------------------------------------
// batches: per-node descriptors and pivot-search arguments built on the
// device from the caller's ctp_node array
// ---------------------------------------------------------------------------

__global__ void batch_setup_kernel(const ctp_node* __restrict__ in, int count, int method, unsigned flags,
                                   double u, double small, double* panels, double* s, int* perm, int* piv,
                                   double* d, int* nelim, int* status, unsigned char* work,
                                   BatchNode* __restrict__ nodes, PivotArgs* __restrict__ pargs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const ctp_node c = in[i];
  const int r = c.n - c.p;
  BatchNode nd;
  nd.n = c.n;
  nd.p = c.p;
  nd.lda = c.lda;
  nd.lds = c.lds;
  nd.nchunks = relaxed_chunk_count(r);
  const int nt = (r + 127) / 128;
  nd.ntiles = (s && c.s_off >= 0) ? nt * (nt + 1) / 2 : 0;
  nd.tile_off = c.tile_off;
  nd.a = panels + c.a_off;
  nd.s = (s && c.s_off >= 0) ? s + c.s_off : nullptr;
  nd.perm = perm + c.out_off;
  nd.piv = piv + c.out_off;
  nd.d = d + 2 * c.out_off;
  nd.nelim = nelim + i;
  nd.status = status + i;
  nd.work = work + c.work_off;
  nodes[i] = nd;
  status[i] = 0;
  nelim[i] = 0;
  const Workspace ws = workspace_layout(c.n, c.p, method);
  PivotArgs g;
  g.p = c.p;
  g.T = nd.a;
  g.lda = c.lda;
  if (method == CTP_RESTRICTED) {
    g.r = 0;
    g.R = nullptr;
    g.ldr = 1;
    g.abs_update = 0;
  } else {
    g.r = c.p;
    g.R = reinterpret_cast<double*>(nd.work + ws.c_off);
    g.ldr = c.p;
    g.abs_update = method == CTP_STRICT;
  }
  g.root = (flags & CTP_FLAG_ROOT) ? 1 : 0;
  g.u = u;
  g.small = small;
  g.perm = nd.perm;
  g.piv = nd.piv;
  g.d = nd.d;
  g.nelim_out = nd.nelim;
  g.status = nd.status;
  g.st = reinterpret_cast<PivState*>(nd.work + ws.st_off);
  g.wbuf = reinterpret_cast<double*>(nd.work + ws.wb_off);
  pargs[i] = g;
}

size_t batch_header_bytes(int count) {
  return align_up((size_t)count * sizeof(BatchNode), 256) + align_up((size_t)count * sizeof(PivotArgs), 256) + 256;
}

int launch_batch_setup(int count, const ctp_node* in, int method, unsigned flags, double u, double small,
                       double* panels, double* s, int* perm, int* piv, double* d, int* nelim, int* status,
                       void* work, BatchNode** nodes_out, void** pargs_out, unsigned int** counter_out,
                       hipStream_t stream) {
  unsigned char* base = static_cast<unsigned char*>(work);
  BatchNode* nodes = reinterpret_cast<BatchNode*>(base);
  PivotArgs* pargs = reinterpret_cast<PivotArgs*>(base + align_up((size_t)count * sizeof(BatchNode), 256));
  unsigned int* counter = reinterpret_cast<unsigned int*>(
      base + align_up((size_t)count * sizeof(BatchNode), 256) + align_up((size_t)count * sizeof(PivotArgs), 256));
  batch_setup_kernel<<<(count + 127) / 128, 128, 0, stream>>>(in, count, method, flags, u, small, panels, s, perm,
                                                             piv, d, nelim, status, base, nodes, pargs);
  *nodes_out = nodes;
  *pargs_out = pargs;
  *counter_out = counter;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int launch_pivot_batch(int count, const void* pargs, int max_p, int max_r, hipStream_t stream) {
  const size_t lds = pivot_lds_bytes(max_p, max_r);
  if (max_p > CTP_MAX_P || lds + 16 * 1024 > 160 * 1024) return -2;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)pivot_factor_batch_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  pivot_factor_batch_kernel<<<count, PIV_THREADS, lds, stream>>>(static_cast<const PivotArgs*>(pargs), count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

size_t pivot_lds_bytes(int p, int r) {
  const int rc = r < RCACHE ? r : RCACHE;
  return (size_t)NSLOT * p * sizeof(double) * 2 + (size_t)NSLOT * rc * sizeof(double);
}

int launch_pivot_factor(int p, double* a11, int lda, int r, double* R, int ldr, int abs_update,
                        int root, int one_wg, double u, double small, int* perm, int* piv, double* d,
                        int* nelim, int* status, void* state, double* wbuf, hipStream_t stream) {
  PivotArgs g;
  g.p = p; g.T = a11; g.lda = lda; g.r = r; g.R = R; g.ldr = ldr;
  g.abs_update = abs_update; g.root = root; g.u = u; g.small = small;
  g.perm = perm; g.piv = piv; g.d = d; g.nelim_out = nelim; g.status = status;
  g.st = static_cast<PivState*>(state);
  g.wbuf = wbuf;
  const size_t lds = pivot_lds_bytes(p, r);
  if (p > CTP_MAX_P || lds + 16 * 1024 > 160 * 1024) return -2;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)pivot_decide_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  if (one_wg) {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)pivot_factor_wg_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    }
    pivot_factor_wg_kernel<<<1, PIV_THREADS, lds, stream>>>(g);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
  }
  const size_t sq = (size_t)p * p;
  const unsigned init_blocks = (unsigned)std::min<size_t>((sq + 255) / 256 + 1, 2048);
  pivot_init_kernel<<<init_blocks, 256, 0, stream>>>(g);
  const int tw = (p + APPLY_TILE - 1) / APPLY_TILE;
  const int apply_blocks = tw * tw + ((r + APPLY_TILE - 1) / APPLY_TILE) * tw;
  // every full batch holds at least NSLOT-1 eliminated columns
  const int rounds = p / (NSLOT - 1) + 2;
  for (int q = 0; q < rounds; ++q) {
    pivot_decide_kernel<<<1, PIV_THREADS, lds, stream>>>(g);
    if (apply_blocks > 0) pivot_apply_kernel<<<apply_blocks, 256, 0, stream>>>(g);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
