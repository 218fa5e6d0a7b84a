// Threshold partial pivoting on the whole panel with a grid-wide reduction
// per candidate pivot: the TPP baseline beside compressed pivoting.
//
// Section 2 states the pivot loop (Listing 1) with the tests (2.1) and
// (2.2) over every row of [A11; A21]; Section 2.1 describes its parallel
// form in which the rows are spread over the processes and every candidate
// needs a reduction of its column maxima over all of them (Variant B, the
// pattern Table 6.1 counts: one message per candidate per process).  Here
// the processes are workgroups: each owns a slice of the rows of A21, and
// every candidate costs one launch whose workgroups reduce their slice and
// whose last-arriving workgroup takes the decision.  No workgroup ever waits
// for another: the kernel boundary orders the steps, and an atomic ticket
// picks the deciding workgroup.
//
// The decisions and the arithmetic are those of the single-workgroup search
// (pivot.hip) and of the oracle, bit for bit (same readings: the candidate
// order, the partner search along row m, the 2x2 test of eq. (2.2), zero
// pivots, the root fallback, ties to the lowest index), with one change of
// representation: nothing moves.  The working copies of A11 (a full square,
// its lower triangle reflected) and of A21 keep their rows and columns in
// the original order; perm / pos map positions to variables and back, and a
// final kernel writes the panel in pivot order.
//
// Updates are delayed in batches of up to PIV_NSLOT - 1 eliminated columns
// (slots): an entry is read as its stored value minus the pending slots'
// products l_i * w_c in elimination order, which is exactly the value the
// eager right-looking loop holds.  A slot stores the pivot column's values
// w over the variables; a row's multiplier for a slot is stored in the
// eliminated column itself (L21 for the rows of A21).  When the batch is
// full the slots are applied to every uneliminated entry in the same order.
//
// One step (tpp_step_kernel, one launch per candidate):
//   every workgroup, on its rows of A21:
//     1. the multipliers of the slots the last decision added;
//     2. a zero pivot's column cleared;
//     3. a full batch applied to the uneliminated columns (the rows of the
//        square take part in this step only);
//     4. the candidate's column m and its partner column t scanned
//        (largest two |a| of each, NaN / infinity seen);
//   then the last-arriving workgroup:
//     5. merges the partial maxima with those of the rows of A11, which it
//        reads itself (the square's interchanges and multipliers are the
//        deciding workgroup's);
//     6. takes the decision (zero, 2x2, 1x1 or reject) and records it;
//     7. moves to the next candidate (new pass, end, or root fallback) and
//        finds the partner of the new candidate along its row.
// The host enqueues steps in chunks and reads the done flag between chunks.
//
// Arithmetic: contraction is off; every update is a rounded product then a
// rounded sum, in the oracle's order.

#include <algorithm>
#include <cstdio>

#include "common.h"

#pragma clang fp contract(off)

#include "threshold_tests.h"

namespace ctp {

constexpr int TPP_THREADS = 256;
constexpr int TPP_WAVES = TPP_THREADS / 64;
constexpr int TPP_ROWS = 64;   // rows of a workgroup
constexpr int TPP_BUCKETS = 64; // first level of the arrival count
constexpr int TPP_MAX_GROUPS = TPP_MAX_GROUPS_WS;
constexpr int TPP_NSLOT = PIV_NSLOT;
constexpr int TPP_PART = TPP_PART_WS;   // per group: v1, v2 of column m, v1, v2 of column t, two bad flags

struct TppState {
  int nelim, m, t, progress;       // m: candidate position; t: partner variable (-1: none)
  int done, finishing, ns, flush;  // ns: slots of the batch; flush: A21 rows apply them this step
  int mat_s0, mat_n, zero_var, scan;
  int ticket, status, pad0, pad1;
  int slot_var[TPP_NSLOT];
  int slot_kind[TPP_NSLOT];        // 1: 1x1, 2: first column of a 2x2, 3: second
  double slot_x[TPP_NSLOT][2];     // 1x1 {d, 0}; 2x2 first {i11, i21}, second {i21, i22}
};
static_assert(sizeof(TppState) <= PIV_STATE_BYTES, "TPP state does not fit its workspace slot");

struct TppArgs {
  int p, r;
  double* a;
  int lda;
  double* xt;      // A11 working square by variables, ld p
  double* xr;      // A21 working copy by variables, ld ldr
  int ldr;
  int* pos;        // variable -> position
  double* w;       // TPP_NSLOT x p: pivot-column values of the slots, by variable
  double* part;    // groups x TPP_PART
  int groups;      // workgroups of a step, TPP_ROWS rows each
  int root;
  double u, small;
  int* perm;       // position -> variable
  int* piv;
  double* d;
  int* nelim_out;
  int* status;
  TppState* st;
};

// ---------------------------------------------------------------------------
// lazily updated values
// ---------------------------------------------------------------------------

// Value of (row, column c) minus the pending slots [0, ns) given the row's
// multipliers l[] (unrolled over the slots, so l stays in registers).
CTP_DEV double tpp_lazy(double v, const double* l, const TppState& S, const double* w, int p, int c, int ns) {
#pragma unroll
  for (int s = 0; s < TPP_NSLOT; ++s) {
    if (s >= ns) break;
    const int kind = S.slot_kind[s];
    if (kind == 1) {
      const double prod = l[s] * w[s * p + c];
      v = v - prod;
    } else if (kind == 2 && s + 1 < TPP_NSLOT) {
      const double upd = l[s] * w[s * p + c] + l[s + 1] * w[(s + 1) * p + c];
      v = v - upd;
    }
  }
  return v;
}

// The flush's columns and their pivot-column values, staged in LDS by the
// workgroup (column j of the staged list is position nelim + j).
__shared__ int tp_fcol[CTP_MAX_P];
__shared__ double tp_fw[TPP_NSLOT][CTP_MAX_P];

// As tpp_lazy, with the pivot-column values of staged column j.
CTP_DEV double tpp_lazy_staged(double v, const double* l, const TppState& S, int j, int ns) {
#pragma unroll
  for (int s = 0; s < TPP_NSLOT; ++s) {
    if (s >= ns) break;
    const int kind = S.slot_kind[s];
    if (kind == 1) {
      const double prod = l[s] * tp_fw[s][j];
      v = v - prod;
    } else if (kind == 2 && s + 1 < TPP_NSLOT) {
      const double upd = l[s] * tp_fw[s][j] + l[s + 1] * tp_fw[s + 1][j];
      v = v - upd;
    }
  }
  return v;
}

// A full batch on the staged columns [j0, j1) of one row (stride ld
// between columns): eight columns' loads in flight at a time.
CTP_DEV void tpp_flush_row(double* __restrict__ row, size_t ld, const double* l, const TppState& S, int j0, int j1,
                           int ns) {
  constexpr int U = 8;
  for (int jb = j0; jb < j1; jb += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (jb + u < j1) v[u] = row[(size_t)tp_fcol[jb + u] * ld];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (jb + u < j1) row[(size_t)tp_fcol[jb + u] * ld] = tpp_lazy_staged(v[u], l, S, jb + u, ns);
  }
}

// Entry (i, c) of the A11 square, lazily (multipliers from the slots'
// eliminated columns of row i).
CTP_DEV double tpp_lazy_t(const TppArgs& g, const TppState& S, int i, int c, int ns) {
  double l[TPP_NSLOT];
#pragma unroll
  for (int s = 0; s < TPP_NSLOT; ++s) l[s] = s < ns ? g.xt[(size_t)S.slot_var[s] * g.p + i] : 0.0;
  return tpp_lazy(g.xt[(size_t)c * g.p + i], l, S, g.w, g.p, c, ns);
}

// ---------------------------------------------------------------------------
// init: working copies, outputs reset
// ---------------------------------------------------------------------------

__global__ void tpp_init_kernel(TppArgs g) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  const int p = g.p;
  for (size_t q = tid; q < (size_t)p * p; q += stride) {
    const int i = (int)(q % p), c = (int)(q / p);
    g.xt[q] = i >= c ? CM(g.a, i, c, g.lda) : CM(g.a, c, i, g.lda);
  }
  for (size_t q = tid; q < (size_t)g.r * p; q += stride) {
    const int i = (int)(q % g.r), c = (int)(q / g.r);
    g.xr[(size_t)c * g.ldr + i] = CM(g.a, p + i, c, g.lda);
  }
  if (tid < TPP_BUCKETS) reinterpret_cast<int*>(g.part + (size_t)TPP_MAX_GROUPS * TPP_PART)[tid] = 0;
  for (size_t k = tid; k < (size_t)p; k += stride) {
    g.perm[k] = (int)k;
    g.pos[k] = (int)k;
    g.piv[k] = PIV_DELAYED;
    g.d[2 * k] = 0.0;
    g.d[2 * k + 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// the deciding workgroup
// ---------------------------------------------------------------------------

__shared__ TppState tp_s;
__shared__ double tp_red[2][TPP_WAVES][2];
__shared__ int tp_redi[TPP_WAVES];
__shared__ int tp_flag[4];

// Workgroup merge of a Top2 (every thread returns the result).
CTP_DEV Top2 tpp_reduce_top2(Top2 t, int slot) {
  for (int off = 32; off > 0; off >>= 1) {
    const double o1 = __shfl_xor(t.v1, off, 64), o2 = __shfl_xor(t.v2, off, 64);
    top2_merge(t, o1, o2);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    tp_red[slot][wave][0] = t.v1;
    tp_red[slot][wave][1] = t.v2;
  }
  __syncthreads();
  Top2 r = top2_empty();
  for (int q = 0; q < TPP_WAVES; ++q) top2_merge(r, tp_red[slot][q][0], tp_red[slot][q][1]);
  r.bad = t.bad;
  __syncthreads();
  return r;
}

// OR of x over the workgroup (every thread returns it).
CTP_DEV int tpp_or(int x) {
  if (threadIdx.x == 0) tp_flag[0] = 0;
  __syncthreads();
  if (x) atomicOr(&tp_flag[0], x);
  __syncthreads();
  const int r = tp_flag[0];
  __syncthreads();
  return r;
}

CTP_DEV bool tpp_any(bool x) { return tpp_or(x ? 1 : 0) != 0; }

// Partner of the candidate at position m: the largest |a(m, j)| over the
// pending positions nelim..m-1 (row m, lazily), ties to the lowest position.
// Returns the partner's variable; sets *bad when a NaN / infinity was read.
CTP_DEV int tpp_partner(const TppArgs& g, const TppState& S, int m, int ns, bool* bad) {
  const int vm = g.perm[m];
  double rv = -1.0;
  int ri = 0x7fffffff;
  bool b = false;
  for (int j = S.nelim + (int)threadIdx.x; j < m; j += TPP_THREADS) {
    double x = fabs(tpp_lazy_t(g, S, vm, g.perm[j], ns));
    b |= nonfinite(x);
    if (x != x) x = -0.5;   // NaN: loses to any number, keeps t a valid index
    if (x > rv) {
      rv = x;
      ri = j;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(rv, off, 64);
    const int oi = __shfl_xor(ri, off, 64);
    if (pv_better(ov, oi, rv, ri)) {
      rv = ov;
      ri = oi;
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    tp_red[0][wave][0] = rv;
    tp_redi[wave] = ri;
  }
  __syncthreads();
  double bv = tp_red[0][0][0];
  int bi = tp_redi[0];
  for (int q = 1; q < TPP_WAVES; ++q)
    if (pv_better(tp_red[0][q][0], tp_redi[q], bv, bi)) {
      bv = tp_red[0][q][0];
      bi = tp_redi[q];
    }
  __syncthreads();
  *bad = tpp_any(b);
  return g.perm[bi];
}

enum { TPP_NONE = 0, TPP_ZERO, TPP_2X2, TPP_1X1, TPP_REJECT };

// Symmetric interchange of positions a and b (bookkeeping only).
CTP_DEV void tpp_swap(const TppArgs& g, int a, int b) {
  if (a == b) return;
  const int va = g.perm[a], vb = g.perm[b];
  g.perm[a] = vb;
  g.perm[b] = va;
  g.pos[va] = b;
  g.pos[vb] = a;
}

// Records an elimination at position nelim: interchanges, D, the slot(s)
// and the multipliers of the A11 rows; the A21 rows follow in the next
// step (mat / zero_var).  vt: first column of a 2x2 (-1 otherwise), vm: the
// 1x1 / zero / second column.  ns: slots pending on A11.
CTP_DEV void tpp_record(const TppArgs& g, TppState& S, int action, int vt, int vm, double d1, double d21, double d2,
                        int& ns) {
  const int p = g.p, k = S.nelim;
  const bool two = action == TPP_2X2;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (two) {
      tpp_swap(g, g.pos[vt], k);
      tpp_swap(g, g.pos[vm], k + 1);
    } else {
      tpp_swap(g, g.pos[vm], k);
    }
  }
  __threadfence_block();
  __syncthreads();
  const int first = k + (two ? 2 : 1);
  double i11 = 0.0, i21 = 0.0, i22 = 0.0;
  if (two) inverse_2x2(d1, d21, d2, i11, i21, i22);
  // the rows below the pivot: pivot-column values (w) and multipliers
  for (int j = first + (int)threadIdx.x; j < p; j += TPP_THREADS) {
    const int vi = g.perm[j];
    if (action == TPP_ZERO) {
      g.xt[(size_t)vm * p + vi] = 0.0;
    } else if (!two) {
      const double w = tpp_lazy_t(g, S, vi, vm, ns);
      g.w[ns * p + vi] = w;
      g.xt[(size_t)vm * p + vi] = w / d1;
    } else {
      const double w1 = tpp_lazy_t(g, S, vi, vt, ns);
      const double w2 = tpp_lazy_t(g, S, vi, vm, ns);
      g.w[ns * p + vi] = w1;
      g.w[(ns + 1) * p + vi] = w2;
      g.xt[(size_t)vt * p + vi] = w1 * i11 + w2 * i21;
      g.xt[(size_t)vm * p + vi] = w1 * i21 + w2 * i22;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (action == TPP_ZERO) {
      g.xt[(size_t)vm * p + vm] = 0.0;
      g.piv[k] = PIV_ZERO;
      g.d[2 * k] = 0.0;
      g.d[2 * k + 1] = 0.0;
      S.zero_var = vm;
      S.status |= ST_ZERO_PIVOT;
    } else if (!two) {
      g.xt[(size_t)vm * p + vm] = d1;
      g.piv[k] = PIV_1X1;
      g.d[2 * k] = d1;
      g.d[2 * k + 1] = 0.0;
      S.slot_kind[ns] = 1;
      S.slot_var[ns] = vm;
      S.slot_x[ns][0] = d1;
      S.slot_x[ns][1] = 0.0;
      S.mat_s0 = ns;
      S.mat_n = 1;
    } else {
      g.xt[(size_t)vt * p + vt] = d1;
      g.xt[(size_t)vt * p + vm] = d21;
      g.xt[(size_t)vm * p + vm] = d2;
      g.piv[k] = PIV_2X2_FIRST;
      g.piv[k + 1] = PIV_2X2_SECOND;
      g.d[2 * k] = d1;
      g.d[2 * k + 1] = d21;
      g.d[2 * k + 2] = d2;
      g.d[2 * k + 3] = 0.0;
      S.slot_kind[ns] = 2;
      S.slot_var[ns] = vt;
      S.slot_x[ns][0] = i11;
      S.slot_x[ns][1] = i21;
      S.slot_kind[ns + 1] = 3;
      S.slot_var[ns + 1] = vm;
      S.slot_x[ns + 1][0] = i21;
      S.slot_x[ns + 1][1] = i22;
      S.mat_s0 = ns;
      S.mat_n = 2;
    }
  }
  __syncthreads();
  if (action != TPP_ZERO) ns += two ? 2 : 1;
}

// Steps 5-7 of the module comment.  S is the workgroup's copy of the state.
CTP_DEV void tpp_decide(const TppArgs& g) {
  TppState& S = tp_s;
  const int p = g.p;
  // the previous step consumed mat / zero / flush; after a flush the batch
  // is empty (the grid applied it to the square and to A21)
  if (threadIdx.x == 0) {
    if (S.flush) {
      S.ns = 0;
      for (int s = 0; s < TPP_NSLOT; ++s) S.slot_kind[s] = 0;
    }
    S.flush = 0;
    S.mat_n = 0;
    S.zero_var = -1;
    S.ticket = 0;
  }
  __syncthreads();
  if (S.finishing) {
    if (threadIdx.x == 0) {
      S.done = 1;
      S.scan = 0;
    }
    __syncthreads();
    return;
  }
  int ns = S.ns;
  int action = TPP_NONE;
  int vt = -1, vm = -1;
  double d1 = 0.0, d21 = 0.0, d2 = 0.0;
  bool fb = false;
  bool bad = false;
  const double inv_u = 1.0 / g.u;
  if (S.scan) {
    vm = g.perm[S.m];
    vt = S.t;
    // partial maxima of the A21 rows
    Top2 cmr = top2_empty(), ctr = top2_empty();
    for (int q = threadIdx.x; q < g.groups; q += TPP_THREADS) {
      const double* pt = g.part + (size_t)q * TPP_PART;
      top2_merge(cmr, pt[0], pt[1]);
      top2_merge(ctr, pt[2], pt[3]);
      cmr.bad |= pt[4] != 0.0;
      ctr.bad |= pt[5] != 0.0;
    }
    // the rows of the square: column m over rows other than m, column t
    // over rows other than t
    for (int j = S.nelim + (int)threadIdx.x; j < p; j += TPP_THREADS) {
      const int vi = g.perm[j];
      if (vi != vm) top2_insert(cmr, fabs(tpp_lazy_t(g, S, vi, vm, ns)));
      if (vt >= 0 && vi != vt) top2_insert(ctr, fabs(tpp_lazy_t(g, S, vi, vt, ns)));
    }
    const Top2 cm = tpp_reduce_top2(cmr, 0);
    const Top2 ct = tpp_reduce_top2(ctr, 1);
    const double amm = tpp_lazy_t(g, S, vm, vm, ns);
    // column t counts as read (for the non-finite status) only where the
    // 2x2 test needs its maximum, as in the one-workgroup search
    const int anybad = tpp_or((cm.bad ? 1 : 0) | (ct.bad ? 2 : 0));
    const bool tbad = (anybad & 2) != 0;
    bad = (anybad & 1) != 0 || nonfinite(amm);
    const double colmax = fmax(fabs(amm), top2_max(cm));
    if (colmax < g.small) {
      action = TPP_ZERO;
    } else if (vt >= 0) {
      const double att = tpp_lazy_t(g, S, vt, vt, ns);
      const double atm = tpp_lazy_t(g, S, vm, vt, ns);    // column t, row m
      const double xtm = tpp_lazy_t(g, S, vt, vm, ns);    // column m, row t
      bad |= nonfinite(att);
      const double maxt = top2_excluding(ct, fabs(atm));
      const double maxm2 = top2_excluding(cm, fabs(xtm));
      if (!reject_2x2_early(att, atm, amm, maxm2, g.small, inv_u)) bad |= tbad;
      if (accept_2x2(att, atm, amm, maxt, maxm2, g.small, inv_u)) {
        action = TPP_2X2;
        d1 = att;
        d21 = atm;
        d2 = amm;
      }
    }
    if (action == TPP_NONE) {
      const double bound = g.u * top2_max(cm);
      action = fabs(amm) >= bound ? TPP_1X1 : TPP_REJECT;
      d1 = amm;
    }
    if (bad && threadIdx.x == 0) S.status |= ST_NONFINITE;
    __syncthreads();
  }
  for (;;) {
    if (action == TPP_REJECT) {
      if (threadIdx.x == 0) S.m = S.m + 1;
    } else if (action != TPP_NONE) {
      const int old_nelim = S.nelim;
      tpp_record(g, S, action, action == TPP_2X2 ? vt : -1, vm, d1, d21, d2, ns);
      const int width = action == TPP_2X2 ? 2 : 1;
      if (threadIdx.x == 0) {
        S.m = (fb ? old_nelim : S.m) + width;
        S.nelim = old_nelim + width;
        S.progress = fb ? 0 : 1;
        S.ns = ns;
      }
      __syncthreads();
      // a full batch goes onto every uneliminated entry in the next step;
      // until then the square is still read lazily with all its slots
      if (ns >= TPP_NSLOT - 1 && threadIdx.x == 0) S.flush = 1;
    }
    __syncthreads();
    action = TPP_NONE;
    fb = false;
    // the next candidate
    if (S.nelim >= p) break;
    if (S.m >= p) {
      if (S.progress) {
        __syncthreads();   // every thread has read m and progress before they change
        if (threadIdx.x == 0) {
          S.progress = 0;
          S.m = S.nelim;
        }
        __syncthreads();
      } else if (!g.root) {
        break;
      } else {
        // root fallback at position nelim (Section 1: the final supernode
        // eliminates every column)
        fb = true;
        const int k = S.nelim;
        vm = g.perm[k];
        const double akk = tpp_lazy_t(g, S, vm, vm, ns);
        if (fabs(akk) >= g.small) {
          action = TPP_1X1;
          d1 = akk;
        } else if (k + 1 < p) {
          const int vn = g.perm[k + 1];
          const double a21 = tpp_lazy_t(g, S, vn, vm, ns);
          const double a22 = tpp_lazy_t(g, S, vn, vn, ns);
          if (det_ok(akk, a21, a22, g.small)) {
            action = TPP_2X2;
            vt = vm;
            vm = vn;
            d1 = akk;
            d21 = a21;
            d2 = a22;
          }
        }
        if (action == TPP_NONE) action = TPP_ZERO;
        if (threadIdx.x == 0) S.status |= ST_ROOT_FALLBACK;
        __syncthreads();
        continue;
      }
    }
    // a candidate to test: its partner, then a scan in the next step
    const int m = S.m;
    int t = -1;
    if (m > S.nelim) {
      bool pb = false;
      t = tpp_partner(g, S, m, ns, &pb);
      if (pb && threadIdx.x == 0) S.status |= ST_NONFINITE;
    }
    if (threadIdx.x == 0) {
      S.t = t;
      S.scan = 1;
    }
    __syncthreads();
    return;
  }
  // end of the loop: the pending batch still has to reach the delayed
  // columns (in the finishing step)
  if (threadIdx.x == 0) {
    if (ns > 0) S.flush = 1;
    S.finishing = 1;
    S.scan = 0;
  }
  __syncthreads();
}

// First candidate and its partner (one workgroup).
__global__ __launch_bounds__(TPP_THREADS) void tpp_start_kernel(TppArgs g) {
  TppState& S = tp_s;
  if (threadIdx.x == 0) {
    S = TppState{};
    S.t = -1;
    S.zero_var = -1;
    S.m = g.p >= 2 ? 1 : 0;
    S.progress = 1;
    S.done = g.p == 0;
    S.scan = g.p > 0;
  }
  __syncthreads();
  if (g.p >= 2) {
    bool pb = false;
    const int t = tpp_partner(g, S, 1, 0, &pb);
    if (threadIdx.x == 0) {
      S.t = t;
      if (pb) S.status |= ST_NONFINITE;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *g.st = S;
    *g.nelim_out = 0;
  }
}

// ---------------------------------------------------------------------------
// one step
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(TPP_THREADS) void tpp_step_kernel(TppArgs g) {
  TppState& S = tp_s;
  if (threadIdx.x == 0) S = *g.st;
  __syncthreads();
  if (S.done) return;
  const int p = g.p;
  // 64 rows per workgroup, one per lane: those of A21, then (for a batch)
  // those of the square.  The four waves share the rows and split a
  // batch's columns; the scan's two columns go to waves 0 and 1.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ns = S.ns;                          // slots after this step's materialisation
  const int nsc = S.flush ? 0 : ns;             // pending for the scan
  const int vm = S.scan ? g.perm[S.m] : -1, vt = S.scan ? S.t : -1;
  Top2 cm = top2_empty(), ct = top2_empty();
  const int q = p - S.nelim;   // uneliminated columns
  if (S.flush) {
    for (int j = threadIdx.x; j < q; j += TPP_THREADS) {
      const int c = g.perm[S.nelim + j];
      tp_fcol[j] = c;
      for (int s = 0; s < ns; ++s) tp_fw[s][j] = g.w[s * p + c];
    }
    __syncthreads();
  }
  const int qs = (q + TPP_WAVES - 1) / TPP_WAVES;   // this wave's share of the batch's columns
  const int qj0 = min(q, wave * qs), qj1 = min(q, qj0 + qs);
  // blocks of 64 rows, grid-strided (the loop is uniform in the workgroup)
  for (int base = blockIdx.x * TPP_ROWS; base < g.r + p; base += gridDim.x * TPP_ROWS) {
  const int i = base + lane;
  const bool rrow = i < g.r;
  if (i >= g.r && i < g.r + p) {
    // a row of the square: only the batch, on its uneliminated entries
    // (its multipliers were written when the slots were recorded)
    const int vi = i - g.r;
    if (S.flush && g.pos[vi] >= S.nelim) {
      double* row = g.xt + vi;
      double l[TPP_NSLOT];
#pragma unroll
      for (int s = 0; s < TPP_NSLOT; ++s) l[s] = s < ns ? row[(size_t)S.slot_var[s] * p] : 0.0;
      tpp_flush_row(row, p, l, S, qj0, qj1, ns);
    }
  }
  double l[TPP_NSLOT];
  double* row = g.xr + (rrow ? i : 0);
  const int ldr = g.ldr;
  // 1. multipliers of the new slot(s): every wave computes them (the same
  //    bits) from the eliminated columns' entries, wave 0 stores them there
  //    once every wave has read those entries
  double lv1 = 0.0, lv2 = 0.0;
  if (rrow) {
    // multipliers of the slots materialised in earlier steps
    const int nold = S.mat_n ? S.mat_s0 : ns;
#pragma unroll
    for (int s = 0; s < TPP_NSLOT; ++s) l[s] = s < nold ? row[(size_t)S.slot_var[s] * ldr] : 0.0;
    if (S.mat_n == 1) {
      const int s0 = S.mat_s0, v = S.slot_var[s0];
      const double x = tpp_lazy(row[(size_t)v * ldr], l, S, g.w, p, v, s0);
      lv1 = x / S.slot_x[s0][0];
#pragma unroll
      for (int s = 0; s < TPP_NSLOT; ++s)
        if (s == s0) l[s] = lv1;
    } else if (S.mat_n == 2) {
      const int s0 = S.mat_s0, v1 = S.slot_var[s0], v2 = S.slot_var[s0 + 1];
      const double x1 = tpp_lazy(row[(size_t)v1 * ldr], l, S, g.w, p, v1, s0);
      const double x2 = tpp_lazy(row[(size_t)v2 * ldr], l, S, g.w, p, v2, s0);
      const double i11 = S.slot_x[s0][0], i21 = S.slot_x[s0][1], i22 = S.slot_x[s0 + 1][1];
      lv1 = x1 * i11 + x2 * i21;
      lv2 = x1 * i21 + x2 * i22;
#pragma unroll
      for (int s = 0; s < TPP_NSLOT; ++s) {
        if (s == s0) l[s] = lv1;
        if (s == s0 + 1) l[s] = lv2;
      }
    }
  }
  if (S.mat_n) __syncthreads();
  if (rrow) {
    if (wave == 0 && S.mat_n) {
      row[(size_t)S.slot_var[S.mat_s0] * ldr] = lv1;
      if (S.mat_n == 2) row[(size_t)S.slot_var[S.mat_s0 + 1] * ldr] = lv2;
    }
    // 2. a zero pivot's column
    if (S.zero_var >= 0 && wave == 0) row[(size_t)S.zero_var * ldr] = 0.0;
    // 3. a full batch onto this wave's share of the uneliminated columns
    if (S.flush) tpp_flush_row(row, ldr, l, S, qj0, qj1, ns);
  }
  // the scan reads columns another wave may just have updated
  if (S.flush) __syncthreads();
  // 4. the candidate's columns
  if (rrow && S.scan) {
    if (wave == 0) top2_insert(cm, fabs(tpp_lazy(row[(size_t)vm * ldr], l, S, g.w, p, vm, nsc)));
    if (wave == 1 && vt >= 0) top2_insert(ct, fabs(tpp_lazy(row[(size_t)vt * ldr], l, S, g.w, p, vt, nsc)));
  }
  }
  if (S.scan && wave < 2) {
    // wave 0 holds column m, wave 1 column t: each merges its own lanes
    Top2 t = wave == 0 ? cm : ct;
    for (int off = 32; off > 0; off >>= 1) {
      const double o1 = __shfl_xor(t.v1, off, 64), o2 = __shfl_xor(t.v2, off, 64);
      top2_merge(t, o1, o2);
    }
    const bool b = __any(t.bad);
    if (lane == 0) {
      double* pt = g.part + (size_t)blockIdx.x * TPP_PART + 2 * wave;
      pt[0] = t.v1;
      pt[1] = t.v2;
      g.part[(size_t)blockIdx.x * TPP_PART + 4 + wave] = b ? 1.0 : 0.0;
    }
  }
  // the last workgroup to arrive decides: first the last of each of up to
  // TPP_BUCKETS buckets of workgroups, then the last of those.  The barrier
  // orders the workgroup's writes before thread 0's device-scope fence (one
  // fence per workgroup: on this GPU it writes back the XCD's L2).
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int nb = min(TPP_BUCKETS, (int)gridDim.x);
    const int bucket = blockIdx.x % nb;
    const int members = ((int)gridDim.x - bucket + nb - 1) / nb;
    int* cnt = reinterpret_cast<int*>(g.part + (size_t)TPP_MAX_GROUPS * TPP_PART);
    bool last = false;
    if (atomicAdd(&cnt[bucket], 1) == members - 1) {
      cnt[bucket] = 0;   // every member has arrived
      __threadfence();
      last = atomicAdd(&g.st->ticket, 1) == nb - 1;
    }
    tp_flag[1] = last;
  }
  __syncthreads();
  if (!tp_flag[1]) return;
  if (threadIdx.x == 0) __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) S.ticket = 0;
  __syncthreads();
  tpp_decide(g);
  if (threadIdx.x == 0) {
    if (S.status) atomicOr(g.status, S.status);
    S.status = 0;
    *g.nelim_out = S.nelim;
    *g.st = S;
  }
}

// ---------------------------------------------------------------------------
// finish: the panel in pivot order
// ---------------------------------------------------------------------------

__global__ void tpp_finish_kernel(TppArgs g) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  const int p = g.p;
  for (size_t q = tid; q < (size_t)p * p; q += stride) {
    const int k1 = (int)(q % p), k2 = (int)(q / p);
    if (k1 >= k2) CM(g.a, k1, k2, g.lda) = g.xt[(size_t)g.perm[k2] * p + g.perm[k1]];
  }
  for (size_t q = tid; q < (size_t)g.r * p; q += stride) {
    const int i = (int)(q % g.r), k = (int)(q / g.r);
    CM(g.a, p + i, k, g.lda) = g.xr[(size_t)g.perm[k] * g.ldr + i];
  }
}

int launch_tpp_grid(int n, int p, double* a, int lda, int root, double u, double small, int* perm, int* piv,
                    double* d, int* nelim, int* status, double* xt, int* pos, double* part, void* state,
                    double* wbuf, double* xr, int ldr, hipStream_t stream) {
  TppArgs g;
  g.p = p;
  g.r = n - p;
  g.a = a;
  g.lda = lda;
  g.xt = xt;
  g.xr = xr;
  g.ldr = ldr;
  g.pos = pos;
  g.w = wbuf;
  g.part = part;
  g.groups = std::max(1, std::min(TPP_MAX_GROUPS, (g.r + p + TPP_ROWS - 1) / TPP_ROWS));
  g.root = root;
  g.u = u;
  g.small = small;
  g.perm = perm;
  g.piv = piv;
  g.d = d;
  g.nelim_out = nelim;
  g.status = status;
  g.st = static_cast<TppState*>(state);
  const size_t work = (size_t)p * p + (size_t)g.r * p;
  const unsigned blocks = (unsigned)std::min<size_t>((work + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(tpp_init_kernel, dim3(blocks), dim3(256), 0, stream, g);
  hipLaunchKernelGGL(tpp_start_kernel, dim3(1), dim3(TPP_THREADS), 0, stream, g);
  // a pass tests every remaining column once; a pass without progress ends
  // the loop or (root) makes a fallback step: at most (p + 1) passes
  const long long max_steps = (long long)(p + 2) * (p + 2) + 16;
  long long steps = 0;
  int chunk = p + 32;
  for (;;) {
    for (int q = 0; q < chunk; ++q) hipLaunchKernelGGL(tpp_step_kernel, dim3(g.groups), dim3(TPP_THREADS), 0, stream, g);
    steps += chunk;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    int done = 0;
    e = hipMemcpyAsync(&done, &g.st->done, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    if (done) break;
    if (steps > max_steps) return CTP_ERR_HIP_BASE - (int)hipErrorUnknown;
    chunk = 64;
  }
  hipLaunchKernelGGL(tpp_finish_kernel, dim3(blocks), dim3(256), 0, stream, g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
