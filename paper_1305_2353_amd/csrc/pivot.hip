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

#include <type_traits>

#include "common.h"

#pragma clang fp contract(off)

#include "threshold_tests.h"

namespace ctp {

constexpr int PIV_MAX_THREADS = 1024;   // workgroup sizes 256, 512 or 1024 (template NT)
constexpr int PIV_MAX_WAVES = PIV_MAX_THREADS / 64;
constexpr int NSLOT = PIV_NSLOT;   // pending eliminated columns per batch
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

// LDS of the decide kernel.  Dynamic part (doubles): multipliers of A11
// rows lA[NSLOT][p], pivot-column values wc[NSLOT][p] (both by position),
// multipliers of the first rc rows of R lR[NSLOT][rc], and the two columns
// under test, colA and colB, each p + rc values (rows of the square by
// position, then the cached rows of R).  rc is as many R rows as fit.
constexpr int PIV_DYN_DOUBLES = 18432;   // 144 KiB

__host__ __device__ inline int pivot_rcache(int p) {
  const int fit = (PIV_DYN_DOUBLES - (2 * NSLOT + 2) * p) / (NSLOT + 2);
  const int rc = fit / 256 * 256;
  return rc < 1024 ? rc : 1024;
}

// Reductions over the workgroup: every thread keeps the two largest |a| of
// a column (values only: when the largest value occurs twice, excluding
// either row leaves it, so no row numbers are needed) and, in the first
// pass, the largest |a(m, j)| with its column.  Waves merge by shuffles,
// then each wave's result goes to one of two alternating slots in LDS, so
// one barrier per reduction suffices (the slot written by reduction k + 2
// was last read before everybody reached reduction k + 1).  The scalars the
// decision needs besides the maxima travel in the same slot.
struct DecideShared {
  double v1[2][PIV_MAX_WAVES], v2[2][PIV_MAX_WAVES], rv[2][PIV_MAX_WAVES];
  int ri[2][PIV_MAX_WAVES];
  double sc[2][3];
  int nelim, m, progress, done, status;
  int kind[NSLOT];
  int sk[NSLOT];
};

HIP_DYNAMIC_SHARED(double, pv_dyn)
__shared__ DecideShared pv_sh;
__shared__ double pv_d[2 * CTP_MAX_P];
__shared__ int pv_perm[CTP_MAX_P];
__shared__ int pv_piv[CTP_MAX_P];

// Index helpers (the arrays are always named directly, so every access is
// an LDS access: no generic pointers into LDS).
CTP_DEV int lA(int p, int s, int i) { return s * p + i; }
CTP_DEV int wc(int p, int s, int j) { return NSLOT * p + s * p + j; }
CTP_DEV int lR(int p, int rc, int s, int i) { return 2 * NSLOT * p + s * rc + i; }
CTP_DEV int colbuf(int p, int rc, int c) { return 2 * NSLOT * p + NSLOT * rc + c * (p + rc); }

// Lazily updated entry (i, j) of the square: the stored value minus the
// pending updates of the ns slots of this batch.
CTP_DEV double lazy_a_from(const PivotArgs& g, int ns, int i, int j, double v) {
  const int p = g.p;
  for (int s = 0; s < ns; ++s) {
    if (pv_sh.kind[s] == 1) {
      const double prod = pv_dyn[lA(p, s, i)] * pv_dyn[wc(p, s, j)];
      v = v - prod;
    } else {
      const double upd = pv_dyn[lA(p, s, i)] * pv_dyn[wc(p, s, j)] + pv_dyn[lA(p, s + 1, i)] * pv_dyn[wc(p, s + 1, j)];
      v = v - upd;
      ++s;
    }
  }
  return v;
}

// Multipliers of R rows: the first rc rows keep theirs in LDS, the others
// read them from the eliminated columns of R.  The two kinds of rows go
// through separate loops (for_r_rows), so an access is always either an LDS
// or a global access, never a pointer that could be both.
template <bool CACHED>
CTP_DEV double r_mult(const PivotArgs& g, int rc, int s, int i) {
  if (CACHED) return pv_dyn[lR(g.p, rc, s, i)];
  return CM(g.R, i, pv_sh.sk[s], g.ldr);
}

template <bool CACHED>
CTP_DEV double lazy_r_from(const PivotArgs& g, int ns, int rc, int i, int j, double v) {
  const int p = g.p;
  for (int s = 0; s < ns; ++s) {
    if (pv_sh.kind[s] == 1) {
      const double lr = r_mult<CACHED>(g, rc, s, i);
      const double w = pv_dyn[wc(p, s, j)];
      if (g.abs_update) {
        const double prod = lr * fabs(w);
        v = v + prod;
      } else {
        const double prod = lr * w;
        v = v - prod;
      }
    } else {
      const double l1 = r_mult<CACHED>(g, rc, s, i), l2 = r_mult<CACHED>(g, rc, s + 1, i);
      const double w1 = pv_dyn[wc(p, s, j)], w2 = pv_dyn[wc(p, s + 1, j)];
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

CTP_DEV double lazy_a(const PivotArgs& g, int ns, int i, int j) {
  return lazy_a_from(g, ns, i, j, CM(g.T, i, j, g.lda));
}

template <bool CACHED>
CTP_DEV double lazy_r(const PivotArgs& g, int ns, int rc, int i, int j) {
  return lazy_r_from<CACHED>(g, ns, rc, i, j, CM(g.R, i, j, g.ldr));
}

// This thread's rows of R: rows i = tid (mod NT), the cached ones (i < rc)
// first.  Every loop that needs a row to stay with one thread uses this.
template <int NT, typename F>
CTP_DEV void for_r_rows(int rc, int r, F&& f) {
  for (int i = threadIdx.x; i < rc; i += NT) f(i, std::true_type{});
  for (int i = rc + threadIdx.x; i < r; i += NT) f(i, std::false_type{});
}


// The first entries a thread reads in a pass, loaded together before any is
// used, so that one memory latency covers them (the scans below would
// otherwise wait for them one loop after another): its first row of the
// square (nelim + tid) and its first row of R (tid, or rc + tid when
// tid >= rc, as for_r_rows visits them) in column `col`, and, for the
// partner search, entry (m, nelim + tid).
struct ScanPre {
  bool ht, hr;
  int ir;
  double xt, xr;
};

template <int NT>
CTP_DEV ScanPre scan_preload(const PivotArgs& g, int rc, int nelim, int col) {
  ScanPre q;
  const int it = nelim + threadIdx.x;
  q.ir = (int)threadIdx.x < rc ? (int)threadIdx.x : rc + (int)threadIdx.x;
  q.ht = it < g.p && it != col;
  q.hr = q.ir < g.r;
  q.xt = q.ht ? CM(g.T, it, col, g.lda) : 0.0;
  q.xr = q.hr ? CM(g.R, q.ir, col, g.ldr) : 0.0;
  return q;
}

// This thread's share of column `col` of the uneliminated trapezoid: rows
// nelim..p-1 of the square except row `col`, then every row of R, in the
// order of the plain loops (square rows nelim + tid + k NT; cached R rows
// tid + k NT, then rc + tid + k NT).  The values of the square's rows and
// of the cached R rows are kept in the column buffer at `cb`.
template <int NT>
CTP_DEV void col_scan(const PivotArgs& g, int ns, int rc, int nelim, int col, int cb, const ScanPre& q, Top2& t) {
  const int it = nelim + threadIdx.x;
  if (q.ht) {
    const double x = lazy_a_from(g, ns, it, col, q.xt);
    pv_dyn[cb + it] = x;
    top2_insert(t, fabs(x));
  }
  for (int i = it + NT; i < g.p; i += NT) {
    if (i == col) continue;
    const double x = lazy_a(g, ns, i, col);
    pv_dyn[cb + i] = x;
    top2_insert(t, fabs(x));
  }
  if ((int)threadIdx.x < rc) {
    if (q.hr) {
      const double x = lazy_r_from<true>(g, ns, rc, q.ir, col, q.xr);
      pv_dyn[cb + g.p + q.ir] = x;
      top2_insert(t, fabs(x));
    }
    for (int i = q.ir + NT; i < rc; i += NT) {
      const double x = lazy_r<true>(g, ns, rc, i, col);
      pv_dyn[cb + g.p + i] = x;
      top2_insert(t, fabs(x));
    }
    for (int i = rc + threadIdx.x; i < g.r; i += NT) top2_insert(t, fabs(lazy_r<false>(g, ns, rc, i, col)));
  } else {
    if (q.hr) top2_insert(t, fabs(lazy_r_from<false>(g, ns, rc, q.ir, col, q.xr)));
    for (int i = q.ir + NT; i < g.r; i += NT) top2_insert(t, fabs(lazy_r<false>(g, ns, rc, i, col)));
  }
}

// Cross-lane moves of the reductions.  Within a row of 16 lanes the
// butterfly uses DPP (quad permutes for lane distance 1 and 2, then the
// half-row and row mirrors, which pair disjoint groups once the quads, then
// the half-rows, agree); across rows, LDS permutes; the workgroup result is
// broadcast with readfirstlane.
constexpr int DPP_XOR1 = 0xB1;          // quad_perm(1, 0, 3, 2)
constexpr int DPP_XOR2 = 0x4E;          // quad_perm(2, 3, 0, 1)
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <- 7 - i within each 8 lanes
constexpr int DPP_MIRROR = 0x140;       // lane i <- 15 - i within each 16 lanes

template <int CTRL>
CTP_DEV int dpp_int(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
CTP_DEV double dpp_dbl(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)dpp_int<CTRL>((int)(unsigned)(b & 0xffffffffull));
  const unsigned hi = (unsigned)dpp_int<CTRL>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

CTP_DEV double first_lane_dbl(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffull));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <bool ARG>
CTP_DEV void red_merge(Top2& t, double& rv, int& ri, double o1, double o2, double ov, int oi) {
  top2_merge(t, o1, o2);
  if (ARG && pv_better(ov, oi, rv, ri)) {
    rv = ov;
    ri = oi;
  }
}

template <bool ARG, int CTRL>
CTP_DEV void red_round_dpp(Top2& t, double& rv, int& ri) {
  const double o1 = dpp_dbl<CTRL>(t.v1), o2 = dpp_dbl<CTRL>(t.v2);
  const double ov = ARG ? dpp_dbl<CTRL>(rv) : 0.0;
  const int oi = ARG ? dpp_int<CTRL>(ri) : 0;
  red_merge<ARG>(t, rv, ri, o1, o2, ov, oi);
}

template <bool ARG>
CTP_DEV void red_round_shfl(Top2& t, double& rv, int& ri, int off) {
  const double o1 = __shfl_xor(t.v1, off, 64), o2 = __shfl_xor(t.v2, off, 64);
  const double ov = ARG ? __shfl_xor(rv, off, 64) : 0.0;
  const int oi = ARG ? __shfl_xor(ri, off, 64) : 0;
  red_merge<ARG>(t, rv, ri, o1, o2, ov, oi);
}

// Workgroup reduction of a column's two largest (and, with ARG, of the
// partner search); the caller reads the slot's scalars, then flips the slot.
template <int NT, bool ARG>
CTP_DEV void reduce_pass(Top2& t, double& rv, int& ri, int slot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  red_round_dpp<ARG, DPP_XOR1>(t, rv, ri);
  red_round_dpp<ARG, DPP_XOR2>(t, rv, ri);
  red_round_dpp<ARG, DPP_HALF_MIRROR>(t, rv, ri);
  red_round_dpp<ARG, DPP_MIRROR>(t, rv, ri);
  red_round_shfl<ARG>(t, rv, ri, 16);
  red_round_shfl<ARG>(t, rv, ri, 32);
  if (lane == 0) {
    pv_sh.v1[slot][wave] = t.v1;
    pv_sh.v2[slot][wave] = t.v2;
    if (ARG) {
      pv_sh.rv[slot][wave] = rv;
      pv_sh.ri[slot][wave] = ri;
    }
  }
  __syncthreads();
  // lane w of every wave takes wave w's partial, the same butterfly over the
  // first NT / 64 lanes merges them, lane 0's result is broadcast
  constexpr int NW = NT / 64;
  Top2 u = top2_empty();
  double bv = -1.0;
  int bi = 0x7fffffff;
  if (lane < NW) {
    u.v1 = pv_sh.v1[slot][lane];
    u.v2 = pv_sh.v2[slot][lane];
    if (ARG) {
      bv = pv_sh.rv[slot][lane];
      bi = pv_sh.ri[slot][lane];
    }
  }
  if constexpr (NW > 1) red_round_dpp<ARG, DPP_XOR1>(u, bv, bi);
  if constexpr (NW > 2) red_round_dpp<ARG, DPP_XOR2>(u, bv, bi);
  if constexpr (NW > 4) red_round_dpp<ARG, DPP_HALF_MIRROR>(u, bv, bi);
  if constexpr (NW > 8) red_round_dpp<ARG, DPP_MIRROR>(u, bv, bi);
  t.v1 = first_lane_dbl(u.v1);
  t.v2 = first_lane_dbl(u.v2);
  if (ARG) {
    rv = first_lane_dbl(bv);
    ri = __builtin_amdgcn_readfirstlane(bi);
  }
}

// Symmetric interchanges (a0, b0) then (a1, b1): afterwards position x
// holds what was at swap_src(x).  A single interchange passes a1 = b1.
struct SwapPlan {
  int x[4];
  int src[4];
};

CTP_DEV int swap_src(int a0, int b0, int a1, int b1, int x) {
  const int y = x == a1 ? b1 : x == b1 ? a1 : x;
  return y == a0 ? b0 : y == b0 ? a0 : y;
}

CTP_DEV SwapPlan swap_plan(int a0, int b0, int a1, int b1) {
  SwapPlan s;
  s.x[0] = a0;
  s.x[1] = b0;
  s.x[2] = a1;
  s.x[3] = b1;
#pragma unroll
  for (int q = 0; q < 4; ++q) s.src[q] = swap_src(a0, b0, a1, b1, s.x[q]);
  return s;
}

// Moves the entries at the plan's positions of one line (a row or a column,
// reached through ld / st): every value is read before any is written.
template <typename V, typename St>
CTP_DEV void permute_store(const SwapPlan& s, const V (&v)[4], St&& st) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (s.src[q] == s.x[q]) continue;
    V val = v[3];
#pragma unroll
    for (int e = 2; e >= 0; --e)
      if (s.src[q] == s.x[e]) val = v[e];
    st(s.x[q], val);
  }
}

template <typename V, typename Ld, typename St>
CTP_DEV void permute_line(const SwapPlan& s, Ld&& ld, St&& st) {
  V v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = ld(s.x[q]);
  permute_store<V>(s, v, st);
}

// Row half of the interchanges: the rows of the square (stored values and
// the L rows of eliminated columns), the rows of the pending multiplier and
// pivot-column vectors, perm.  The column half runs inside the elimination
// loops, by the thread that owns the row.
template <int NT>
CTP_DEV void swap_rows(const PivotArgs& g, int ns, const SwapPlan& s) {
  const int p = g.p;
  for (int j = threadIdx.x; j < p; j += NT)
    permute_line<double>(s, [&](int x) { return CM(g.T, x, j, g.lda); },
                         [&](int x, double v) { CM(g.T, x, j, g.lda) = v; });
  for (int q = threadIdx.x; q < ns; q += NT) {
    permute_line<double>(s, [&](int x) { return pv_dyn[lA(p, q, x)]; },
                         [&](int x, double v) { pv_dyn[lA(p, q, x)] = v; });
    permute_line<double>(s, [&](int x) { return pv_dyn[wc(p, q, x)]; },
                         [&](int x, double v) { pv_dyn[wc(p, q, x)] = v; });
  }
  if (threadIdx.x == 0)
    permute_line<int>(s, [&](int x) { return pv_perm[x]; }, [&](int x, int v) { pv_perm[x] = v; });
}

enum { ACT_NONE = 0, ACT_ZERO, ACT_2X2, ACT_1X1, ACT_REJECT };

// Before pass B: is the pair (partner t = ri, candidate m) rejected by the
// 2x2 test whatever column t holds?  Every thread evaluates the same bits:
// a_tt lazily from the square, |a_tm| = rv from the partner search, column
// m's maximum over rows other than m and t from its column buffer.  Then
// column t is not scanned and the 1x1 test decides; a non-finite a_tt is
// still reported (it was read).  On a rejection the workgroup meets before
// returning: what follows (the interchanges) rewrites the LDS entries read
// here.  The decision is the same in every thread, since all read the same
// values before that barrier.
CTP_DEV bool reject_early(const PivotArgs& g, int ns, int ri, double rv, double amm, const Top2& cm, int cA,
                          double inv_u) {
  if (!(rv >= 0.0)) return false;   // no finite partner value
  const double att = lazy_a(g, ns, ri, ri);
  const bool early = reject_2x2_early(att, rv, amm, top2_excluding(cm, fabs(pv_dyn[cA + ri])), g.small, inv_u);
  if (early) {
    if (nonfinite(att) && threadIdx.x == 0) atomicOr(&pv_sh.status, ST_NONFINITE);
    __syncthreads();
  }
  return early;
}

// The pivot loop.  Its state (nelim, m, progress, the number of pending
// slots) is uniform: every thread takes the same decisions from the same
// reduced values and keeps its own copy, so a rejected candidate costs only
// its reductions.  Barriers per elimination: one between the row and the
// column half of the interchanges, one at the end.
template <int NT>
CTP_DEV void pivot_decide_body(const PivotArgs& g) {
  const int p = g.p;
  const int rc = min(g.r, pivot_rcache(p));
  const int cA = colbuf(p, rc, 0), cB = colbuf(p, rc, 1);

  PivState* st = g.st;
  if (threadIdx.x == 0) {
    pv_sh.nelim = st->nelim;
    pv_sh.m = st->m;
    pv_sh.progress = st->progress;
    pv_sh.done = st->done;
    pv_sh.status = 0;
  }
  __syncthreads();
  if (pv_sh.done) {
    // the previous apply consumed the last batch
    if (threadIdx.x == 0) st->nslot = 0;
    return;
  }
  int nelim = pv_sh.nelim, m = pv_sh.m, progress = pv_sh.progress;
  for (int k = threadIdx.x; k < p; k += NT) {
    pv_perm[k] = g.perm[k];
    pv_piv[k] = g.piv[k];
    pv_d[2 * k] = g.d[2 * k];
    pv_d[2 * k + 1] = g.d[2 * k + 1];
  }
  __syncthreads();

  const double inv_u = 1.0 / g.u;
  int ns = 0;     // pending slots of this batch
  int slot = 0;   // alternating LDS slot of the reductions
  while (nelim < p && ns < NSLOT - 1) {
    int action = ACT_NONE;
    int t = -1;
    int mc = m;        // position the action applies to
    bool fb = false;   // root fallback step (no column buffers)
    double d1 = 0.0, d21 = 0.0, d2 = 0.0;   // pivot: d1 (1x1) or [d1 d21; d21 d2]
    if (m >= p) {
      if (progress) {
        // end of a pass that eliminated something: a new pass
        progress = 0;
        m = nelim;
        continue;
      }
      if (!g.root) break;
      // A pass without progress in the last panel: eliminate the column at
      // nelim regardless of u (1x1 unless below small, else a 2x2 with the
      // next column if its determinant is safely nonzero, else zero).
      fb = true;
      const int k = nelim;
      const double akk = lazy_a(g, ns, k, k);
      double a21 = 0.0, a22 = 0.0;
      bool two = false;
      if (!(fabs(akk) >= g.small) && k + 1 < p) {
        a21 = lazy_a(g, ns, k + 1, k);
        a22 = lazy_a(g, ns, k + 1, k + 1);
        two = det_ok(akk, a21, a22, g.small);
      }
      if (fabs(akk) >= g.small) {
        action = ACT_1X1;
        mc = k;
        d1 = akk;
      } else if (two) {
        action = ACT_2X2;
        t = k;
        mc = k + 1;
        d1 = akk;
        d21 = a21;
        d2 = a22;
      } else {
        action = ACT_ZERO;
        mc = k;
      }
      if (threadIdx.x == 0) atomicOr(&pv_sh.status, ST_ROOT_FALLBACK);
      // every thread has read the block before its owners overwrite it
      __syncthreads();
    } else {
      // pass A: column m (rows other than m) into colA with its largest two,
      // the partner search along row m, the diagonal entry (thread 0)
      const ScanPre qa = scan_preload<NT>(g, rc, nelim, m);
      const int jp = nelim + threadIdx.x;
      const double xp = jp < m ? CM(g.T, m, jp, g.lda) : 0.0;
      const double xd = threadIdx.x == 0 ? CM(g.T, m, m, g.lda) : 0.0;
      Top2 cm = top2_empty();
      col_scan<NT>(g, ns, rc, nelim, m, cA, qa, cm);
      double rv = -1.0;
      int ri = 0x7fffffff;
      for (int j = jp; j < m; j += NT) {
        double x = fabs(j == jp ? lazy_a_from(g, ns, m, j, xp) : lazy_a(g, ns, m, j));
        cm.bad |= nonfinite(x);
        if (x != x) x = -0.5;   // NaN: loses to any number, keeps t a valid index
        if (x > rv) {
          rv = x;
          ri = j;
        }
      }
      if (threadIdx.x == 0) {
        const double v = lazy_a_from(g, ns, m, m, xd);
        pv_sh.sc[slot][0] = v;
        cm.bad |= nonfinite(v);
      }
      if (cm.bad) atomicOr(&pv_sh.status, ST_NONFINITE);
      reduce_pass<NT, true>(cm, rv, ri, slot);
      const double amm = pv_sh.sc[slot][0];
      slot ^= 1;
      const double maxm = top2_max(cm);
      const double colmax = fmax(fabs(amm), maxm);
      if (colmax < g.small) {
        action = ACT_ZERO;
      } else if (m > nelim && !reject_early(g, ns, ri, rv, amm, cm, cA, inv_u)) {
        t = ri;
        // pass B: column t (rows other than t) into colB with its largest
        // two; a_tt (thread 0), a_mt (the owner of row m) and a_tm (read
        // back from colA by thread 0) travel with the reduction
        const ScanPre qb = scan_preload<NT>(g, rc, nelim, t);
        const double xtt = threadIdx.x == 0 ? CM(g.T, t, t, g.lda) : 0.0;
        Top2 ct = top2_empty();
        col_scan<NT>(g, ns, rc, nelim, t, cB, qb, ct);
        if (threadIdx.x == 0) {
          const double v = lazy_a_from(g, ns, t, t, xtt);
          pv_sh.sc[slot][0] = v;
          pv_sh.sc[slot][2] = pv_dyn[cA + t];
          ct.bad |= nonfinite(v);
        }
        if (ct.bad) atomicOr(&pv_sh.status, ST_NONFINITE);
        if (threadIdx.x == (m - nelim) % NT) pv_sh.sc[slot][1] = pv_dyn[cB + m];
        double dv = -1.0;
        int di = 0;
        reduce_pass<NT, false>(ct, dv, di, slot);
        const double att = pv_sh.sc[slot][0], atm = pv_sh.sc[slot][1], xtm = pv_sh.sc[slot][2];
        slot ^= 1;
        const double maxt = top2_excluding(ct, fabs(atm));    // rows other than t, m
        const double maxm2 = top2_excluding(cm, fabs(xtm));   // rows other than m, t
        if (accept_2x2(att, atm, amm, maxt, maxm2, g.small, inv_u)) {
          action = ACT_2X2;
          d1 = att;
          d21 = atm;
          d2 = amm;
        }
      }
      if (action == ACT_NONE) {
        const double bound = g.u * maxm;
        action = (fabs(amm) >= bound) ? ACT_1X1 : ACT_REJECT;
        d1 = amm;
      }
    }
    if (action == ACT_REJECT) {
      m = m + 1;
      continue;
    }

    // interchanges: (mc, k) for a 1x1 or zero pivot, (t, k) then (mc, k+1)
    // for a 2x2 pivot
    const int k = nelim;
    const bool two = action == ACT_2X2;
    const SwapPlan sp = two ? swap_plan(t, k, mc, k + 1) : swap_plan(mc, k, k, k);
    const bool moves = sp.src[0] != sp.x[0] || sp.src[1] != sp.x[1] || sp.src[2] != sp.x[2] || sp.src[3] != sp.x[3];
    if (moves) {
      swap_rows<NT>(g, ns, sp);
      __syncthreads();
    }
    const int s0 = ns;
    // 2x2 inverse (the same for every row)
    double i11 = 0.0, i21 = 0.0, i22 = 0.0;
    if (two) inverse_2x2(d1, d21, d2, i11, i21, i22);
    // this thread's first cached R row: its interchange values are read
    // here, so that they travel with the square's (one memory round trip
    // for both halves of the column phase)
    double rpre[4];
    const bool rpre_ok = moves && (int)threadIdx.x < rc && (int)threadIdx.x < g.r;
    if (rpre_ok) {
#pragma unroll
      for (int q = 0; q < 4; ++q) rpre[q] = CM(g.R, threadIdx.x, sp.x[q], g.ldr);
    }
    // the square: column half of the interchanges, then the pivot columns
    // (pivot-column values from the column buffers: old column m, and old
    // column t for a 2x2, at the row's old position)
    for (int i = threadIdx.x; i < p; i += NT) {
      if (moves)
        permute_line<double>(sp, [&](int x) { return CM(g.T, i, x, g.lda); },
                             [&](int x, double v) { CM(g.T, i, x, g.lda) = v; });
      if (i < k) continue;
      const int si = swap_src(sp.x[0], sp.x[1], sp.x[2], sp.x[3], i);
      if (action == ACT_ZERO) {
        CM(g.T, i, k, g.lda) = 0.0;
      } else if (!two) {
        if (i == k) {
          CM(g.T, k, k, g.lda) = d1;
        } else {
          const double w = fb ? lazy_a(g, ns, i, k) : pv_dyn[cA + si];
          const double l = w / d1;
          CM(g.T, i, k, g.lda) = l;
          pv_dyn[lA(p, s0, i)] = l;
          pv_dyn[wc(p, s0, i)] = w;
        }
      } else {
        if (i == k) {
          CM(g.T, k, k, g.lda) = d1;
        } else if (i == k + 1) {
          CM(g.T, k + 1, k, g.lda) = d21;
          CM(g.T, k + 1, k + 1, g.lda) = d2;
        } else {
          const double w1 = fb ? lazy_a(g, ns, i, k) : pv_dyn[cB + si];
          const double w2 = fb ? lazy_a(g, ns, i, k + 1) : pv_dyn[cA + si];
          const double l1 = w1 * i11 + w2 * i21;
          const double l2 = w1 * i21 + w2 * i22;
          CM(g.T, i, k, g.lda) = l1;
          CM(g.T, i, k + 1, g.lda) = l2;
          pv_dyn[lA(p, s0, i)] = l1;
          pv_dyn[lA(p, s0 + 1, i)] = l2;
          pv_dyn[wc(p, s0, i)] = w1;
          pv_dyn[wc(p, s0 + 1, i)] = w2;
        }
      }
    }
    // R: column half of the interchanges, then the pivot columns
    const double adk = fabs(d1);
    const double j11 = fabs(i11), j21 = fabs(i21), j22 = fabs(i22);
    for_r_rows<NT>(rc, g.r, [&](int i, auto cached) {
      constexpr bool C = decltype(cached)::value;
      if (moves) {
        auto st = [&](int x, double v) { CM(g.R, i, x, g.ldr) = v; };
        if (C && rpre_ok && i == (int)threadIdx.x) permute_store<double>(sp, rpre, st);
        else permute_line<double>(sp, [&](int x) { return CM(g.R, i, x, g.ldr); }, st);
      }
      if (action == ACT_ZERO) {
        CM(g.R, i, k, g.ldr) = 0.0;
      } else if (!two) {
        const double x = (C && !fb) ? pv_dyn[cA + p + i] : lazy_r<C>(g, ns, rc, i, k);
        const double l = g.abs_update ? x / adk : x / d1;
        CM(g.R, i, k, g.ldr) = l;
        if (C) pv_dyn[lR(p, rc, s0, i)] = l;
      } else {
        const double x1 = (C && !fb) ? pv_dyn[cB + p + i] : lazy_r<C>(g, ns, rc, i, k);
        const double x2 = (C && !fb) ? pv_dyn[cA + p + i] : lazy_r<C>(g, ns, rc, i, k + 1);
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
        if (C) {
          pv_dyn[lR(p, rc, s0, i)] = l1;
          pv_dyn[lR(p, rc, s0 + 1, i)] = l2;
        }
      }
    });
    if (threadIdx.x == 0) {
      if (action == ACT_ZERO) {
        pv_piv[k] = PIV_ZERO;
        pv_d[2 * k] = 0.0;
        pv_d[2 * k + 1] = 0.0;
        atomicOr(&pv_sh.status, ST_ZERO_PIVOT);
      } else if (!two) {
        pv_piv[k] = PIV_1X1;
        pv_d[2 * k] = d1;
        pv_d[2 * k + 1] = 0.0;
        pv_sh.kind[s0] = 1;
        pv_sh.sk[s0] = k;
      } else {
        pv_piv[k] = PIV_2X2_FIRST;
        pv_piv[k + 1] = PIV_2X2_SECOND;
        pv_d[2 * k] = d1;
        pv_d[2 * k + 1] = d21;
        pv_d[2 * k + 2] = d2;
        pv_d[2 * k + 3] = 0.0;
        pv_sh.kind[s0] = 2;
        pv_sh.kind[s0 + 1] = 3;
        pv_sh.sk[s0] = k;
        pv_sh.sk[s0 + 1] = k + 1;
      }
    }
    // after an elimination: the next candidate and the progress flag (a
    // fallback step restarts the pass and does not count as progress)
    const int width = action == ACT_ZERO ? 1 : two ? 2 : 1;
    ns += action == ACT_ZERO ? 0 : width;
    m = (fb ? nelim : m) + width;
    nelim += width;
    progress = fb ? 0 : 1;
    __syncthreads();
  }
  __syncthreads();

  // Save the batch for the apply kernel and the loop state for the next launch.
  const bool batch_full = ns >= NSLOT - 1;
  for (int q = threadIdx.x; q < ns * p; q += NT) g.wbuf[q] = pv_dyn[NSLOT * p + q];
  for (int k = threadIdx.x; k < p; k += NT) {
    g.perm[k] = pv_perm[k];
    g.piv[k] = pv_piv[k];
    g.d[2 * k] = pv_d[2 * k];
    g.d[2 * k + 1] = pv_d[2 * k + 1];
  }
  if (threadIdx.x == 0) {
    const bool finished = nelim >= p || !batch_full;
    st->nelim = nelim;
    st->m = m;
    st->progress = progress;
    st->done = finished;
    st->nslot = ns;
    for (int s = 0; s < NSLOT; ++s) {
      st->slot_k[s] = pv_sh.sk[s];
      st->slot_kind[s] = s < ns ? pv_sh.kind[s] : 0;
    }
    *g.nelim_out = nelim;
    if (pv_sh.status) atomicOr(g.status, pv_sh.status);
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void pivot_decide_kernel(PivotArgs g) { pivot_decide_body<NT>(g); }

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

template <int NT>
CTP_DEV void pivot_factor_wg_body(const PivotArgs& g) {
  pivot_init_body(g, threadIdx.x, NT);
  __syncthreads();
  const int rounds = g.p / (NSLOT - 1) + 2;
  for (int q = 0; q < rounds; ++q) {
    pivot_decide_body<NT>(g);
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
      for (int b = threadIdx.x / 256; b < tiles; b += NT / 256)
        pivot_apply_tile(g, b, threadIdx.x % 256, nslot, nelim, pw_kind, pw_sk);
    }
    __syncthreads();
    if (done || nslot == 0) break;
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void pivot_factor_wg_kernel(PivotArgs g) { pivot_factor_wg_body<NT>(g); }

// one workgroup per supernode of a batch
template <int NT>
__global__ __launch_bounds__(NT) void pivot_factor_batch_kernel(const PivotArgs* __restrict__ args, int count) {
  if ((int)blockIdx.x >= count) return;
  const PivotArgs g = args[blockIdx.x];
  pivot_factor_wg_body<NT>(g);
}

// Workgroup size of the search.  The loop is a chain of short scans, each
// ended by a workgroup reduction whose cost grows with the number of waves,
// so when every row of R is cached the search runs with 512 threads (256
// for at most 256 rows), a few rows per thread; with R rows beyond the
// cached ones (TPP on a tall panel) the scans stream from memory and get
// 1024 threads.  The apply works on tiles of 256 threads.
inline int pivot_threads(int p, int r) {
  const int rc = pivot_rcache(p);
  if (r > rc) return 1024;
  return p + r <= 256 ? 256 : 512;
}

template <typename K>
static hipError_t pivot_lds_attr(K kern, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

size_t pivot_lds_bytes(int p, int r);

// ---------------------------------------------------------------------------
// batches: per-node descriptors and pivot-search arguments built on the
// device from the caller's ctp_node array
// ---------------------------------------------------------------------------

__global__ void batch_setup_kernel(const ctp_node* __restrict__ in, int count, int method, unsigned flags,
                                   double u, double small, double* panels, double* s, int* perm, int* piv,
                                   double* d, int* nelim, int* status, unsigned char* work,
                                   BatchNode* __restrict__ nodes, PivotArgs* __restrict__ pargs, int reset) {
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
  if (reset) {
    status[i] = 0;
    nelim[i] = 0;
  }
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
                       int reset, hipStream_t stream) {
  unsigned char* base = static_cast<unsigned char*>(work);
  BatchNode* nodes = reinterpret_cast<BatchNode*>(base);
  PivotArgs* pargs = reinterpret_cast<PivotArgs*>(base + align_up((size_t)count * sizeof(BatchNode), 256));
  unsigned int* counter = reinterpret_cast<unsigned int*>(
      base + align_up((size_t)count * sizeof(BatchNode), 256) + align_up((size_t)count * sizeof(PivotArgs), 256));
  hipLaunchKernelGGL(batch_setup_kernel, dim3((count + 127) / 128), dim3(128), 0, stream, in, count, method, flags, u, small, panels, s, perm,
                                                             piv, d, nelim, status, base, nodes, pargs, reset);
  *nodes_out = nodes;
  *pargs_out = pargs;
  *counter_out = counter;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int launch_pivot_batch(int count, const void* pargs, int max_p, int max_r, hipStream_t stream) {
  const size_t lds = pivot_lds_bytes(max_p, max_r);
  if (max_p > CTP_MAX_P || lds + 16 * 1024 > 160 * 1024) return -2;
  const PivotArgs* a = static_cast<const PivotArgs*>(pargs);
  hipError_t e0;
  switch (pivot_threads(max_p, max_r)) {
    case 256:
      e0 = pivot_lds_attr(pivot_factor_batch_kernel<256>, lds);
      if (e0 != hipSuccess) return CTP_ERR_HIP_BASE - (int)e0;
      hipLaunchKernelGGL(pivot_factor_batch_kernel<256>, dim3(count), dim3(256), lds, stream, a, count);
      break;
    case 512:
      e0 = pivot_lds_attr(pivot_factor_batch_kernel<512>, lds);
      if (e0 != hipSuccess) return CTP_ERR_HIP_BASE - (int)e0;
      hipLaunchKernelGGL(pivot_factor_batch_kernel<512>, dim3(count), dim3(512), lds, stream, a, count);
      break;
    default:
      e0 = pivot_lds_attr(pivot_factor_batch_kernel<1024>, lds);
      if (e0 != hipSuccess) return CTP_ERR_HIP_BASE - (int)e0;
      hipLaunchKernelGGL(pivot_factor_batch_kernel<1024>, dim3(count), dim3(1024), lds, stream, a, count);
      break;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

size_t pivot_lds_bytes(int p, int r) {
  const int rcap = pivot_rcache(p);
  const int rc = r < rcap ? r : rcap;
  return ((size_t)2 * NSLOT * p + (size_t)NSLOT * rc + 2 * ((size_t)p + rc)) * sizeof(double);
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
  const int nt = pivot_threads(p, r);
  hipError_t e0 = hipSuccess;
  if (one_wg) {
    if (nt == 256) {
      e0 = pivot_lds_attr(pivot_factor_wg_kernel<256>, lds);
      if (e0 == hipSuccess) hipLaunchKernelGGL(pivot_factor_wg_kernel<256>, dim3(1), dim3(256), lds, stream, g);
    } else if (nt == 512) {
      e0 = pivot_lds_attr(pivot_factor_wg_kernel<512>, lds);
      if (e0 == hipSuccess) hipLaunchKernelGGL(pivot_factor_wg_kernel<512>, dim3(1), dim3(512), lds, stream, g);
    } else {
      e0 = pivot_lds_attr(pivot_factor_wg_kernel<1024>, lds);
      if (e0 == hipSuccess) hipLaunchKernelGGL(pivot_factor_wg_kernel<1024>, dim3(1), dim3(1024), lds, stream, g);
    }
    if (e0 != hipSuccess) return CTP_ERR_HIP_BASE - (int)e0;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
  }
  e0 = nt == 256 ? pivot_lds_attr(pivot_decide_kernel<256>, lds)
                 : nt == 512 ? pivot_lds_attr(pivot_decide_kernel<512>, lds) : pivot_lds_attr(pivot_decide_kernel<1024>, lds);
  if (e0 != hipSuccess) return CTP_ERR_HIP_BASE - (int)e0;
  const size_t sq = (size_t)p * p;
  const unsigned init_blocks = (unsigned)std::min<size_t>((sq + 255) / 256 + 1, 2048);
  hipLaunchKernelGGL(pivot_init_kernel, dim3(init_blocks), dim3(256), 0, stream, g);
  const int tw = (p + APPLY_TILE - 1) / APPLY_TILE;
  const int apply_blocks = tw * tw + ((r + APPLY_TILE - 1) / APPLY_TILE) * tw;
  // every full batch holds at least NSLOT-1 eliminated columns
  const int rounds = p / (NSLOT - 1) + 2;
  for (int q = 0; q < rounds; ++q) {
    if (nt == 256) hipLaunchKernelGGL(pivot_decide_kernel<256>, dim3(1), dim3(256), lds, stream, g);
    else if (nt == 512) hipLaunchKernelGGL(pivot_decide_kernel<512>, dim3(1), dim3(512), lds, stream, g);
    else hipLaunchKernelGGL(pivot_decide_kernel<1024>, dim3(1), dim3(1024), lds, stream, g);
    if (apply_blocks > 0) hipLaunchKernelGGL(pivot_apply_kernel, dim3(apply_blocks), dim3(256), 0, stream, g);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
