// Threshold pivot search on a trapezoid [A11; R] in one workgroup
// (Section 2, the TPP kernel with tests (2.1)/(2.2), run on the compressed
// trapezoid of Section 4 (Fig. 4.1 (c)) or, for TPP, on the whole panel).
//
// R is the compressed matrix C (strict: absolute-value update eq. (4.4);
// relaxed: ordinary update eq. (4.3)), the real A21 (TPP) or empty
// (restricted pivoting, Section 3.2).
//
// Readings of the paper (the same as the oracle's):
//  * candidate m starts at the second column, advances by 2 after a 2x2
//    pivot, by 1 after a 1x1 pivot or a double failure; when m runs off
//    the end a new pass starts at the first uneliminated column (tried
//    alone as a 1x1) if the pass eliminated anything (the first pass
//    always gets a second one);
//  * the determinant test rejects when |det| <= max(small, |det0|/2,
//    |det1|/2); the 2x2 scale uses max(|a_tt|, |a_tm|, |a_mm|);
//  * the 2x2 stability test is |D^-1| (maxt, maxm)^T <= 1/u (eq. (2.2));
//  * column maxima run over the whole uneliminated symmetric column and
//    every row of R;
//  * interchanges are symmetric swaps (t to position nelim, then m to
//    nelim+1 for a 2x2 pivot);
//  * zero pivot: every entry of the column below `small`: D = 0, zero L
//    column, no update;
//  * ties go to the lowest index.
//
// Arithmetic: every update is a rounded product followed by a rounded sum
// (floating-point contraction is switched off in this file) in the order
//      1x1:  l_i = w_i / d;  a_ij = a_ij - l_i * w_j
//      2x2:  s = 1/max|D|, det = (a22*s)*a11 - (a21*s)*a21, f = s/det,
//            Dinv = [[f*a22, -(f*a21)], [., f*a11]],
//            l_i1 = w_i1*Dinv11 + w_i2*Dinv21, l_i2 = w_i1*Dinv12 + w_i2*Dinv22,
//            a_ij = a_ij - (l_i1*w_j1 + l_i2*w_j2)
// so that every decision and every factor entry is reproducible bit for
// bit by any implementation that applies the same operations.
//
// Storage: A11 lower triangle in place (the panel), R column-major; the
// trailing trapezoid is updated right-looking after each pivot.  Both stay
// in global memory (L2-resident at the sizes used); each pivot step is a
// handful of workgroup reductions plus one sweep of the trailing block.

#include "common.h"

#pragma clang fp contract(off)

namespace ctp {

constexpr int PIV_THREADS = 1024;
constexpr int PIV_WAVES = PIV_THREADS / 64;
constexpr int PIV_RCHUNK = 2048;      // R rows whose multipliers are staged in LDS at once

struct PivotArgs {
  int p;
  double* a11;   // A11 (lower triangle), column-major, lda
  int lda;
  int r;
  double* R;     // bottom block, column-major, ldr (may be null when r == 0)
  int ldr;
  int abs_update;   // 1: strict rule for R
  double u, small;
  int* perm;
  int* piv;
  double* d;
  int* nelim_out;
  int* status;
};

// Value of the symmetric A11 at (i, j) from lower storage.
CTP_DEV double& sym(double* a, int lda, int i, int j) {
  return i >= j ? CM(a, i, j, lda) : CM(a, j, i, lda);
}

struct Shared {
  double red_v[PIV_WAVES];
  int red_i[PIV_WAVES];
  double red_v2[PIV_WAVES];
  // decision broadcast
  int nelim, m, progress, action, t;
  double maxm, maxt, maxm2;
};

// Workgroup max of v (every thread passes its partial).  Returns the max
// to every thread.
CTP_DEV double block_max(double v, Shared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  if (lane == 0) sh.red_v[wave] = v;
  __syncthreads();
  double r = sh.red_v[0];
  for (int w = 1; w < PIV_WAVES; ++w) r = fmax(r, sh.red_v[w]);
  __syncthreads();
  return r;
}

CTP_DEV void block_max2(double& v1, double& v2, Shared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v1 = wave_max(v1);
  v2 = wave_max(v2);
  if (lane == 0) { sh.red_v[wave] = v1; sh.red_v2[wave] = v2; }
  __syncthreads();
  double r1 = sh.red_v[0], r2 = sh.red_v2[0];
  for (int w = 1; w < PIV_WAVES; ++w) { r1 = fmax(r1, sh.red_v[w]); r2 = fmax(r2, sh.red_v2[w]); }
  __syncthreads();
  v1 = r1;
  v2 = r2;
}

// Argmax of v with the lowest index on ties; returns the index.
CTP_DEV int block_argmax(double v, int idx, Shared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  if (lane == 0) { sh.red_v[wave] = v; sh.red_i[wave] = idx; }
  __syncthreads();
  double bv = sh.red_v[0];
  int bi = sh.red_i[0];
  for (int w = 1; w < PIV_WAVES; ++w) {
    double ov = sh.red_v[w];
    int oi = sh.red_i[w];
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  __syncthreads();
  return bi;
}

// max |a(i, col)| over uneliminated A11 rows i in [nelim, p) \ {x1, x2}
// and all rows of R: this thread's partial.
CTP_DEV double col_partial(const PivotArgs& g, int nelim, int col, int x1, int x2) {
  double v = 0.0;
  for (int i = nelim + threadIdx.x; i < g.p; i += PIV_THREADS)
    if (i != x1 && i != x2) v = fmax(v, fabs(sym(g.a11, g.lda, i, col)));
  for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) v = fmax(v, fabs(CM(g.R, i, col, g.ldr)));
  return v;
}

// Symmetric interchange of positions a < b (lower storage), R columns,
// perm.  Callers synchronise afterwards.
CTP_DEV void sym_swap(const PivotArgs& g, int a, int b, int* perm_s) {
  if (a == b) return;
  if (a > b) { int t = a; a = b; b = t; }
  double* A = g.a11;
  const int lda = g.lda, p = g.p;
  // rows a and b left of column a (includes the L rows of eliminated columns)
  for (int j = threadIdx.x; j < a; j += PIV_THREADS) {
    double x = CM(A, a, j, lda), y = CM(A, b, j, lda);
    CM(A, a, j, lda) = y; CM(A, b, j, lda) = x;
  }
  // between: column a below a  <->  row b right of a
  for (int i = a + 1 + threadIdx.x; i < b; i += PIV_THREADS) {
    double x = CM(A, i, a, lda), y = CM(A, b, i, lda);
    CM(A, i, a, lda) = y; CM(A, b, i, lda) = x;
  }
  // below b: column a <-> column b
  for (int i = b + 1 + threadIdx.x; i < p; i += PIV_THREADS) {
    double x = CM(A, i, a, lda), y = CM(A, i, b, lda);
    CM(A, i, a, lda) = y; CM(A, i, b, lda) = x;
  }
  if (threadIdx.x == 0) {
    double x = CM(A, a, a, lda), y = CM(A, b, b, lda);
    CM(A, a, a, lda) = y; CM(A, b, b, lda) = x;
    int t = perm_s[a]; perm_s[a] = perm_s[b]; perm_s[b] = t;
  }
  for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) {
    double x = CM(g.R, i, a, g.ldr), y = CM(g.R, i, b, g.ldr);
    CM(g.R, i, a, g.ldr) = y; CM(g.R, i, b, g.ldr) = x;
  }
}

// Trailing update after a 1x1 pivot at position k.
CTP_DEV void eliminate_1x1(const PivotArgs& g, int k, double* wcol, double* lcol, double* rl) {
  double* A = g.a11;
  const int lda = g.lda, p = g.p;
  const double dk = CM(A, k, k, lda);
  for (int i = k + 1 + threadIdx.x; i < p; i += PIV_THREADS) {
    double w = CM(A, i, k, lda);
    wcol[i] = w;
    lcol[i] = w / dk;
  }
  __syncthreads();
  // A11: columns j > k, rows i >= j; each wave takes whole columns.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = k + 1 + wave; j < p; j += PIV_WAVES) {
    const double wj = wcol[j];
    for (int i = j + lane; i < p; i += 64) {
      double prod = lcol[i] * wj;
      CM(A, i, j, lda) = CM(A, i, j, lda) - prod;
    }
  }
  for (int i = k + 1 + threadIdx.x; i < p; i += PIV_THREADS) CM(A, i, k, lda) = lcol[i];
  // R rows, in chunks whose multipliers fit in LDS.
  const double adk = fabs(dk);
  for (int r0 = 0; r0 < g.r; r0 += PIV_RCHUNK) {
    const int r1 = min(g.r, r0 + PIV_RCHUNK);
    __syncthreads();
    for (int i = r0 + threadIdx.x; i < r1; i += PIV_THREADS) {
      double x = CM(g.R, i, k, g.ldr);
      rl[i - r0] = g.abs_update ? x / adk : x / dk;
    }
    __syncthreads();
    for (int j = k + 1 + wave; j < p; j += PIV_WAVES) {
      const double wj = wcol[j];
      const double awj = fabs(wj);
      for (int i = r0 + lane; i < r1; i += 64) {
        double cur = CM(g.R, i, j, g.ldr);
        if (g.abs_update) {
          double prod = rl[i - r0] * awj;
          CM(g.R, i, j, g.ldr) = cur + prod;
        } else {
          double prod = rl[i - r0] * wj;
          CM(g.R, i, j, g.ldr) = cur - prod;
        }
      }
    }
    for (int i = r0 + threadIdx.x; i < r1; i += PIV_THREADS) CM(g.R, i, k, g.ldr) = rl[i - r0];
  }
}

// Trailing update after a 2x2 pivot at positions (k, k+1).
CTP_DEV void eliminate_2x2(const PivotArgs& g, int k, double* w1c, double* w2c, double* l1c,
                           double* l2c, double* rl1, double* rl2) {
  double* A = g.a11;
  const int lda = g.lda, p = g.p;
  const double a11 = CM(A, k, k, lda), a21 = CM(A, k + 1, k, lda), a22 = CM(A, k + 1, k + 1, lda);
  const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
  const double det = (a22 * s) * a11 - (a21 * s) * a21;
  const double f = s / det;
  const double i11 = f * a22, i21 = -(f * a21), i22 = f * a11;
  for (int i = k + 2 + threadIdx.x; i < p; i += PIV_THREADS) {
    double w1 = CM(A, i, k, lda), w2 = CM(A, i, k + 1, lda);
    w1c[i] = w1;
    w2c[i] = w2;
    l1c[i] = w1 * i11 + w2 * i21;
    l2c[i] = w1 * i21 + w2 * i22;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = k + 2 + wave; j < p; j += PIV_WAVES) {
    const double wj1 = w1c[j], wj2 = w2c[j];
    for (int i = j + lane; i < p; i += 64) {
      double upd = l1c[i] * wj1 + l2c[i] * wj2;
      CM(A, i, j, lda) = CM(A, i, j, lda) - upd;
    }
  }
  for (int i = k + 2 + threadIdx.x; i < p; i += PIV_THREADS) {
    CM(A, i, k, lda) = l1c[i];
    CM(A, i, k + 1, lda) = l2c[i];
  }
  const double j11 = fabs(i11), j21 = fabs(i21), j22 = fabs(i22);
  for (int r0 = 0; r0 < g.r; r0 += PIV_RCHUNK) {
    const int r1 = min(g.r, r0 + PIV_RCHUNK);
    __syncthreads();
    for (int i = r0 + threadIdx.x; i < r1; i += PIV_THREADS) {
      double x1 = CM(g.R, i, k, g.ldr), x2 = CM(g.R, i, k + 1, g.ldr);
      if (g.abs_update) {
        rl1[i - r0] = x1 * j11 + x2 * j21;
        rl2[i - r0] = x1 * j21 + x2 * j22;
      } else {
        rl1[i - r0] = x1 * i11 + x2 * i21;
        rl2[i - r0] = x1 * i21 + x2 * i22;
      }
    }
    __syncthreads();
    for (int j = k + 2 + wave; j < p; j += PIV_WAVES) {
      const double wj1 = w1c[j], wj2 = w2c[j];
      const double awj1 = fabs(wj1), awj2 = fabs(wj2);
      for (int i = r0 + lane; i < r1; i += 64) {
        double cur = CM(g.R, i, j, g.ldr);
        if (g.abs_update) {
          double upd = rl1[i - r0] * awj1 + rl2[i - r0] * awj2;
          CM(g.R, i, j, g.ldr) = cur + upd;
        } else {
          double upd = rl1[i - r0] * wj1 + rl2[i - r0] * wj2;
          CM(g.R, i, j, g.ldr) = cur - upd;
        }
      }
    }
    for (int i = r0 + threadIdx.x; i < r1; i += PIV_THREADS) {
      CM(g.R, i, k, g.ldr) = rl1[i - r0];
      CM(g.R, i, k + 1, g.ldr) = rl2[i - r0];
    }
  }
}

enum { ACT_NONE = 0, ACT_ZERO, ACT_2X2, ACT_1X1, ACT_REJECT, ACT_PASS, ACT_STOP };

// Dynamic LDS: perm/piv (2p ints), d (2p doubles), 4 column buffers of p
// doubles, 2 R multiplier buffers of PIV_RCHUNK doubles.
__global__ __launch_bounds__(PIV_THREADS) void pivot_factor_kernel(PivotArgs g) {
  extern __shared__ unsigned char smem_raw[];
  double* d_s = reinterpret_cast<double*>(smem_raw);
  double* c1 = d_s + 2 * (size_t)g.p;
  double* c2 = c1 + g.p;
  double* c3 = c2 + g.p;
  double* c4 = c3 + g.p;
  double* rl1 = c4 + g.p;
  double* rl2 = rl1 + PIV_RCHUNK;
  int* perm_s = reinterpret_cast<int*>(rl2 + PIV_RCHUNK);
  int* piv_s = perm_s + g.p;
  __shared__ Shared sh;

  const int p = g.p;
  for (int k = threadIdx.x; k < p; k += PIV_THREADS) {
    perm_s[k] = k;
    piv_s[k] = PIV_DELAYED;
    d_s[2 * k] = 0.0;
    d_s[2 * k + 1] = 0.0;
  }
  if (threadIdx.x == 0) {
    sh.nelim = 0;
    sh.m = p >= 2 ? 1 : 0;
    sh.progress = 1;
  }
  __syncthreads();

  const double inv_u = 1.0 / g.u;
  int status_bits = 0;
  while (true) {
    const int nelim = sh.nelim;
    const int m = sh.m;
    if (nelim >= p) break;
    if (m >= p) {
      __syncthreads();
      if (threadIdx.x == 0) {
        if (!sh.progress) sh.action = ACT_STOP;
        else { sh.action = ACT_PASS; sh.progress = 0; sh.m = nelim; }
      }
      __syncthreads();
      if (sh.action == ACT_STOP) break;
      continue;
    }
    // column m: maxm over everything but the diagonal (zero test and 1x1)
    double maxm = block_max(col_partial(g, nelim, m, m, m), sh);
    const double amm = CM(g.a11, m, m, g.lda);
    const double colmax = fmax(fabs(amm), maxm);
    if (!isfinite(colmax)) status_bits |= ST_NONFINITE;
    int action = ACT_NONE;
    int t = -1;
    if (colmax < g.small) {
      action = ACT_ZERO;
    } else if (m > nelim) {
      // partner t: largest |a(m, j)| over the pending columns nelim..m-1
      double v = -1.0;
      int idx = 0x7fffffff;
      for (int j = nelim + threadIdx.x; j < m; j += PIV_THREADS) {
        double x = fabs(CM(g.a11, m, j, g.lda));
        if (x != x) x = -0.5;   // NaN: loses to any number, but keeps t a valid index
        if (x > v) { v = x; idx = j; }
      }
      t = block_argmax(v, idx, sh);
      double maxt = col_partial(g, nelim, t, t, m);
      double maxm2 = col_partial(g, nelim, m, t, m);
      block_max2(maxt, maxm2, sh);
      // 2x2 test (eq. (2.2)), evaluated identically by every thread
      const double att = CM(g.a11, t, t, g.lda), atm = CM(g.a11, m, t, g.lda);
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

    if (action == ACT_ZERO) {
      sym_swap(g, m, nelim, perm_s);
      __syncthreads();
      const int k = nelim;
      for (int i = k + 1 + threadIdx.x; i < p; i += PIV_THREADS) CM(g.a11, i, k, g.lda) = 0.0;
      for (int i = threadIdx.x; i < g.r; i += PIV_THREADS) CM(g.R, i, k, g.ldr) = 0.0;
      if (threadIdx.x == 0) {
        CM(g.a11, k, k, g.lda) = 0.0;
        piv_s[k] = PIV_ZERO;
        d_s[2 * k] = 0.0;
        sh.nelim = nelim + 1;
        sh.m = m + 1;
        sh.progress = 1;
      }
      status_bits |= ST_ZERO_PIVOT;
    } else if (action == ACT_2X2) {
      sym_swap(g, t, nelim, perm_s);
      __syncthreads();
      sym_swap(g, m, nelim + 1, perm_s);
      __syncthreads();
      const int k = nelim;
      if (threadIdx.x == 0) {
        piv_s[k] = PIV_2X2_FIRST;
        piv_s[k + 1] = PIV_2X2_SECOND;
        d_s[2 * k] = CM(g.a11, k, k, g.lda);
        d_s[2 * k + 1] = CM(g.a11, k + 1, k, g.lda);
        d_s[2 * k + 2] = CM(g.a11, k + 1, k + 1, g.lda);
        d_s[2 * k + 3] = 0.0;
      }
      eliminate_2x2(g, k, c1, c2, c3, c4, rl1, rl2);
      if (threadIdx.x == 0) {
        sh.nelim = nelim + 2;
        sh.m = m + 2;
        sh.progress = 1;
      }
    } else if (action == ACT_1X1) {
      sym_swap(g, m, nelim, perm_s);
      __syncthreads();
      const int k = nelim;
      if (threadIdx.x == 0) {
        piv_s[k] = PIV_1X1;
        d_s[2 * k] = CM(g.a11, k, k, g.lda);
      }
      eliminate_1x1(g, k, c1, c2, rl1);
      if (threadIdx.x == 0) {
        sh.nelim = nelim + 1;
        sh.m = m + 1;
        sh.progress = 1;
      }
    } else {
      if (threadIdx.x == 0) sh.m = m + 1;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int k = threadIdx.x; k < p; k += PIV_THREADS) {
    g.perm[k] = perm_s[k];
    g.piv[k] = piv_s[k];
    g.d[2 * k] = d_s[2 * k];
    g.d[2 * k + 1] = d_s[2 * k + 1];
  }
  if (threadIdx.x == 0) *g.nelim_out = sh.nelim;
  if (threadIdx.x == 0 && status_bits) atomicOr(g.status, status_bits);
}

size_t pivot_lds_bytes(int p) {
  return (size_t)2 * p * sizeof(double) + (size_t)4 * p * sizeof(double) +
         (size_t)2 * PIV_RCHUNK * sizeof(double) + (size_t)2 * p * sizeof(int);
}

int launch_pivot_factor(int p, double* a11, int lda, int r, double* R, int ldr, int abs_update,
                        double u, double small, int* perm, int* piv, double* d, int* nelim,
                        int* status, hipStream_t stream) {
  PivotArgs g;
  g.p = p; g.a11 = a11; g.lda = lda; g.r = r; g.R = R; g.ldr = ldr;
  g.abs_update = abs_update; g.u = u; g.small = small;
  g.perm = perm; g.piv = piv; g.d = d; g.nelim_out = nelim; g.status = status;
  size_t lds = pivot_lds_bytes(p);
  if (lds > 160 * 1024) return -2;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)pivot_factor_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  pivot_factor_kernel<<<1, PIV_THREADS, lds, stream>>>(g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
