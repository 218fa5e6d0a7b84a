// Dense symmetric indefinite LDL^T built from supernode panels, the solve
// with its factors and FP64 iterative refinement.
//
// Section 1 describes a multifrontal code: each supernode is factorized
// (Factor), its block of L below the pivots is solved for (Solve), the
// Schur complement is formed for the parent (Form), failed pivots are
// delayed to the parent, and the root eliminates everything.  A dense
// matrix factorized right-looking in panels of pw columns is that chain
// with one child per node:
//   panel = delayed columns of the previous panel + the next pw columns,
//           every row below them;
//   Factor + Solve on the panel with the chosen pivot rule (the supernode
//   entry points), the panel's interchanges applied to the rows of the L
//   columns already done and composed into one global permutation;
//   trailing matrix -= L21 W^T (Form, subtracted), W = L21 D;
//   the last panel (no rows below) eliminates every column (CTP_FLAG_ROOT).
// The host reads back nelim after each panel (panel widths depend on it).
//
// Reduced precision (ctp_opts.prec 1 / 2): the trailing matrix lives in an
// FP32 copy; each panel's triangular solve (L21, W) and the trailing update
// run on FP32 / BF16 matrix cores with FP32 accumulation, from operand rows
// the solve converts once; the pivot search, the 2x2 inverses and D^-1 stay
// FP64 (on the FP32 trailing values).  The solve with the factors is FP64;
// refinement computes residuals with the original FP64 matrix.
//
// Solve with the factors, P A P^T = L D L^T:
//   y = P b;  L y' = y (forward);  z = D^-1 y';  L^T x' = z (backward);
//   x = P^T x'.
// The diagonal blocks of L (DB = 128 columns) are inverted once at the end
// of the factorization and L^T is mirrored into the upper triangle, so each
// block step of either sweep is a dense product with coalesced columns:
//   forward  block j: z_j = Linv_j y_j; rows below: y_R -= L(R, j) z_j
//   backward block j: x_j = Linv_j^T z_j; rows above: z_R -= L^T(R, j) x_j
// (one launch per block, every workgroup recomputing the small product on
// the matrix cores).

#include <algorithm>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "common.h"

namespace ctp {

int supernode_with_hook(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv, double* d,
                        int* nelim, int* status, void* work, size_t lwork, hipStream_t stream,
                        int (*hook)(void*), void* hook_arg);
int launch_schur_w_sub(int n, int p, const double* a, int lda, const double* w, int ldw,
                       const int* nelim, double* c, int ldc, int tc0, int tc1, hipStream_t stream);
int launch_lowp_update_ops(int r, int K, const int* nelim, float* c, int ldc, int prec, void* ops, int tc0,
                           int tc1, hipStream_t stream);

constexpr int DB = 128;   // diagonal block of the solve

// Per-system strides (elements) of a batch of systems, system = blockIdx.z;
// all zero for one system.  a: matrix / factors; v: perm and piv (ints);
// d: D; y: solve vectors; b: right-hand sides (and xbar); x: the forward
// solution; g: Abar; w: the system's block of the workspace (doubles).
struct DZ {
  long long a = 0, v = 0, d = 0, y = 0, b = 0, x = 0, g = 0, w = 0;
};

// ---------------------------------------------------------------------------
// panel bookkeeping
// ---------------------------------------------------------------------------

// Rows k0..k0+pe-1 of the L columns 0..k0-1 follow the panel's interchanges:
// new row q = old row perm_p[q].  One workgroup per column.
__global__ __launch_bounds__(256) void dense_perm_left_kernel(double* a, int lda, int k0, int pe,
                                                              const int* __restrict__ perm_p) {
  __shared__ double col[CTP_MAX_P];
  double* c = a + (size_t)blockIdx.x * lda + k0;
  for (int q = threadIdx.x; q < pe; q += blockDim.x) col[q] = c[perm_p[q]];
  __syncthreads();
  for (int q = threadIdx.x; q < pe; q += blockDim.x) c[q] = col[q];
}

// One panel step of a batch of systems: system s (blockIdx.y) has its
// panel at k0 with pe columns; slot indexes its nelim in the step's array.
struct DenseStep {
  int k0, pe, active, slot;
};

__global__ __launch_bounds__(256) void dense_perm_left_batch_kernel(double* a, int lda, long long stride,
                                                                    const DenseStep* __restrict__ steps,
                                                                    const int* __restrict__ pperm) {
  __shared__ double col[CTP_MAX_P];
  const DenseStep st = steps[blockIdx.y];
  if (!st.active || (int)blockIdx.x >= st.k0) return;
  const int* perm_p = pperm + (size_t)blockIdx.y * CTP_MAX_P;
  double* c = a + (size_t)blockIdx.y * stride + (size_t)blockIdx.x * lda + st.k0;
  for (int q = threadIdx.x; q < st.pe; q += blockDim.x) col[q] = c[perm_p[q]];
  __syncthreads();
  for (int q = threadIdx.x; q < st.pe; q += blockDim.x) c[q] = col[q];
}

// Global permutation, pivot types and D of the panel's eliminated columns.
__global__ __launch_bounds__(512) void dense_bookkeep_kernel(int k0, int pe, const int* __restrict__ perm_p,
                                                             const int* __restrict__ piv_p,
                                                             const double* __restrict__ d_p,
                                                             const int* __restrict__ nelim_p, int* gperm,
                                                             int* gpiv, double* gd) {
  __shared__ int old[CTP_MAX_P];
  const int ne = min(max(*nelim_p, 0), pe);
  for (int q = threadIdx.x; q < pe; q += blockDim.x) old[q] = gperm[k0 + q];
  __syncthreads();
  for (int q = threadIdx.x; q < pe; q += blockDim.x) gperm[k0 + q] = old[perm_p[q]];
  for (int q = threadIdx.x; q < ne; q += blockDim.x) {
    gpiv[k0 + q] = piv_p[q];
    gd[2 * (k0 + q)] = d_p[2 * q];
    gd[2 * (k0 + q) + 1] = d_p[2 * q + 1];
  }
}

// Same, one workgroup per system of a batch.
__global__ __launch_bounds__(512) void dense_bookkeep_batch_kernel(int N, const DenseStep* __restrict__ steps,
                                                                   const int* __restrict__ pperm,
                                                                   const int* __restrict__ ppiv,
                                                                   const double* __restrict__ pd,
                                                                   const int* __restrict__ pnelim, int* gperm,
                                                                   int* gpiv, double* gd) {
  __shared__ int old[CTP_MAX_P];
  const int sys = blockIdx.x;
  const DenseStep st = steps[sys];
  if (!st.active) return;
  const int* perm_p = pperm + (size_t)sys * CTP_MAX_P;
  const int* piv_p = ppiv + (size_t)sys * CTP_MAX_P;
  const double* d_p = pd + (size_t)sys * 2 * CTP_MAX_P;
  int* gp = gperm + (size_t)sys * N;
  const int k0 = st.k0, pe = st.pe;
  const int ne = min(max(pnelim[st.slot], 0), pe);
  for (int q = threadIdx.x; q < pe; q += blockDim.x) old[q] = gp[k0 + q];
  __syncthreads();
  for (int q = threadIdx.x; q < pe; q += blockDim.x) gp[k0 + q] = old[perm_p[q]];
  for (int q = threadIdx.x; q < ne; q += blockDim.x) {
    gpiv[(size_t)sys * N + k0 + q] = piv_p[q];
    gd[(size_t)sys * 2 * N + 2 * (k0 + q)] = d_p[2 * q];
    gd[(size_t)sys * 2 * N + 2 * (k0 + q) + 1] = d_p[2 * q + 1];
  }
}

// gperm[i] = i mod N over count systems of order N
// nelim and status of the panel just factorized, into pinned host memory
// (the host reads them after the stream synchronizes): one tiny kernel
// instead of two device-to-host copies.
__global__ void dense_publish_kernel(const int* __restrict__ nelim, const int* __restrict__ status,
                                     volatile int* out) {
  out[0] = *nelim;
  out[1] = *status;
  __threadfence_system();
}

__global__ void dense_iota_kernel(int* gperm, int N, long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) gperm[i] = (int)(i % N);
}

// FP32 working copy of the lower triangle (columns j, rows j..N-1).
__global__ __launch_bounds__(256) void dense_to_f32_kernel(const double* __restrict__ a, int lda,
                                                           float* __restrict__ w32, int ld32, int N) {
  const int j = blockIdx.y;
  for (int i = j + blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
    w32[(size_t)j * ld32 + i] = (float)a[(size_t)j * lda + i];
}

// Panel columns c0..c1-1, rows c0..N-1, from the FP32 working copy.
__global__ __launch_bounds__(256) void dense_from_f32_kernel(double* __restrict__ a, int lda,
                                                             const float* __restrict__ w32, int ld32,
                                                             int c0, int N) {
  const int j = c0 + blockIdx.y;
  for (int i = j + blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
    a[(size_t)j * lda + i] = (double)w32[(size_t)j * ld32 + i];
}

// ---------------------------------------------------------------------------
// solve preparation: L^T into the upper triangle, inverses of the diagonal
// blocks of the unit lower L (entries that hold D are read as 0 / 1)
// ---------------------------------------------------------------------------

CTP_DEV double l_entry(const double* a, int lda, const int* piv, int i, int k) {
  // L(i, k) of the unit lower factor, i > k
  if (i == k + 1 && piv[k] == PIV_2X2_FIRST) return 0.0;
  return a[(size_t)k * lda + i];
}

// U(k, i) = L(i, k) for i > k, stored at row k, column i (upper triangle).
__global__ __launch_bounds__(256) void dense_mirror_kernel(double* a, int lda, const int* __restrict__ piv,
                                                           int N, DZ z) {
  // 32 x 32 tiles of the strictly lower triangle, transposed through LDS
  __shared__ double t[32][33];
  a += blockIdx.z * z.a;
  piv += blockIdx.z * z.v;
  const int bi = blockIdx.x, bk = blockIdx.y;   // tile row (i), tile column (k)
  if (bi < bk) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows of threads
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = bi * 32 + tx, k = bk * 32 + yy;
    double v = 0.0;
    if (i < N && k < N && i > k) v = l_entry(a, lda, piv, i, k);
    t[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int k = bk * 32 + tx, i = bi * 32 + yy;   // write U(k, i) at row k, column i
    if (i < N && k < N && i > k) a[(size_t)i * lda + k] = t[tx][yy];
  }
}

// Inverse of the unit lower diagonal block b (columns b*DB ..): thread j
// owns column j of X = L_bb^-1 (kept in LDS) and solves L x = e_j column
// by column: at step k, column k of L below the diagonal is staged in LDS
// once for the workgroup and every column j <= k takes x(i) -= L(i, k) x(k)
// for its rows i > k.
extern __shared__ double dn_dyn[];
constexpr int LINV_LDS = DB * (DB + 1) * (int)sizeof(double);

__global__ __launch_bounds__(DB) void dense_linv_kernel(const double* __restrict__ a, int lda,
                                                        const int* __restrict__ piv, int N,
                                                        double* __restrict__ linv, double* __restrict__ linvt, DZ z) {
  __shared__ double lcol[DB];
  double (*X)[DB + 1] = reinterpret_cast<double (*)[DB + 1]>(dn_dyn);
  a += blockIdx.z * z.a;
  piv += blockIdx.z * z.v;
  linv += blockIdx.z * z.w;
  linvt += blockIdx.z * z.w;
  const int b = blockIdx.x;
  const int c0 = b * DB;
  const int nb = min(DB, N - c0);
  const int j = threadIdx.x;
  for (int i = 0; i < DB; ++i) X[i][j] = (i == j && j < nb) ? 1.0 : 0.0;
  for (int k = 0; k + 1 < nb; ++k) {
    __syncthreads();   // the previous step's reads of lcol are done
    {
      const int i = threadIdx.x;
      lcol[i] = (i > k && i < nb) ? l_entry(a, lda, piv, c0 + i, c0 + k) : 0.0;
    }
    __syncthreads();
    if (j <= k) {
      const double xk = X[k][j];
      for (int i = k + 1; i < nb; ++i) X[i][j] = fma(-lcol[i], xk, X[i][j]);
    }
  }
  __syncthreads();
  double* L = linv + (size_t)b * DB * DB;
  double* LT = linvt + (size_t)b * DB * DB;
  for (int i = 0; i < DB; ++i) {
    L[(size_t)j * DB + i] = X[i][j];     // column-major Linv
    LT[(size_t)i * DB + j] = X[i][j];    // column-major Linv^T
  }
}

// ---------------------------------------------------------------------------
// solve sweeps
// ---------------------------------------------------------------------------

// y (N x nrhs, ldy) <- P b
__global__ void dense_gather_kernel(const double* __restrict__ b, int ldb, const int* __restrict__ perm,
                                    double* __restrict__ y, int ldy, int N, int nrhs, DZ z) {
  b += blockIdx.z * z.b;
  perm += blockIdx.z * z.v;
  y += blockIdx.z * z.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < N && c < nrhs) y[(size_t)c * ldy + i] = b[(size_t)c * ldb + perm[i]];
}

// x <- P^T y
__global__ void dense_scatter_kernel(const double* __restrict__ y, int ldy, const int* __restrict__ perm,
                                     double* __restrict__ x, int ldx, int N, int nrhs, DZ z) {
  y += blockIdx.z * z.y;
  perm += blockIdx.z * z.v;
  x += blockIdx.z * z.b;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < N && c < nrhs) x[(size_t)c * ldx + perm[i]] = y[(size_t)c * ldy + i];
}

// z <- D^-1 y (1x1 and 2x2 blocks; a zero pivot gives 0)
__global__ void dense_dsolve_kernel(const int* __restrict__ piv, const double* __restrict__ d,
                                    double* __restrict__ y, int ldy, int N, int nrhs, DZ z) {
  piv += blockIdx.z * z.v;
  d += blockIdx.z * z.d;
  y += blockIdx.z * z.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= N || c >= nrhs) return;
  double* yc = y + (size_t)c * ldy;
  const int pt = piv[i];
  if (pt == PIV_2X2_FIRST) {
    const double a11 = d[2 * i], a21 = d[2 * i + 1], a22 = d[2 * i + 2];
    const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
    const double det = (a22 * s) * a11 - (a21 * s) * a21;
    const double f = s / det;
    const double y1 = yc[i], y2 = yc[i + 1];
    yc[i] = (f * a22) * y1 - (f * a21) * y2;
    yc[i + 1] = -(f * a21) * y1 + (f * a11) * y2;
  } else if (pt == PIV_1X1) {
    yc[i] = yc[i] / d[2 * i];
  } else if (pt == PIV_ZERO) {
    yc[i] = 0.0;
  }
}

constexpr int SW_THREADS = 256;
constexpr int SW_MAXRHS = 16;

// One block step of a sweep, on the FP64 matrix cores.  The diagonal
// block's inverse M (column-major DB x DB, applied as t = M v_blk); rows of
// the update: the DB-row chunks listed by the grid (workgroup 0 writes t
// into the block rows of the second vector vo, workgroup q >= 1 updates
// chunk rlo + (q-1)*DB of v with the off-diagonal block of F, whose column
// k of the block sits at F + (c0 + k) * ldf).  Every workgroup reads v_blk
// and none writes it, so the result does not depend on which workgroups
// of the launch run at the same time; a sweep reads v and leaves its
// solution, block by block, in vo.  Both products of the step
// -- t = M v_blk (128 x 128 by 128 x nrhs) and the update of a 128-row
// chunk by F(chunk, blk) t -- are v_mfma_f64_16x16x4 products with the
// right-hand sides as the 16 columns of B (nrhs <= 16, the rest zero).
// Wave w owns row blocks 2w, 2w+1 (16 rows each) of the 128-row tile.
typedef double d4w __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void dense_sweep_mfma_kernel(const double* __restrict__ F, int ldf,
                                                                const double* __restrict__ M, int c0, int nb,
                                                                int rlo, int rhi, const int* __restrict__ piv,
                                                                double* __restrict__ v, double* __restrict__ vo,
                                                                int ldv, int nrhs, DZ z) {
  __shared__ double vb[DB][17];   // v_blk, then t, by (k, rhs)
  F += blockIdx.z * z.a;
  M += blockIdx.z * z.w;
  if (piv) piv += blockIdx.z * z.v;
  v += blockIdx.z * z.y;
  vo += blockIdx.z * z.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  for (int q = tid; q < DB * 16; q += 256) {
    const int k = q % DB, c = q / DB;
    vb[k][c] = (k < nb && c < nrhs) ? v[(size_t)c * ldv + c0 + k] : 0.0;
  }
  __syncthreads();
  // t = M v_blk; all 64 A fragments of this lane are loaded first so that
  // their latencies overlap
  d4w acc[2];
  double af[2][DB / 4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int s = 0; s < DB / 4; ++s) af[x][s] = M[(size_t)(4 * s + fk) * DB + (2 * wave + x) * 16 + fr];
  for (int x = 0; x < 2; ++x) acc[x] = d4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < DB / 4; ++s) {
    const double b = vb[4 * s + fk][fr];
#pragma unroll
    for (int x = 0; x < 2; ++x) acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x][s], b, acc[x], 0, 0, 0);
  }
  __syncthreads();   // every wave has read v_blk
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) vb[(2 * wave + x) * 16 + fk + 4 * q][fr] = acc[x][q];
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int q = tid; q < DB * 16; q += 256) {
      const int k = q % DB, c = q / DB;
      if (k < nb && c < nrhs) vo[(size_t)c * ldv + c0 + k] = vb[k][c];
    }
    return;
  }
  // rows r0 .. r0+127 of the chunk: v -= F(rows, blk) t
  const int r0 = rlo + (blockIdx.x - 1) * DB;
  const bool strad = piv && nb > 0 && piv[c0 + nb - 1] == PIV_2X2_FIRST;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int i = r0 + (2 * wave + x) * 16 + fr;
    const int ic = i < rhi ? i : rhi - 1;
#pragma unroll
    for (int s = 0; s < DB / 4; ++s) {
      const int k = 4 * s + fk;
      const bool kv = k < nb;
      double a = F[(size_t)(c0 + (kv ? k : 0)) * ldf + ic];
      if (!kv || (strad && i == c0 + nb && k == nb - 1)) a = 0.0;
      af[x][s] = a;
    }
  }
  for (int x = 0; x < 2; ++x) acc[x] = d4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < DB / 4; ++s) {
    const double b = vb[4 * s + fk][fr];
#pragma unroll
    for (int x = 0; x < 2; ++x) acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x][s], b, acc[x], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + (2 * wave + x) * 16 + fk + 4 * q;
      if (i < rhi && fr < nrhs) v[(size_t)fr * ldv + i] -= acc[x][q];
    }
}

// ---------------------------------------------------------------------------
// refinement: residual r = b - A x and the norms of the backward error
// ---------------------------------------------------------------------------

// r <- r - A(rows, cols) x(cols) for a 256-row stripe and a 512-column
// chunk (r starts as b); arow accumulates the absolute row sums of A.
constexpr int RES_ROWS = 256, RES_COLS = 512;

__global__ __launch_bounds__(RES_ROWS) void dense_residual_kernel(const double* __restrict__ A, int lda,
                                                                  const double* __restrict__ x, int ldx,
                                                                  double* __restrict__ r, int ldr, int N,
                                                                  int nrhs, double* __restrict__ arow) {
  __shared__ double xs[SW_MAXRHS][RES_COLS];
  const int j0 = blockIdx.y * RES_COLS;
  const int j1 = min(N, j0 + RES_COLS);
  for (int q = threadIdx.x; q < nrhs * RES_COLS; q += RES_ROWS) {
    const int c = q / RES_COLS, jj = q % RES_COLS;
    xs[c][jj] = j0 + jj < N ? x[(size_t)c * ldx + j0 + jj] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * RES_ROWS + threadIdx.x;
  if (i >= N) return;
  double acc[SW_MAXRHS];
  for (int c = 0; c < SW_MAXRHS; ++c) acc[c] = 0.0;
  double as = 0.0;
  // eight column loads in flight before their products (the products and
  // the row sum still run in column order)
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    double av[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) av[u] = A[(size_t)(j + u) * lda + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      as += fabs(av[u]);
#pragma unroll
      for (int c = 0; c < SW_MAXRHS; ++c)
        if (c < nrhs) acc[c] = fma(av[u], xs[c][j + u - j0], acc[c]);
    }
  }
  for (; j < j1; ++j) {
    const double aij = A[(size_t)j * lda + i];
    as += fabs(aij);
#pragma unroll
    for (int c = 0; c < SW_MAXRHS; ++c)
      if (c < nrhs) acc[c] = fma(aij, xs[c][j - j0], acc[c]);
  }
  if (arow) atomicAdd(arow + i, as);
  for (int c = 0; c < nrhs; ++c) atomicAdd(r + (size_t)c * ldr + i, -acc[c]);
}

CTP_DEV void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

// norms: [0] ||A||_inf, then per column c: [1+c] ||r||, [1+nrhs+c] ||x||, [1+2nrhs+c] ||b||
__global__ __launch_bounds__(256) void dense_norms_kernel(const double* __restrict__ arow,
                                                          const double* __restrict__ r, int ldr,
                                                          const double* __restrict__ x, int ldx,
                                                          const double* __restrict__ b, int ldb, int N,
                                                          int nrhs, double* norms) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double va = 0.0;
  double vr[SW_MAXRHS], vx[SW_MAXRHS], vb[SW_MAXRHS];
  for (int c = 0; c < SW_MAXRHS; ++c) vr[c] = vx[c] = vb[c] = 0.0;
  // a NaN counts as infinite (fmax would drop it from the maxima)
  auto mag = [](double v) { return v != v ? INFINITY : fabs(v); };
  if (i < N) {
    va = mag(arow[i]);
    for (int c = 0; c < nrhs; ++c) {
      vr[c] = mag(r[(size_t)c * ldr + i]);
      vx[c] = mag(x[(size_t)c * ldx + i]);
      vb[c] = mag(b[(size_t)c * ldb + i]);
    }
  }
  va = wave_max(va);
  for (int c = 0; c < nrhs; ++c) {
    vr[c] = wave_max(vr[c]);
    vx[c] = wave_max(vx[c]);
    vb[c] = wave_max(vb[c]);
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(norms, va);
    for (int c = 0; c < nrhs; ++c) {
      atomic_max_nonneg(norms + 1 + c, vr[c]);
      atomic_max_nonneg(norms + 1 + nrhs + c, vx[c]);
      atomic_max_nonneg(norms + 1 + 2 * nrhs + c, vb[c]);
    }
  }
}

__global__ void dense_copy_kernel(double* __restrict__ dst, int ldd, const double* __restrict__ src, int lds,
                                  int N, int nrhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < N && c < nrhs) dst[(size_t)c * ldd + i] = src[(size_t)c * lds + i];
}

__global__ void dense_fill_kernel(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void dense_axpy_kernel(double* __restrict__ x, int ldx, const double* __restrict__ dx, int lddx,
                                  int N, int nrhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < N && c < nrhs) x[(size_t)c * ldx + i] += dx[(size_t)c * lddx + i];
}

// ---------------------------------------------------------------------------
// adjoint of x = A^-1 b for symmetric A:  bbar = A^-1 xbar (the same
// factors), Abar = -sum_c (bbar_c x_c^T + x_c bbar_c^T) / 2, full N x N
// ---------------------------------------------------------------------------

// Entry (i, j), i >= j, is computed once and written to (i, j) and (j, i),
// so Abar is exactly symmetric whatever the compiler contracts.
__global__ __launch_bounds__(256) void dense_sym_outer_kernel(const double* __restrict__ bbar, int ldb,
                                                              const double* __restrict__ x, int ldx, int N,
                                                              int nrhs, double* __restrict__ abar, int ldg, DZ z) {
  __shared__ double bj[SW_MAXRHS], xj[SW_MAXRHS];
  bbar += blockIdx.z * z.b;
  x += blockIdx.z * z.x;
  abar += blockIdx.z * z.g;
  const int j = blockIdx.y;
  if (threadIdx.x < nrhs) {
    bj[threadIdx.x] = bbar[(size_t)threadIdx.x * ldb + j];
    xj[threadIdx.x] = x[(size_t)threadIdx.x * ldx + j];
  }
  __syncthreads();
  const int i = j + blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int c = 0; c < nrhs; ++c) s += bbar[(size_t)c * ldb + i] * xj[c] + x[(size_t)c * ldx + i] * bj[c];
  const double v = -0.5 * s;
  abar[(size_t)j * ldg + i] = v;
  abar[(size_t)i * ldg + j] = v;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

struct DenseWork {
  size_t sn_off = 0, sn_bytes = 0;     // two supernode workspaces (largest panel), sn_bytes each
  // panel outputs, two sets (stride pout_bytes): panels alternate between
  // the two so that a panel's trailing update can still read its W and
  // nelim while the next panel is factored
  size_t pperm_off = 0, ppiv_off = 0, pd_off = 0, pnelim_off = 0, pstatus_off = 0, pout_bytes = 0;
  size_t linv_off = 0, linvt_off = 0;  // inverses of the diagonal blocks
  size_t w32_off = 0;                  // FP32 trailing matrix (reduced precision)
  int ld32 = 0;
  size_t y_off = 0;                    // solve / refinement vectors
  size_t arow_off = 0;                 // absolute row sums of A (refinement)
  size_t norms_off = 0;
  size_t total = 0;
};

static int dense_nblocks(int N) { return (N + DB - 1) / DB; }

static DenseWork dense_layout(int N, int pw, const ctp_opts* o, int nrhs_max) {
  DenseWork w;
  size_t off = 0;
  ctp_opts so = *o;
  size_t sn = 0;
  const int pmax = CTP_MAX_P < N ? CTP_MAX_P : N;
  // every term of the supernode workspace grows with n and p except the W
  // buffer ((n - p) x p): the size at (2N, pmax) bounds every panel shape
  ctp_workspace_size(2 * N, pmax, &so, &sn);
  w.sn_off = off;
  w.sn_bytes = align_up(sn, 256);
  off = align_up(off + 2 * w.sn_bytes, 256);
  const size_t p0 = off;
  w.pperm_off = off; off = align_up(off + CTP_MAX_P * sizeof(int), 256);
  w.ppiv_off = off; off = align_up(off + CTP_MAX_P * sizeof(int), 256);
  w.pd_off = off; off = align_up(off + 2 * CTP_MAX_P * sizeof(double), 256);
  w.pnelim_off = off; off = align_up(off + sizeof(int), 256);
  w.pstatus_off = off; off = align_up(off + sizeof(int), 256);
  w.pout_bytes = off - p0;
  off += w.pout_bytes;
  const size_t nbk = (size_t)dense_nblocks(N);
  w.linv_off = off; off = align_up(off + nbk * DB * DB * sizeof(double), 256);
  w.linvt_off = off; off = align_up(off + nbk * DB * DB * sizeof(double), 256);
  if (o->prec != 0) {
    w.ld32 = (int)align_up((size_t)N, 64);
    w.w32_off = off; off = align_up(off + (size_t)w.ld32 * N * sizeof(float), 256);
  }
  w.y_off = off; off = align_up(off + (size_t)3 * N * (nrhs_max > 0 ? nrhs_max : 1) * sizeof(double), 256);
  w.arow_off = off; off = align_up(off + (size_t)(N > 0 ? N : 1) * sizeof(double), 256);
  w.norms_off = off; off = align_up(off + (1 + 3 * SW_MAXRHS) * sizeof(double), 256);
  w.total = off;
  (void)pw;
  return w;
}

size_t batch_header_bytes(int count);

// Workspace of a batch of systems: one block per system (the inverses of
// the diagonal blocks of L and their transposes, the solve vectors for up
// to SW_MAXRHS right-hand sides), the panel outputs of every system, the
// step descriptors, two node arrays (panels with rows below them, last
// panels) and the area of the batched supernode calls, sized for nodes of
// up to (2N, CTP_MAX_P) like the single-system driver.
struct BatchedDenseWork {
  size_t sys_bytes = 0;                             // one system's block
  size_t linv_off = 0, linvt_off = 0, y_off = 0;    // inside a system's block
  size_t sys_off = 0;
  size_t pperm_off = 0, ppiv_off = 0, pd_off = 0, pnelim_off = 0, pstatus_off = 0;
  size_t steps_off = 0, nodes_off = 0;
  size_t batch_off = 0, batch_bytes = 0;
  size_t total = 0;
};

static BatchedDenseWork dense_batched_layout(int count, int N, const ctp_opts* o) {
  BatchedDenseWork w;
  const size_t nbk = (size_t)dense_nblocks(N);
  const size_t c = (size_t)(count > 0 ? count : 1);
  size_t off = 0;
  w.linv_off = off; off = align_up(off + nbk * DB * DB * sizeof(double), 256);
  w.linvt_off = off; off = align_up(off + nbk * DB * DB * sizeof(double), 256);
  w.y_off = off; off = align_up(off + (size_t)2 * (N > 0 ? N : 1) * SW_MAXRHS * sizeof(double), 256);
  w.sys_bytes = off;
  size_t t = 0;
  w.sys_off = t; t = align_up(t + c * w.sys_bytes, 256);
  w.pperm_off = t; t = align_up(t + c * CTP_MAX_P * sizeof(int), 256);
  w.ppiv_off = t; t = align_up(t + c * CTP_MAX_P * sizeof(int), 256);
  w.pd_off = t; t = align_up(t + c * 2 * CTP_MAX_P * sizeof(double), 256);
  w.pnelim_off = t; t = align_up(t + 2 * c * sizeof(int), 256);
  w.pstatus_off = t; t = align_up(t + 2 * c * sizeof(int), 256);
  w.steps_off = t; t = align_up(t + c * sizeof(DenseStep), 256);
  w.nodes_off = t; t = align_up(t + 2 * c * sizeof(ctp_node), 256);
  const int pmax = CTP_MAX_P < N ? CTP_MAX_P : (N > 0 ? N : 1);
  const Workspace ws = workspace_layout(2 * (N > 0 ? N : 1), pmax, o->method);
  w.batch_bytes = batch_header_bytes((int)c) + c * align_up(ws.total, 256);
  w.batch_off = t; t = align_up(t + w.batch_bytes, 256);
  w.total = t;
  return w;
}

}  // namespace ctp

using namespace ctp;

static int dense_check(int N, int pw, const double* a, int lda, const ctp_opts* opts) {
  if (N < 0) return -1;
  if (pw < 1 || pw > CTP_MAX_P) return -2;
  if (!a && N > 0) return -3;
  if (lda < (N > 1 ? N : 1)) return -4;
  if (!opts || opts->prec < 0 || opts->prec > 2) return -5;
  return 0;
}

extern "C" {

int ctp_dense_workspace_size(int N, int pw, const ctp_opts* opts, int nrhs_max, size_t* bytes) {
  if (N < 0) return -1;
  if (pw < 1 || pw > CTP_MAX_P) return -2;
  if (!opts || opts->prec < 0 || opts->prec > 2) return -3;
  if (nrhs_max < 0 || nrhs_max > SW_MAXRHS) return -4;
  if (!bytes) return -5;
  *bytes = dense_layout(N, pw, opts, nrhs_max).total;
  return 0;
}

// The dense driver's two streams, one pair per device, created on first use
// (default priority, non-blocking): 0 the factorization chain, 1 the
// trailing updates that overlap it.  (Restricting stream 1 to all CUs but a
// few, so that the chain's one-workgroup pivot search always finds a free
// CU, measured 6 ms slower per factorization at N = 16384.)
// Runs and clears a deferred host step (the hook of supernode_with_hook).
static int run_deferred(void* f) {
  auto* slot = static_cast<std::function<int()>*>(f);
  std::function<int()> step = std::move(*slot);
  *slot = nullptr;
  return step ? step() : 0;
}

// Pinned, device-visible (nelim, status) pair per host thread and device;
// allocated on first use and kept (a few bytes) for the thread's lifetime.
static volatile int* dense_readback() {
  static thread_local int* buf[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!buf[dev] && hipHostMalloc(reinterpret_cast<void**>(&buf[dev]), 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    buf[dev] = nullptr;
  return buf[dev];
}

static hipStream_t dense_stream(int which) {
  static hipStream_t st[64][2] = {};
  static std::mutex m;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(m);
  hipStream_t& s = st[dev][which];
  if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  return s;
}

// Right-looking factorization of the dense matrix as a chain of supernodes
// (panel = the previous panel's delayed columns + the next pw columns; the
// last panel with CTP_FLAG_ROOT), with a look-ahead of one panel: the
// trailing update of panel k is split at the new columns of panel k+1.
// Those tile columns are updated in the chain right away, so panel k+1 can
// be factored at once; the rest of the update runs on the second stream,
// beside panel k+1's compression, pivot search and solve (which touch only
// panel k+1's own columns).  Panels alternate between two supernode
// workspaces and two sets of panel outputs, because the rest of panel k's
// update still reads its W and nelim while panel k+1 is factored.  Before
// panel k+1's own updates, and before its row interchanges are applied to
// the columns left of it (which include the L21 rows that the rest of panel
// k's update reads), the chain waits for that rest.  The caller's stream is
// joined by events at the start and at the end.
int ctp_ldlt_dense(int N, int pw, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                   double* d, int* status, int* npanels, void* work, size_t lwork, hipStream_t caller) {
  int rc = dense_check(N, pw, a, lda, opts);
  if (rc) return rc;
  if (N > 0 && (!perm || !piv || !d)) return -6;
  if (!status) return -9;
  DenseWork L = dense_layout(N, pw, opts, 0);
  if (!work || lwork < L.total) return -12;
  if (N == 0) return 0;
  unsigned char* base = static_cast<unsigned char*>(work);
  float* w32 = reinterpret_cast<float*>(base + L.w32_off);
  const bool lowp = opts->prec != 0;
  hipStream_t stream = dense_stream(0), side = dense_stream(1);
  if (!stream || !side) return CTP_ERR_HIP_BASE - (int)hipErrorInvalidValue;
  hipEvent_t ev_ready = nullptr, ev_rest = nullptr;
  if (hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ev_rest, hipEventDisableTiming) != hipSuccess) {
    if (ev_ready) hipEventDestroy(ev_ready);
    return CTP_ERR_HIP_BASE - (int)hipGetLastError();
  }
  // the chain starts after the caller's earlier work
  if (hipEventRecord(ev_ready, caller) != hipSuccess || hipStreamWaitEvent(stream, ev_ready, 0) != hipSuccess) {
    hipEventDestroy(ev_ready);
    hipEventDestroy(ev_rest);
    return CTP_ERR_HIP_BASE - (int)hipGetLastError();
  }
  bool rest_pending = false;
  volatile int* readback = dense_readback();   // null: read back with copies instead
  std::function<int()> rest_deferred;   // part 1 of the last panel's trailing update, not yet enqueued
  // every exit: the chain takes over the side stream's last work, the
  // caller's stream takes over the chain
  auto finish = [&](int code) {
    if (rest_pending) hipStreamWaitEvent(stream, ev_rest, 0);
    hipEventRecord(ev_ready, stream);
    hipStreamWaitEvent(caller, ev_ready, 0);
    hipEventDestroy(ev_ready);
    hipEventDestroy(ev_rest);
    return code;
  };

  dense_iota_kernel<<<(N + 255) / 256, 256, 0, stream>>>(perm, N, N);
  if (lowp) dense_to_f32_kernel<<<dim3(4, N), 256, 0, stream>>>(a, lda, w32, L.ld32, N);

  ctp_opts po = *opts;
  int k0 = 0, width = pw < N ? pw : N, carried = 0, panels = 0;
  int acc_status = 0;
  while (k0 < N) {
    if (width > CTP_MAX_P) return finish(-900);   // delays grew a panel past CTP_MAX_P
    const int n = N - k0;
    const bool root = n == width;
    double* ap = a + (size_t)k0 * lda + k0;
    const int q = panels & 1;
    unsigned char* sn = base + L.sn_off + q * L.sn_bytes;
    const size_t po_off = q * L.pout_bytes;
    int* pperm = reinterpret_cast<int*>(base + L.pperm_off + po_off);
    int* ppiv = reinterpret_cast<int*>(base + L.ppiv_off + po_off);
    double* pd = reinterpret_cast<double*>(base + L.pd_off + po_off);
    int* pnelim = reinterpret_cast<int*>(base + L.pnelim_off + po_off);
    int* pstatus = reinterpret_cast<int*>(base + L.pstatus_off + po_off);
    // reduced precision: the new columns of the panel come from the FP32 copy
    if (lowp && width > carried)
      dense_from_f32_kernel<<<dim3(4, width - carried), 256, 0, stream>>>(a, lda, w32, L.ld32, k0 + carried, N);
    po.flags = opts->flags | (root ? CTP_FLAG_ROOT : 0u);
    // the previous panel's deferred update starts once this panel's
    // compression is enqueued (the hook), so that the compression's
    // workgroups are not queued behind the update's
    rc = supernode_with_hook(n, width, ap, lda, &po, pperm, ppiv, pd, pnelim, pstatus, sn, L.sn_bytes, stream,
                             rest_deferred ? run_deferred : nullptr, &rest_deferred);
    if (rc) return finish(rc);
    int ne = 0, st = 0;
    if (readback) {
      dense_publish_kernel<<<1, 1, 0, stream>>>(pnelim, pstatus, readback);
      if (hipStreamSynchronize(stream) != hipSuccess) return finish(CTP_ERR_HIP_BASE - (int)hipGetLastError());
      ne = readback[0];
      st = readback[1];
    } else if (hipMemcpyAsync(&ne, pnelim, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
               hipMemcpyAsync(&st, pstatus, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
               hipStreamSynchronize(stream) != hipSuccess) {
      return finish(CTP_ERR_HIP_BASE - (int)hipGetLastError());
    }
    acc_status |= st;
    ++panels;
    // the previous panel's remaining update is done before this panel's
    // interchanges reach the columns left of it and before its own updates
    if (rest_pending) {
      if (hipStreamWaitEvent(stream, ev_rest, 0) != hipSuccess) return finish(CTP_ERR_HIP_BASE - (int)hipGetLastError());
      rest_pending = false;
    }
    if (k0 > 0) dense_perm_left_kernel<<<k0, 256, 0, stream>>>(a, lda, k0, width, pperm);
    dense_bookkeep_kernel<<<1, 512, 0, stream>>>(k0, width, pperm, ppiv, pd, pnelim, perm, piv, d);
    const int next_carried = width - ne, next_k0 = k0 + ne;
    const int next_width = N - next_k0 < next_carried + pw ? N - next_k0 : next_carried + pw;
    if (n > width && ne > 0) {
      // the W = L21 D that the solve left in the supernode workspace
      Workspace ws = workspace_layout(n, width, po.method);
      const double* w = reinterpret_cast<const double*>(sn + ws.w_off);
      const int r = n - width;
      const int nt = (r + 127) / 128;
      // tile columns holding the next panel's new columns
      const int tc = std::min(nt, (next_width - next_carried + 127) / 128);
      // part 0 (the next panel's tile columns) on the chain now, part 1
      // (the rest) on the side stream once the next panel's compression is
      // enqueued
      auto update = [=](int t0, int t1, hipStream_t s) {
        if (!lowp)
          return launch_schur_w_sub(n, width, ap, lda, w, ws.ldw, pnelim,
                                    a + (size_t)(k0 + width) * lda + (k0 + width), lda, t0, t1, s);
        // the operand rows of L21 and W that the reduced-precision Solve
        // converted into the supernode workspace
        return launch_lowp_update_ops(r, width, pnelim, w32 + (size_t)(k0 + width) * L.ld32 + (k0 + width),
                                      L.ld32, opts->prec, sn + align_up(ws.total, 256), t0, t1, s);
      };
      if (tc > 0 && (rc = update(0, tc, stream)) != 0) return finish(rc);
      if (tc < nt) {
        rest_deferred = [=, &rest_pending]() {
          if (hipEventRecord(ev_ready, stream) != hipSuccess || hipStreamWaitEvent(side, ev_ready, 0) != hipSuccess)
            return CTP_ERR_HIP_BASE - (int)hipGetLastError();
          const int e = update(tc, nt, side);
          if (e) return e;
          if (hipEventRecord(ev_rest, side) != hipSuccess) return CTP_ERR_HIP_BASE - (int)hipGetLastError();
          rest_pending = true;
          return 0;
        };
      }
    }
    carried = next_carried;
    k0 = next_k0;
    width = next_width;
  }
  if (rest_deferred && (rc = run_deferred(&rest_deferred)) != 0) return finish(rc);   // not reached: a panel with rows below has a successor
  if (rest_pending) {
    hipStreamWaitEvent(stream, ev_rest, 0);
    rest_pending = false;
  }
  // solve preparation
  {
    dim3 mg(dense_nblocks(N) * (DB / 32), dense_nblocks(N) * (DB / 32));
    dense_mirror_kernel<<<mg, 256, 0, stream>>>(a, lda, piv, N, DZ{});
    hipFuncSetAttribute(reinterpret_cast<const void*>(dense_linv_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, LINV_LDS);
    dense_linv_kernel<<<dense_nblocks(N), DB, LINV_LDS, stream>>>(a, lda, piv, N,
                                                          reinterpret_cast<double*>(base + L.linv_off),
                                                          reinterpret_cast<double*>(base + L.linvt_off), DZ{});
  }
  int* st_out = status;
  hipMemcpyAsync(st_out, &acc_status, sizeof(int), hipMemcpyHostToDevice, stream);
  if (hipStreamSynchronize(stream) != hipSuccess) return finish(CTP_ERR_HIP_BASE - (int)hipGetLastError());
  if (npanels) *npanels = panels;
  hipError_t e = hipGetLastError();
  return finish(e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e);
}

int ctp_ldlt_solve(int N, int nrhs, const double* a, int lda, const int* perm, const int* piv,
                   const double* d, double* b, int ldb, const ctp_opts* opts, int pw, void* work,
                   size_t lwork, hipStream_t stream) {
  if (N < 0) return -1;
  if (nrhs < 0 || nrhs > SW_MAXRHS) return -2;
  if (!a && N > 0) return -3;
  if (lda < (N > 1 ? N : 1)) return -4;
  if (N > 0 && (!perm || !piv || !d)) return -5;
  if (!b && N > 0 && nrhs > 0) return -8;
  if (ldb < (N > 1 ? N : 1)) return -9;
  if (!opts || opts->prec < 0 || opts->prec > 2) return -10;
  if (pw < 1 || pw > CTP_MAX_P) return -11;
  DenseWork L = dense_layout(N, pw, opts, nrhs);
  if (!work || lwork < L.total) return -13;
  if (N == 0 || nrhs == 0) return 0;
  unsigned char* base = static_cast<unsigned char*>(work);
  // two solve vectors: the forward sweep reads y1 and leaves L^-1 y in y2,
  // the backward sweep reads y2 and leaves the solution in y1
  double* y1 = reinterpret_cast<double*>(base + L.y_off);
  double* y2 = y1 + (size_t)N * nrhs;
  const int ldy = N;
  const double* linv = reinterpret_cast<const double*>(base + L.linv_off);
  const double* linvt = reinterpret_cast<const double*>(base + L.linvt_off);
  const dim3 eg((N + 255) / 256, nrhs);
  dense_gather_kernel<<<eg, 256, 0, stream>>>(b, ldb, perm, y1, ldy, N, nrhs, DZ{});
  const int nbk = dense_nblocks(N);
  for (int j = 0; j < nbk; ++j) {          // forward: L y' = y
    const int c0 = j * DB, nb = N - c0 < DB ? N - c0 : DB;
    const int rlo = c0 + nb, rhi = N;
    const int chunks = (rhi - rlo + DB - 1) / DB;
    dense_sweep_mfma_kernel<<<1 + chunks, 256, 0, stream>>>(a, lda, linv + (size_t)j * DB * DB, c0, nb, rlo, rhi,
                                                            piv, y1, y2, ldy, nrhs, DZ{});
  }
  dense_dsolve_kernel<<<eg, 256, 0, stream>>>(piv, d, y2, ldy, N, nrhs, DZ{});
  for (int j = nbk - 1; j >= 0; --j) {     // backward: L^T x' = z, L^T in the upper triangle
    const int c0 = j * DB, nb = N - c0 < DB ? N - c0 : DB;
    const int rlo = 0, rhi = c0;
    const int chunks = (rhi - rlo + DB - 1) / DB;
    dense_sweep_mfma_kernel<<<1 + chunks, 256, 0, stream>>>(a, lda, linvt + (size_t)j * DB * DB, c0, nb, rlo, rhi,
                                                            nullptr, y2, y1, ldy, nrhs, DZ{});
  }
  dense_scatter_kernel<<<eg, 256, 0, stream>>>(y1, ldy, perm, b, ldb, N, nrhs, DZ{});
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int ctp_ldlt_refine(int N, int nrhs, const double* a0, int lda0, const double* f, int ldf,
                    const int* perm, const int* piv, const double* d, const double* b, int ldb,
                    double* x, int ldx, const ctp_opts* opts, int pw, double tol, int max_steps,
                    int* steps, double* bwd_hist, void* work, size_t lwork, hipStream_t stream) {
  if (N < 0) return -1;
  if (nrhs < 1 || nrhs > SW_MAXRHS) return -2;
  if (!a0 || lda0 < (N > 1 ? N : 1)) return -3;
  if (!f || ldf < (N > 1 ? N : 1)) return -5;
  if (!b || ldb < (N > 1 ? N : 1)) return -10;
  if (!x || ldx < (N > 1 ? N : 1)) return -12;
  if (!opts) return -14;
  if (max_steps < 0) return -17;
  DenseWork L = dense_layout(N, pw, opts, nrhs);
  if (!work || lwork < L.total) return -20;
  if (N == 0) return 0;
  unsigned char* base = static_cast<unsigned char*>(work);
  double* r = reinterpret_cast<double*>(base + L.y_off) + (size_t)2 * N * nrhs;   // after the solve vectors
  double* arow = reinterpret_cast<double*>(base + L.arow_off);
  double* norms = reinterpret_cast<double*>(base + L.norms_off);
  const int nn = 1 + 3 * nrhs;
  const dim3 eg((N + 255) / 256, nrhs);
  const dim3 rg((N + RES_ROWS - 1) / RES_ROWS, (N + RES_COLS - 1) / RES_COLS);
  // x = solve(b)
  dense_copy_kernel<<<eg, 256, 0, stream>>>(x, ldx, b, ldb, N, nrhs);
  int rc = ctp_ldlt_solve(N, nrhs, f, ldf, perm, piv, d, x, ldx, opts, pw, work, lwork, stream);
  if (rc) return rc;
  std::vector<double> hn(nn);
  int k = 0;
  for (;;) {
    // r = b - A x (the row sums of |A| on the first pass), then the norms
    dense_copy_kernel<<<eg, 256, 0, stream>>>(r, N, b, ldb, N, nrhs);
    if (k == 0) dense_fill_kernel<<<(N + 255) / 256, 256, 0, stream>>>(arow, N, 0.0);
    dense_residual_kernel<<<rg, RES_ROWS, 0, stream>>>(a0, lda0, x, ldx, r, N, N, nrhs, k == 0 ? arow : nullptr);
    dense_fill_kernel<<<1, 64, 0, stream>>>(norms, nn, 0.0);
    dense_norms_kernel<<<(N + 255) / 256, 256, 0, stream>>>(arow, r, N, x, ldx, b, ldb, N, nrhs, norms);
    if (hipMemcpyAsync(hn.data(), norms, nn * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return CTP_ERR_HIP_BASE - (int)hipGetLastError();
    // an infinite norm (overflow, or a NaN in A, b, x or r) gives an
    // infinite backward error, which ends the refinement unconverged
    double be = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double nr = hn[1 + c], den = hn[0] * hn[1 + nrhs + c] + hn[1 + 2 * nrhs + c];
      double v;
      if (!std::isfinite(nr) || !std::isfinite(den)) v = INFINITY;
      else if (den > 0.0) v = nr / den;
      else v = nr > 0.0 ? INFINITY : 0.0;
      be = v > be ? v : be;
    }
    if (bwd_hist) bwd_hist[k] = be;
    if (be <= tol || k >= max_steps || !std::isfinite(be)) break;
    rc = ctp_ldlt_solve(N, nrhs, f, ldf, perm, piv, d, r, N, opts, pw, work, lwork, stream);
    if (rc) return rc;
    dense_axpy_kernel<<<eg, 256, 0, stream>>>(x, ldx, r, N, N, nrhs);
    ++k;
  }
  if (steps) *steps = k;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int ctp_ldlt_adjoint(int N, int nrhs, const double* a, int lda, const int* perm, const int* piv,
                     const double* d, const double* x, int ldx, double* xbar, int ldxb, double* abar,
                     int ldg, const ctp_opts* opts, int pw, void* work, size_t lwork, hipStream_t stream) {
  if (N < 0) return -1;
  if (nrhs < 0 || nrhs > SW_MAXRHS) return -2;
  if (!x || ldx < (N > 1 ? N : 1)) return -8;
  if (!xbar || ldxb < (N > 1 ? N : 1)) return -10;
  if (!abar || ldg < (N > 1 ? N : 1)) return -12;
  if (N == 0 || nrhs == 0) return 0;
  // bbar = A^-1 xbar (A symmetric: A^-T = A^-1), in place of xbar
  int rc = ctp_ldlt_solve(N, nrhs, a, lda, perm, piv, d, xbar, ldxb, opts, pw, work, lwork, stream);
  if (rc) return rc;
  dense_sym_outer_kernel<<<dim3((N + 255) / 256, N), 256, 0, stream>>>(xbar, ldxb, x, ldx, N, nrhs, abar, ldg, DZ{});
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// ---------------------------------------------------------------------------
// batches of systems
// ---------------------------------------------------------------------------

static bool batched_method_ok(const ctp_opts* o) {
  return o && o->prec == 0 && (o->method == CTP_STRICT || o->method == CTP_RELAXED || o->method == CTP_RESTRICTED);
}

int ctp_dense_batched_workspace_size(int count, int N, int pw, const ctp_opts* opts, size_t* bytes) {
  if (count < 0) return -1;
  if (N < 0) return -2;
  if (pw < 1 || pw > CTP_MAX_P) return -3;
  if (!batched_method_ok(opts)) return -4;
  if (!bytes) return -5;
  *bytes = dense_batched_layout(count, N, opts).total;
  return 0;
}

int ctp_ldlt_dense_batched(int count, int N, int pw, double* a, int lda, long long stride, const ctp_opts* opts,
                           int* perm, int* piv, double* d, int* status, int* nsteps, void* work, size_t lwork,
                           hipStream_t stream) {
  if (count < 0) return -1;
  if (N < 0) return -2;
  if (pw < 1 || pw > CTP_MAX_P) return -3;
  if (!a && count > 0 && N > 0) return -4;
  if (lda < (N > 1 ? N : 1)) return -5;
  if (count > 1 && stride < (long long)lda * N) return -6;
  if (!batched_method_ok(opts)) return -7;
  if (count > 0 && N > 0 && (!perm || !piv || !d)) return -8;
  if (count > 0 && !status) return -11;
  const BatchedDenseWork L = dense_batched_layout(count, N, opts);
  if (!work || lwork < L.total) return -14;
  if (nsteps) *nsteps = 0;
  if (count == 0) return 0;
  std::vector<int> acc(count, 0);
  if (N == 0) {
    if (hipMemcpyAsync(status, acc.data(), count * sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return CTP_ERR_HIP_BASE - (int)hipGetLastError();
    return 0;
  }
  unsigned char* base = static_cast<unsigned char*>(work);
  int* pperm = reinterpret_cast<int*>(base + L.pperm_off);
  int* ppiv = reinterpret_cast<int*>(base + L.ppiv_off);
  double* pd = reinterpret_cast<double*>(base + L.pd_off);
  int* pnelim = reinterpret_cast<int*>(base + L.pnelim_off);
  int* pstatus = reinterpret_cast<int*>(base + L.pstatus_off);
  DenseStep* dsteps = reinterpret_cast<DenseStep*>(base + L.steps_off);
  ctp_node* dnodes = reinterpret_cast<ctp_node*>(base + L.nodes_off);
  void* barea = base + L.batch_off;

  const long long total = (long long)count * N;
  dense_iota_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>(perm, N, total);

  std::vector<int> k0(count, 0), width(count, pw < N ? pw : N), done(count, 0);
  std::vector<DenseStep> steps(count);
  std::vector<ctp_node> nm, nr;
  std::vector<int> hnel(2 * count), hst(2 * count);
  ctp_opts om = *opts, orr = *opts;
  om.flags = (opts->flags & ~(CTP_FLAG_ROOT | CTP_FLAG_S_TILED)) | CTP_FLAG_S_SUBTRACT;
  orr.flags = (opts->flags & ~(CTP_FLAG_S_SUBTRACT | CTP_FLAG_S_TILED)) | CTP_FLAG_ROOT;
  int nstep = 0;
  while (true) {
    nm.clear();
    nr.clear();
    int maxk0 = 0;
    for (int s = 0; s < count; ++s) {
      steps[s] = DenseStep{k0[s], width[s], 0, 0};
      if (done[s]) continue;
      if (width[s] > CTP_MAX_P) return CTP_ERR_PANEL_TOO_WIDE;
      const int n = N - k0[s];
      const bool root = n == width[s];
      ctp_node c;
      std::memset(&c, 0, sizeof(c));
      c.n = n;
      c.p = width[s];
      c.lda = lda;
      c.lds = lda;
      c.a_off = (long long)s * stride + (long long)k0[s] * lda + k0[s];
      c.s_off = root ? -1 : (long long)s * stride + (long long)(k0[s] + width[s]) * lda + (k0[s] + width[s]);
      c.out_off = (long long)s * CTP_MAX_P;
      steps[s].active = 1;
      if (root) {
        steps[s].slot = count + (int)nr.size();
        nr.push_back(c);
      } else {
        steps[s].slot = (int)nm.size();
        nm.push_back(c);
      }
      if (k0[s] > maxk0) maxk0 = k0[s];
    }
    if (nm.empty() && nr.empty()) break;
    // panels with rows below them: Factor + Solve + Form subtracted into the
    // trailing matrices; last panels: Factor with the root rule
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<ctp_node>& nodes = pass == 0 ? nm : nr;
      if (nodes.empty()) continue;
      const ctp_opts* po = pass == 0 ? &om : &orr;
      ctp_batch_info info;
      int rc = ctp_batch_plan((int)nodes.size(), nodes.data(), po, &info);
      if (rc) return rc;
      if (info.work_bytes > L.batch_bytes) return -14;
      ctp_node* dn = dnodes + (pass == 0 ? 0 : count);
      if (hipMemcpyAsync(dn, nodes.data(), nodes.size() * sizeof(ctp_node), hipMemcpyHostToDevice, stream) !=
          hipSuccess)
        return CTP_ERR_HIP_BASE - (int)hipGetLastError();
      rc = ctp_supernode_batched((int)nodes.size(), dn, &info, a, pass == 0 ? a : nullptr, pperm, ppiv, pd,
                                 pnelim + (pass == 0 ? 0 : count), pstatus + (pass == 0 ? 0 : count), po, barea,
                                 L.batch_bytes, stream);
      if (rc) return rc;
    }
    if (hipMemcpyAsync(dsteps, steps.data(), count * sizeof(DenseStep), hipMemcpyHostToDevice, stream) != hipSuccess)
      return CTP_ERR_HIP_BASE - (int)hipGetLastError();
    if (maxk0 > 0)
      dense_perm_left_batch_kernel<<<dim3(maxk0, count), 256, 0, stream>>>(a, lda, stride, dsteps, pperm);
    dense_bookkeep_batch_kernel<<<count, 512, 0, stream>>>(N, dsteps, pperm, ppiv, pd, pnelim, perm, piv, d);
    if (hipMemcpyAsync(hnel.data(), pnelim, 2 * count * sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(hst.data(), pstatus, 2 * count * sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return CTP_ERR_HIP_BASE - (int)hipGetLastError();
    for (int s = 0; s < count; ++s) {
      if (!steps[s].active) continue;
      const int ne = hnel[steps[s].slot];
      acc[s] |= hst[steps[s].slot];
      const int carried = width[s] - ne;
      k0[s] += ne;
      width[s] = N - k0[s] < carried + pw ? N - k0[s] : carried + pw;
      if (k0[s] >= N) done[s] = 1;
    }
    ++nstep;
  }
  // solve preparation for every system
  {
    DZ z;
    z.a = stride;
    z.v = N;
    z.w = (long long)(L.sys_bytes / sizeof(double));
    const int nb32 = dense_nblocks(N) * (DB / 32);
    dense_mirror_kernel<<<dim3(nb32, nb32, count), 256, 0, stream>>>(a, lda, piv, N, z);
    hipFuncSetAttribute(reinterpret_cast<const void*>(dense_linv_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                        LINV_LDS);
    dense_linv_kernel<<<dim3(dense_nblocks(N), 1, count), DB, LINV_LDS, stream>>>(
        a, lda, piv, N, reinterpret_cast<double*>(base + L.sys_off + L.linv_off),
        reinterpret_cast<double*>(base + L.sys_off + L.linvt_off), z);
  }
  if (hipMemcpyAsync(status, acc.data(), count * sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return CTP_ERR_HIP_BASE - (int)hipGetLastError();
  if (nsteps) *nsteps = nstep;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int ctp_ldlt_solve_batched(int count, int N, int nrhs, const double* a, int lda, long long stride, const int* perm,
                           const int* piv, const double* d, double* b, int ldb, long long bstride,
                           const ctp_opts* opts, int pw, void* work, size_t lwork, hipStream_t stream) {
  if (count < 0) return -1;
  if (N < 0) return -2;
  if (nrhs < 0 || nrhs > SW_MAXRHS) return -3;
  if (!a && count > 0 && N > 0) return -4;
  if (lda < (N > 1 ? N : 1)) return -5;
  if (count > 1 && stride < (long long)lda * N) return -6;
  if (count > 0 && N > 0 && (!perm || !piv || !d)) return -7;
  if (!b && count > 0 && N > 0 && nrhs > 0) return -10;
  if (ldb < (N > 1 ? N : 1)) return -11;
  if (count > 1 && bstride < (long long)ldb * nrhs) return -12;
  if (!batched_method_ok(opts)) return -13;
  if (pw < 1 || pw > CTP_MAX_P) return -14;
  const BatchedDenseWork L = dense_batched_layout(count, N, opts);
  if (!work || lwork < L.total) return -16;
  if (count == 0 || N == 0 || nrhs == 0) return 0;
  unsigned char* base = static_cast<unsigned char*>(work);
  double* y1 = reinterpret_cast<double*>(base + L.sys_off + L.y_off);
  double* y2 = y1 + (size_t)N * nrhs;
  const double* linv = reinterpret_cast<const double*>(base + L.sys_off + L.linv_off);
  const double* linvt = reinterpret_cast<const double*>(base + L.sys_off + L.linvt_off);
  const int ldy = N;
  DZ z;
  z.a = stride;
  z.v = N;
  z.d = 2LL * N;
  z.y = (long long)(L.sys_bytes / sizeof(double));
  z.b = bstride;
  z.w = z.y;
  const dim3 eg((N + 255) / 256, nrhs, count);
  dense_gather_kernel<<<eg, 256, 0, stream>>>(b, ldb, perm, y1, ldy, N, nrhs, z);
  const int nbk = dense_nblocks(N);
  for (int j = 0; j < nbk; ++j) {
    const int c0 = j * DB, nb = N - c0 < DB ? N - c0 : DB;
    const int chunks = (N - (c0 + nb) + DB - 1) / DB;
    dense_sweep_mfma_kernel<<<dim3(1 + chunks, 1, count), 256, 0, stream>>>(
        a, lda, linv + (size_t)j * DB * DB, c0, nb, c0 + nb, N, piv, y1, y2, ldy, nrhs, z);
  }
  dense_dsolve_kernel<<<eg, 256, 0, stream>>>(piv, d, y2, ldy, N, nrhs, z);
  for (int j = nbk - 1; j >= 0; --j) {
    const int c0 = j * DB, nb = N - c0 < DB ? N - c0 : DB;
    const int chunks = (c0 + DB - 1) / DB;
    dense_sweep_mfma_kernel<<<dim3(1 + chunks, 1, count), 256, 0, stream>>>(
        a, lda, linvt + (size_t)j * DB * DB, c0, nb, 0, c0, nullptr, y2, y1, ldy, nrhs, z);
  }
  dense_scatter_kernel<<<eg, 256, 0, stream>>>(y1, ldy, perm, b, ldb, N, nrhs, z);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int ctp_ldlt_adjoint_batched(int count, int N, int nrhs, const double* a, int lda, long long stride,
                             const int* perm, const int* piv, const double* d, const double* x, int ldx,
                             long long xstride, double* xbar, int ldxb, long long xbstride, double* abar, int ldg,
                             long long gstride, const ctp_opts* opts, int pw, void* work, size_t lwork,
                             hipStream_t stream) {
  if (count < 0) return -1;
  if (N < 0) return -2;
  if (nrhs < 0 || nrhs > SW_MAXRHS) return -3;
  if (count > 0 && N > 0 && nrhs > 0) {
    if (!x || ldx < (N > 1 ? N : 1) || (count > 1 && xstride < (long long)ldx * nrhs)) return -10;
    if (!xbar || ldxb < (N > 1 ? N : 1) || (count > 1 && xbstride < (long long)ldxb * nrhs)) return -13;
    if (!abar || ldg < (N > 1 ? N : 1) || (count > 1 && gstride < (long long)ldg * N)) return -16;
  }
  if (count == 0 || N == 0 || nrhs == 0) return 0;
  // bbar = A^-1 xbar for every system, in place of xbar
  int rc = ctp_ldlt_solve_batched(count, N, nrhs, a, lda, stride, perm, piv, d, xbar, ldxb, xbstride, opts, pw, work,
                                  lwork, stream);
  if (rc) return rc;
  DZ z;
  z.b = xbstride;
  z.x = xstride;
  z.g = gstride;
  dense_sym_outer_kernel<<<dim3((N + 255) / 256, N, count), 256, 0, stream>>>(xbar, ldxb, x, ldx, N, nrhs, abar, ldg,
                                                                              z);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // extern "C"
