// Solve task on the column-permuted A21 (Section 1; Fig. 4.1 (d)-(e)).
//
// Each row of A21 is independent: with x = row of A21 P^T,
//     W_E  = x_E (L_EE^T)^-1          (forward substitution, L unit lower)
//     x_d' = x_d - W_E L_dE^T         (delayed columns)
//     L21  = W_E D^-1                 (1x1 and 2x2 blocks)
// so one sweep over k = 0..nelim-1 of "x_j -= x_k L(j,k) for j > k" over
// all p columns yields W_E and the delayed columns together.
//
// Mapping: 8 threads per row, thread c of a row owns columns c, c+8, ...
// in registers (NC = ceil(p/8) of them), 32 rows per workgroup.  Columns
// of L are staged in LDS eight at a time; the pivot value x_k is broadcast
// inside the row's 8 lanes.  The permutation is applied as a gather when
// the row is loaded (no data movement); all loads of a workgroup finish
// before any store, so the update is in place.

#include "common.h"

namespace ctp {

constexpr int SOLVE_TPR = 8;                       // threads per row
constexpr int SOLVE_THREADS = 256;
constexpr int SOLVE_RPB = SOLVE_THREADS / SOLVE_TPR;  // rows per workgroup

template <int NC>
__global__ __launch_bounds__(SOLVE_THREADS) void solve_rows_kernel(
    int r, int p, double* __restrict__ a, int lda, const int* __restrict__ perm,
    const int* __restrict__ piv, const double* __restrict__ d, const int* __restrict__ nelim_p) {
  constexpr int PW = SOLVE_TPR * NC;               // padded width
  __shared__ double Lc[SOLVE_TPR][PW];
  __shared__ int piv_s[PW];
  const int tid = threadIdx.x;
  const int c = tid % SOLVE_TPR;
  const int row = blockIdx.x * SOLVE_RPB + tid / SOLVE_TPR;
  const bool valid = row < r;
  const int nelim = min(max(*nelim_p, 0), p);
  double* a21 = a + p;

  for (int j = tid; j < PW; j += SOLVE_THREADS) piv_s[j] = j < p ? piv[j] : PIV_DELAYED;

  double x[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int j = c + SOLVE_TPR * q;
    x[q] = (valid && j < p) ? a21[(size_t)perm[j] * lda + row] : 0.0;
  }

  // Chunks of 8 pivot columns.  The register holding the chunk's own
  // columns is selected once into `cur` (the chunk index is not a
  // compile-time constant), updated there, and written back at the end.
#pragma unroll 1
  for (int kb = 0; kb < NC; ++kb) {
    const int k0 = kb * SOLVE_TPR;
    if (k0 >= nelim) break;
    __syncthreads();
    // Stage L(:, k0..k0+7): zero on and above the diagonal and for the
    // in-block entry of a 2x2 pivot (its slot holds D(k+1,k)).
    // All loads first (clamped, always in bounds), masks afterwards, so the
    // loads of a chunk are in flight together.
    constexpr int NIT = (SOLVE_TPR * PW + SOLVE_THREADS - 1) / SOLVE_THREADS;
    constexpr int GRP = NIT < 8 ? NIT : 8;     // loads in flight per group
#pragma unroll
    for (int g0 = 0; g0 < NIT; g0 += GRP) {
      double lv[GRP];
#pragma unroll
      for (int it = 0; it < GRP; ++it) {
        const int idx = tid + (g0 + it) * SOLVE_THREADS;
        const int k = min(k0 + idx / PW, p - 1);
        const int j = min(idx % PW, p - 1);
        lv[it] = CM(a, j, k, lda);
      }
#pragma unroll
      for (int it = 0; it < GRP; ++it) {
        const int idx = tid + (g0 + it) * SOLVE_THREADS;
        if (idx < SOLVE_TPR * PW) {
          const int kk = idx / PW, j = idx % PW;
          const int k = k0 + kk;
          const bool keep = k < nelim && j > k && j < p &&
                            !(j == k + 1 && piv_s[k] == PIV_2X2_FIRST);
          Lc[kk][j] = keep ? lv[it] : 0.0;
        }
      }
    }
    __syncthreads();
    double cur = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (q == kb) cur = x[q];
    const int jc = c + k0;
    const int kend = min(SOLVE_TPR, nelim - k0);
    for (int kk = 0; kk < kend; ++kk) {
      const int k = k0 + kk;
      if (piv_s[k] == PIV_ZERO && c == kk) cur = 0.0;   // dropped column
      const double xk = __shfl(cur, kk, SOLVE_TPR);
      // Lc holds exact zeros on and above the diagonal, so the update is
      // applied to every column without a branch.
#pragma unroll
      for (int q = 0; q < NC; ++q) x[q] = fma(-xk, Lc[kk][c + SOLVE_TPR * q], x[q]);
      cur = fma(-xk, Lc[kk][jc], cur);
    }
#pragma unroll
    for (int q = 0; q < NC; ++q)
      if (q == kb) x[q] = cur;
  }

  // L21 = W D^-1.  A 2x2 block needs the neighbouring column, which lives
  // in the next (previous) lane, or in the register after (before) it for
  // the last (first) lane of the row's group.
  double carry = 0.0;   // W value of column j-1 before it was overwritten
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const double nxt_src = (c == 0) ? (q + 1 < NC ? x[q + 1] : 0.0) : x[q];
    const double prv_src = (c == SOLVE_TPR - 1) ? carry : x[q];
    const double nxt = __shfl(nxt_src, (c + 1) % SOLVE_TPR, SOLVE_TPR);
    const double prv = __shfl(prv_src, (c + SOLVE_TPR - 1) % SOLVE_TPR, SOLVE_TPR);
    const int j = c + SOLVE_TPR * q;
    double v = x[q];
    if (j < nelim) {
      const int pt = piv_s[j];
      if (pt == PIV_1X1) {
        v = x[q] / d[2 * j];
      } else if (pt == PIV_ZERO) {
        v = 0.0;
      } else {
        const int k = (pt == PIV_2X2_FIRST) ? j : j - 1;
        const double a11 = d[2 * k], a21 = d[2 * k + 1], a22 = d[2 * k + 2];
        const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
        const double det = (a22 * s) * a11 - (a21 * s) * a21;
        const double f = s / det;
        const double i11 = f * a22, i21 = -(f * a21), i22 = f * a11;
        const double w1 = (pt == PIV_2X2_FIRST) ? x[q] : prv;
        const double w2 = (pt == PIV_2X2_FIRST) ? nxt : x[q];
        v = (pt == PIV_2X2_FIRST) ? (w1 * i11 + w2 * i21) : (w1 * i21 + w2 * i22);
      }
    }
    carry = x[q];
    x[q] = v;
  }
  __syncthreads();   // every gather load of this workgroup is done
  if (valid) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int j = c + SOLVE_TPR * q;
      if (j < p) a21[(size_t)j * lda + row] = x[q];
    }
  }
}

int launch_solve(int n, int p, double* a, int lda, const int* perm, const int* piv,
                 const double* d, const int* nelim, hipStream_t stream) {
  const int r = n - p;
  if (r <= 0 || p <= 0) return 0;
  const int nc = (p + SOLVE_TPR - 1) / SOLVE_TPR;
  dim3 grid((r + SOLVE_RPB - 1) / SOLVE_RPB);
#define CTP_SOLVE_CASE(NCV)                                                                    \
  if (nc <= NCV) {                                                                             \
    solve_rows_kernel<NCV><<<grid, SOLVE_THREADS, 0, stream>>>(r, p, a, lda, perm, piv, d, nelim); \
  } else
  CTP_SOLVE_CASE(1) CTP_SOLVE_CASE(2) CTP_SOLVE_CASE(4) CTP_SOLVE_CASE(8) CTP_SOLVE_CASE(16)
  CTP_SOLVE_CASE(32) CTP_SOLVE_CASE(64) { return -2; }
#undef CTP_SOLVE_CASE
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
