// Solve task on the column-permuted A21 (Section 1; Fig. 4.1 (d)-(e)).
//
// Every row of A21 is independent: with x = row of A21 P^T,
//     W_E  = x_E (L_EE^T)^-1          (forward substitution, L unit lower)
//     x_d' = x_d - W_E L_dE^T         (delayed columns)
//     L21  = W_E D^-1                 (1x1 and 2x2 blocks)
//
// Two kernels:
//  1. gather: W = A21 P^T column by column into the workspace (the
//     permutation is applied once, as a copy; the panel can then be
//     overwritten in place without losing original columns);
//  2. blocked left-looking triangular solve on the matrix cores.  One wave
//     owns 16 rows and walks the p columns in blocks of 16:
//        X_b = W_b - W_{<b} L_{b,<b}^T        (v_mfma_f64_16x16x4, K = 16b)
//        forward substitution inside the 16 x 16 diagonal block of L
//        (pivot values broadcast across the lanes that hold a row);
//     the solved block goes back to the workspace (the A operand of later
//     blocks) and, multiplied by D^-1, to the panel as L21.  A 2x2 pivot
//     that straddles two blocks is finished when the second block is done.
//  Delayed columns (positions >= nelim) receive the GEMM and in-block
//  updates from every eliminated column and are written unscaled.

#include "common.h"

namespace ctp {

typedef double d4s __attribute__((ext_vector_type(4)));

constexpr int SOLVE_THREADS = 256;   // 4 waves, 16 rows each
constexpr int SOLVE_ROWS = 64;

// Column j of W = A21 P^T (rows chunk*4096 ..), and with the first chunk
// column j of A11 into the compact p x p copy lc: the solve's L operand,
// whose columns are then 8p bytes apart instead of 8 lda bytes (every step
// of the solve reads four columns of L; at lda = 100000 those sit in four
// different pages).
CTP_DEV void solve_gather_body(int r, int p, const double* __restrict__ a, int lda, const int* __restrict__ perm,
                               double* __restrict__ w, int ldw, double* __restrict__ lc, int j, int chunk) {
  const double* src = a + p + (size_t)perm[j] * lda;
  double* dst = w + (size_t)j * ldw;
  const int i0 = chunk * 4096;
  const int i1 = min(r, i0 + 4096);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) dst[i] = src[i];
  if (chunk == 0)
    for (int i = threadIdx.x; i < p; i += blockDim.x) lc[(size_t)j * p + i] = a[(size_t)j * lda + i];
}

__global__ __launch_bounds__(256) void solve_gather_kernel(int r, int p, const double* __restrict__ a, int lda,
                                                         const int* __restrict__ perm, double* __restrict__ w,
                                                         int ldw, double* __restrict__ lc) {
  solve_gather_body(r, p, a, lda, perm, w, ldw, lc, blockIdx.y, blockIdx.x);
}

// 2x2 pivot inverse entries, scaled as in the pivot search.
CTP_DEV void inv2x2(double a11, double a21, double a22, double& i11, double& i21, double& i22) {
  const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
  const double det = (a22 * s) * a11 - (a21 * s) * a21;
  const double f = s / det;
  i11 = f * a22;
  i21 = -(f * a21);
  i22 = f * a11;
}

__shared__ int slv_piv[CTP_MAX_P + 32];
__shared__ double slv_d[2 * CTP_MAX_P + 64];

CTP_DEV void solve_mfma_body(int r, int p, double* __restrict__ a, int lda, const int* __restrict__ piv,
                             const double* __restrict__ d, const int* __restrict__ nelim_p,
                             double* __restrict__ w, int ldw, const double* __restrict__ lc, int bx) {
  int* piv_s = slv_piv;
  double* d_s = slv_d;
  for (int k = threadIdx.x; k < p + 32; k += SOLVE_THREADS) {
    piv_s[k] = k < p ? piv[k] : PIV_DELAYED;
    d_s[2 * k] = k < p ? d[2 * k] : 0.0;
    d_s[2 * k + 1] = k < p ? d[2 * k + 1] : 0.0;
  }
  __syncthreads();

  const int nelim = min(max(*nelim_p, 0), p);
  const int lane = threadIdx.x & 63;
  const int r0 = (bx * SOLVE_THREADS + (int)threadIdx.x) / 64 * 16;   // first row of this wave
  if (r0 >= r) return;
  double* a21 = a + p;
  const int ga = lane >> 4;          // accumulator rows ga + 4q
  const int c = lane & 15;           // accumulator column
  const int fr = lane & 15;          // fragment row (A operand) / column (B operand)
  const int fk = lane >> 4;          // fragment k
  const int rmax = r - 1;
  const int arow = min(r0 + fr, rmax);
  int rows[4];
  bool rv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rows[q] = r0 + ga + 4 * q;
    rv[q] = rows[q] < r;
    rows[q] = min(rows[q], rmax);
  }

  const int nb = (p + 15) / 16;
  double carry[4] = {0.0, 0.0, 0.0, 0.0};   // previous block's column 15 (lanes c == 15)
  for (int b = 0; b < nb; ++b) {
    const int j0 = 16 * b;
    const int jc = j0 + c;                   // this lane's column
    const bool cv = jc < p;
    const int jcc = min(jc, p - 1);
    d4s acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = w[(size_t)jcc * ldw + rows[q]];

    // X_b -= W_{<b} L_{b,<b}^T over the eliminated columns k < min(j0, nelim):
    // 16 columns of k per step on four independent accumulators (the MFMAs
    // of a step do not wait for each other), the next step's fragments
    // loaded while the current step's products run.  Every step but the
    // last is full and cannot meet the 2x2 pivot that may straddle the
    // block boundary (k = j0 - 1), so it runs on pointer increments without
    // masks; the last step takes the masked loads.
    const int kend = min(j0, nelim);
    const int bj = min(j0 + fr, p - 1);      // B operand: row j0+fr of L
    const bool brow = j0 + fr < p;
    if (kend > 0) {
      const int klast = (kend - 1) / 16 * 16;   // first k of the last step
      d4s part[4];
      part[0] = acc;
#pragma unroll
      for (int u = 1; u < 4; ++u) part[u] = d4s{0.0, 0.0, 0.0, 0.0};
      const size_t wstep = (size_t)4 * ldw, lstep = (size_t)4 * p;
      const double* wp = w + (size_t)fk * ldw + arow;   // W(arow, k), k = fk + 4u + k0
      const double* lp = lc + (size_t)fk * p + bj;      // L(bj, k)
      double an[4], bn[4];
      if (klast > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          an[u] = -wp[u * wstep];
          bn[u] = brow ? lp[u * lstep] : 0.0;
        }
      }
      for (int k0 = 0; k0 < klast; k0 += 16) {
        double ac[4], bc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ac[u] = an[u];
          bc[u] = bn[u];
        }
        wp += 4 * wstep;
        lp += 4 * lstep;
        if (k0 + 16 < klast) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            an[u] = -wp[u * wstep];
            bn[u] = brow ? lp[u * lstep] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) part[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u], bc[u], part[u], 0, 0, 0);
      }
      // last step: k = klast .. kend-1
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = klast + 4 * u + fk;
        const bool kv = k < kend;
        const int kc = kv ? k : 0;
        double af = w[(size_t)kc * ldw + arow];
        double bf = CM(lc, bj, kc, p);
        // L(j0, j0-1) is the in-block entry of a 2x2 pivot straddling the
        // block boundary: it holds D, not L.
        const bool straddle = (j0 + fr == k + 1) && piv_s[kc] == PIV_2X2_FIRST;
        af = kv ? -af : 0.0;
        bf = (kv && !straddle && brow) ? bf : 0.0;
        part[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, part[u], 0, 0, 0);
      }
      acc = (part[0] + part[1]) + (part[2] + part[3]);
    }

    // forward substitution inside the block
    const int kkend = min(16, nelim - j0);
    for (int kk = 0; kk < kkend; ++kk) {
      const int k = j0 + kk;
      double lv = CM(lc, jcc, k, p);
      const bool keep = cv && c > kk && !(c == kk + 1 && piv_s[k] == PIV_2X2_FIRST);
      lv = keep ? lv : 0.0;
      if (piv_s[k] == PIV_ZERO && c == kk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = 0.0;
      }
      const int src = (lane & 48) | kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double xk = __shfl(acc[q], src, 64);
        acc[q] = fma(-xk, lv, acc[q]);
      }
    }

    // solved block -> workspace (A operand of later blocks)
    if (cv && jc < nelim) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (rv[q]) w[(size_t)jc * ldw + rows[q]] = acc[q];
    }
    __threadfence_block();

    // outputs: L21 = W D^-1 for eliminated columns, raw for delayed ones
    const int pt = piv_s[jcc];
    double nxt[4], prv[4], prevc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      nxt[q] = __shfl(acc[q], (lane + 1) & 63, 64);
      prv[q] = __shfl(acc[q], (lane + 63) & 63, 64);
      prevc[q] = __shfl(carry[q], (lane & 48) | 15, 64);
    }
    if (cv) {
      double i11 = 0.0, i21 = 0.0, i22 = 0.0;
      if (jc < nelim && (pt == PIV_2X2_FIRST || pt == PIV_2X2_SECOND)) {
        const int k = pt == PIV_2X2_FIRST ? jc : jc - 1;
        inv2x2(d_s[2 * k], d_s[2 * k + 1], d_s[2 * k + 2], i11, i21, i22);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!rv[q]) continue;
        double* rowp = a21 + rows[q];
        if (jc >= nelim) {
          rowp[(size_t)jc * lda] = acc[q];
        } else if (pt == PIV_1X1) {
          rowp[(size_t)jc * lda] = acc[q] / d_s[2 * jc];
        } else if (pt == PIV_ZERO) {
          rowp[(size_t)jc * lda] = 0.0;
        } else if (pt == PIV_2X2_FIRST) {
          if (c < 15) rowp[(size_t)jc * lda] = acc[q] * i11 + nxt[q] * i21;
          // c == 15: finished with the next block
        } else {
          const double w1 = c > 0 ? prv[q] : prevc[q];
          const double w2 = acc[q];
          rowp[(size_t)jc * lda] = w1 * i21 + w2 * i22;
          if (c == 0) rowp[(size_t)(jc - 1) * lda] = w1 * i11 + w2 * i21;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) carry[q] = acc[q];
  }
}

__global__ __launch_bounds__(SOLVE_THREADS, 3) void solve_mfma_kernel(
    int r, int p, double* __restrict__ a, int lda, const int* __restrict__ piv,
    const double* __restrict__ d, const int* __restrict__ nelim_p, double* __restrict__ w, int ldw,
    const double* __restrict__ lc) {
  solve_mfma_body(r, p, a, lda, piv, d, nelim_p, w, ldw, lc, blockIdx.x);
}

// Batched: the node is blockIdx.z (gather) / blockIdx.y (solve).
__global__ __launch_bounds__(256) void solve_gather_batch_kernel(const BatchNode* __restrict__ nodes, int method) {
  const BatchNode& nd = nodes[blockIdx.z];
  const int r = nd.n - nd.p;
  if ((int)blockIdx.y >= nd.p || (int)blockIdx.x * 4096 >= r) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  solve_gather_body(r, nd.p, nd.a, nd.lda, nd.perm, reinterpret_cast<double*>(nd.work + ws.w_off), ws.ldw,
                    reinterpret_cast<double*>(nd.work + ws.lc_off), blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(SOLVE_THREADS, 3) void solve_mfma_batch_kernel(const BatchNode* __restrict__ nodes,
                                                                         int method) {
  const BatchNode& nd = nodes[blockIdx.y];
  const int r = nd.n - nd.p;
  if ((int)blockIdx.x * SOLVE_ROWS >= r) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  solve_mfma_body(r, nd.p, nd.a, nd.lda, nd.piv, nd.d, nd.nelim, reinterpret_cast<double*>(nd.work + ws.w_off),
                  ws.ldw, reinterpret_cast<const double*>(nd.work + ws.lc_off), blockIdx.x);
}

int launch_solve_batch(int count, const BatchNode* nodes, int method, int max_p, int max_r, hipStream_t stream) {
  if (count <= 0 || max_r <= 0 || max_p <= 0) return 0;
  solve_gather_batch_kernel<<<dim3((max_r + 4095) / 4096, max_p, count), 256, 0, stream>>>(nodes, method);
  solve_mfma_batch_kernel<<<dim3((max_r + SOLVE_ROWS - 1) / SOLVE_ROWS, count), SOLVE_THREADS, 0, stream>>>(nodes,
                                                                                                        method);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// W = L21 D for the eliminated columns, from L21 and D (used after the
// threshold-partial-pivoting factorization, which leaves L21 in the panel
// but no W).  One column per blockIdx.y; a 2x2 pivot mixes two columns.
__global__ __launch_bounds__(256) void form_w_kernel(int r, int p, const double* __restrict__ l21,
                                                     int lda, const int* __restrict__ piv,
                                                     const double* __restrict__ d,
                                                     const int* __restrict__ nelim_p,
                                                     double* __restrict__ w, int ldw) {
  const int k = blockIdx.y;
  const int nelim = min(max(*nelim_p, 0), p);
  if (k >= nelim) return;
  const int pt = piv[k];
  const int i0 = blockIdx.x * 4096;
  const int i1 = min(r, i0 + 4096);
  double* dst = w + (size_t)k * ldw;
  const double* lk = l21 + (size_t)k * lda;
  if (pt == PIV_2X2_FIRST || pt == PIV_2X2_SECOND) {
    const int k1 = pt == PIV_2X2_FIRST ? k : k - 1;     // first column of the pair
    const double* l1 = l21 + (size_t)k1 * lda;
    const double* l2 = l1 + lda;
    // column k of D restricted to the pair: (D(k1, k), D(k1+1, k))
    const double c1 = pt == PIV_2X2_FIRST ? d[2 * k1] : d[2 * k1 + 1];
    const double c2 = pt == PIV_2X2_FIRST ? d[2 * k1 + 1] : d[2 * k1 + 2];
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) dst[i] = l1[i] * c1 + l2[i] * c2;
  } else {
    const double dk = pt == PIV_1X1 ? d[2 * k] : 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) dst[i] = lk[i] * dk;
  }
}

int launch_form_w(int n, int p, const double* a, int lda, const int* piv, const double* d,
                  const int* nelim, double* w, int ldw, hipStream_t stream) {
  const int r = n - p;
  if (r <= 0 || p <= 0) return 0;
  dim3 gg((r + 4095) / 4096, p);
  form_w_kernel<<<gg, 256, 0, stream>>>(r, p, a + p, lda, piv, d, nelim, w, ldw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int launch_solve(int n, int p, double* a, int lda, const int* perm, const int* piv,
                 const double* d, const int* nelim, double* w, int ldw, double* lc, hipStream_t stream) {
  const int r = n - p;
  if (r <= 0 || p <= 0) return 0;
  dim3 gg((r + 4095) / 4096, p);
  solve_gather_kernel<<<gg, 256, 0, stream>>>(r, p, a, lda, perm, w, ldw, lc);
  solve_mfma_kernel<<<(r + SOLVE_ROWS - 1) / SOLVE_ROWS, SOLVE_THREADS, 0, stream>>>(r, p, a, lda, piv, d,
                                                                                 nelim, w, ldw, lc);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
