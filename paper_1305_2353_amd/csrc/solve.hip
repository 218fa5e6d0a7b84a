// Solve task on the column-permuted A21 (Section 1; Fig. 4.1 (d)-(e)).
//
// Every row of A21 is independent: with x = row of A21 P^T,
//     W_E  = x_E (L_EE^T)^-1          (forward substitution, L unit lower)
//     x_d' = x_d - W_E L_dE^T         (delayed columns)
//     L21  = W_E D^-1                 (1x1 and 2x2 blocks)
// W = L21 D stays in the workspace as the Form's second operand.  The
// kernels are described with solve_rl_body below; after threshold partial
// pivoting (which leaves L21 in the panel) form_w_kernel only writes W.

#include <type_traits>

#include "common.h"

namespace ctp {

typedef double d4s __attribute__((ext_vector_type(4)));
typedef float f4s __attribute__((ext_vector_type(4)));

// 2x2 pivot inverse entries, scaled as in the pivot search.
CTP_DEV void inv2x2(double a11, double a21, double a22, double& i11, double& i21, double& i22) {
  const double s = 1.0 / fmax(fmax(fabs(a11), fabs(a21)), fabs(a22));
  const double det = (a22 * s) * a11 - (a21 * s) * a21;
  const double f = s / det;
  i11 = f * a22;
  i21 = -(f * a21);
  i22 = f * a11;
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

// ---------------------------------------------------------------------------
// Blocked triangular solve: W = X L'^-T, X = A21 P^T, with L' the unit lower
// triangular p x p matrix of the factorization modified so that
//   * the entry below the first column of a 2x2 pivot (it holds D) is 0,
//   * the column of a zero pivot is 0 below the diagonal (its W is dropped),
//   * a delayed column (position >= nelim) is a unit column; its row keeps
//     the L_dE entries,
// so that the rows of the result are [ W_E , X_d - W_E L_dE^T ]: W of the
// eliminated columns and the updated delayed columns at once.  The columns
// go in panels of up to 256:
//   lc       L' (masked as above) into a compact p x p copy (X is not
//            copied: the diagonal kernels read it from A21 through perm);
//   diag     per panel: a workgroup of four waves takes 64 rows (16 per
//            wave) and solves them against the panel's diagonal block of
//            L', right-looking in 16-column blocks held as FP64
//            matrix-core accumulators: forward substitution inside the
//            16 x 16 diagonal block (column kk broadcast to the lanes of
//            its rows by a DPP row share), then the product with the
//            block's W subtracted from the later blocks of the panel on the
//            matrix cores.  The columns of earlier panels enter first, as
//            one product -W_1 L'_21^T into the same accumulators.  The L'
//            columns a step needs are shared by the four waves through a
//            double-buffered LDS copy;
//   scale    L21 = W D^-1 into the panel (delayed columns copied
//            unscaled), W kept in the workspace for the Form.
// Every step is exact substitution or an exact product: the accuracy is
// that of a blocked forward substitution.
// ---------------------------------------------------------------------------

constexpr int SV_PANEL = 256;             // columns per panel
constexpr int SV_LDW = 17;                // LDS stride of a 16-entry column (padded)

// Column j of L' (rows 0..p-1) into lc.
CTP_DEV void solve_lc_body(int p, const double* __restrict__ a, int lda, const int* __restrict__ piv,
                           const int* __restrict__ nelim_p, double* __restrict__ lc, int j) {
  const int nelim = min(max(*nelim_p, 0), p);
  const int pj = piv[j];
  const bool col = j < nelim && pj != PIV_ZERO;
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const bool keep = col && i > j && !(i == j + 1 && pj == PIV_2X2_FIRST);
    lc[(size_t)j * p + i] = keep ? a[(size_t)j * lda + i] : (i == j ? 1.0 : 0.0);
  }
}

// Column j of L' (the diagonal kernels read X straight from A21 through
// perm, so nothing else is gathered).
__global__ __launch_bounds__(256) void solve_lc_kernel(int p, const double* __restrict__ a, int lda,
                                                     const int* __restrict__ piv, const int* __restrict__ nelim_p,
                                                     double* __restrict__ lc) {
  solve_lc_body(p, a, lda, piv, nelim_p, lc, blockIdx.x);
}

// DPP move of a double: every lane <- lane k of its row of 16.
constexpr int SV_ROW_SHARE = 0x150;

template <int K>
CTP_DEV double sv_share(double x) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(bits & 0xffffffffull), SV_ROW_SHARE + K, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(bits >> 32), SV_ROW_SHARE + K, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int K>
CTP_DEV float sv_share(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), SV_ROW_SHARE + K, 0xf, 0xf, true));
}

// Arithmetic of the diagonal-panel kernel, by precision (opts.prec).
// 0, FP64: the FP64 matrix cores (v_mfma_f64_16x16x4f64); accumulator
//    element q of lane l is row l/16 + 4q, column l % 16.
// 1, FP32: X and L' rounded to FP32, the substitution in FP32, the products
//    on the FP32 matrix cores (v_mfma_f32_16x16x4f32, the same operand
//    fragments as FP64: lane l holds A(l % 16, k0 + l/16), B(k0 + l/16,
//    l % 16)); accumulator element q of lane l is row 4(l/16) + q, column
//    l % 16.
// 2, BF16: as FP32, but the products take BF16 operands
//    (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation: lane l holds A(l % 16,
//    4(l/16) + v) and B(4(l/16) + v, l % 16), v = 0..3).
// X is read from and written to the FP64 workspace in every case.
typedef short s4s __attribute__((ext_vector_type(4)));
typedef __bf16 b4s __attribute__((ext_vector_type(4)));

template <int PREC> struct SvArith;
template <> struct SvArith<0> {
  using T = double;
  using acc_t = d4s;
  static CTP_DEV int row(int ga, int q) { return ga + 4 * q; }
  static CTP_DEV acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct SvArith<1> {
  using T = float;
  using acc_t = f4s;
  static CTP_DEV int row(int ga, int q) { return 4 * ga + q; }
  static CTP_DEV acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct SvArith<2> {
  using T = float;
  using acc_t = f4s;
  static CTP_DEV int row(int ga, int q) { return 4 * ga + q; }
  static CTP_DEV acc_t mma16(const float* a, const float* b, acc_t c) {
    const b4s ab = {(__bf16)a[0], (__bf16)a[1], (__bf16)a[2], (__bf16)a[3]};
    const b4s bb = {(__bf16)b[0], (__bf16)b[1], (__bf16)b[2], (__bf16)b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4s, ab), __builtin_bit_cast(s4s, bb), c, 0,
                                                      0, 0);
  }
};

// LDS of the diagonal-panel kernel: the 16 columns of L' of the current
// block (rows from the block's first column to the end of the panel), two
// buffers, and a transposition area per wave.  Entry (row j0 + i, column j0
// + kk) of block b's buffer is at lbuf[kk * SV_LROWS + i]; the stride (16
// mod 32 doubles) puts the four 16-lane groups of a wave, which read four
// consecutive columns, on distinct banks.
constexpr int SV_LROWS = SV_PANEL + 16;
constexpr int SV_LBUF = 16 * SV_LROWS;

// LDS-only workgroup barrier: outstanding global loads and stores are not
// waited for (the compiler waits for each load where its value is used).
CTP_DEV void sv_lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One workgroup of four waves, 16 rows each: rows r0.. of the panel of
// columns c0..c0+16 NBP-1 of x (in place).  Accumulator layout: element q of
// lane l is row l/16 + 4q, column l % 16 of its block.
//
// acc[k] holds block b + k while block b is worked: the accumulators of the
// blocks to come collect the updates of earlier blocks, and a block's X is
// added one iteration ahead (loaded at the start of the iteration, added at
// its end, when the array has moved down by one).  Each iteration loads one
// block of X and stores one, and the L' columns of the next block travel
// through registers (fetched at the start of an iteration, written to LDS
// at its end): the memory traffic is spread over the whole loop and hidden
// behind the arithmetic of the current block.
//
// xsrc (optional): the panel's own X columns are read from A21 (xsrc, leading
// dimension ldsrc) through perm instead of from x, so that no gather pass
// copies them into the workspace first; the results go to x as before.
template <int PREC, int NBP>
CTP_DEV void solve_diag_wg(int r, int p, int c0, const int* __restrict__ piv, int nelim, double* __restrict__ x,
                           int ldx, const double* __restrict__ lc, typename SvArith<PREC>::T* lsh,
                           typename SvArith<PREC>::T* stage, int r0, const double* __restrict__ xsrc = nullptr,
                           int ldsrc = 0, const int* __restrict__ perm = nullptr) {
  using A = SvArith<PREC>;
  using T = typename A::T;
  using acc_t = typename A::acc_t;
  const int tid = threadIdx.x, lane = tid & 63;
  const int ga = lane >> 4, c = lane & 15;
  const int nbe = min(NBP, (nelim - c0 + 15) / 16);   // blocks of the panel with eliminated columns
  const int nkc = (min(c0, nelim) + 7) / 8;            // 8-column chunks of earlier eliminated columns
  if (nbe <= 0 && nkc == 0 && !xsrc) return;           // nothing updates this panel: X is final
  const int nb = min(NBP, (p - c0 + 15) / 16);         // blocks with columns below p
  int rows[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) rows[q] = min(r0 + A::row(ga, q), r - 1);
  // bit b: column c0 + 16 b + c has a zero pivot
  int pv[NBP];
#pragma unroll
  for (int b = 0; b < NBP; ++b) pv[b] = piv[min(c0 + 16 * b + c, p - 1)];
  unsigned zb = 0;
#pragma unroll
  for (int b = 0; b < NBP; ++b) zb |= (c0 + 16 * b + c < p && pv[b] == PIV_ZERO ? 1u : 0u) << b;
  // L' staging: thread t carries column j0 + t/16, rows j0 + t%16 + 16 m.
  // Rows and columns past p are clamped to p - 1: they only reach lanes and
  // blocks of columns past p, which are never stored.
  // A block is staged in two halves (m below or from NH), to halve the
  // registers that carry it.
  const int skk = tid >> 4, si = tid & 15;
  constexpr int NH = (NBP + 1) / 2;
  T lreg[NH];
  auto fetch_l = [&](int b, int half) __attribute__((always_inline)) {
    const int j0 = c0 + 16 * b;
    const int col = j0 + skk;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int m = half * NH + h;
      const int row = j0 + si + 16 * m;
      if (m < NBP - b) lreg[h] = (T)lc[(size_t)min(col, p - 1) * p + min(row, p - 1)];
    }
  };
  auto put_l = [&](int b, int half) __attribute__((always_inline)) {
    T* buf = lsh + (b & 1) * SV_LBUF + skk * SV_LROWS + si;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int m = half * NH + h;
      if (m < NBP - b) buf[16 * m] = lreg[h];
    }
  };
  // (direct reads: the A21 column behind position j is perm[j]; load_x is
  // issued an iteration ahead of its use, which covers the extra load)
  auto load_x = [&](int b, T* v) __attribute__((always_inline)) {
    const int j = min(c0 + 16 * b + c, p - 1);
    if (xsrc) {
      const double* col = xsrc + (size_t)perm[j] * ldsrc;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (T)col[rows[q]];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (T)x[(size_t)j * ldx + rows[q]];
    }
  };
  // a wave with rows below r stores all 16 of its rows: the rows past r
  // (up to the next multiple of 16) are padding of x, whose leading
  // dimension is r rounded up to a multiple of 32
  const bool wave_rows = r0 < r;
  auto store_x = [&](int b, const T* v) __attribute__((always_inline)) {
    const int j = c0 + 16 * b + c;
    if (wave_rows && j < p) {
#pragma unroll
      for (int q = 0; q < 4; ++q) x[(size_t)j * ldx + r0 + A::row(ga, q)] = (double)v[q];
    }
  };
  if (nbe <= 0 && nkc == 0) {
    // nothing updates this panel: its X, read from A21, is final
    for (int b = 0; b < nb; ++b) {
      T v[4];
      load_x(b, v);
      store_x(b, v);
    }
    return;
  }
  acc_t acc[NBP];
#pragma unroll
  for (int k = 0; k < NBP; ++k) acc[k] = acc_t{0, 0, 0, 0};
  if (nkc > 0) {
    // the earlier panels' eliminated columns: acc[k] = -W(:, 0:8 nkc)
    // L'(c0 + 16 k + :, 0:8 nkc)^T, eight columns at a time (thread t
    // stages L' column 8 kc + t/32, rows c0 + t%32 + 32 m); A fragment u of
    // lane l is W(row l % 16, column 8 kc + l/16 + 4u)
    const int ra = min(r0 + c, r - 1);
    const int ucol = tid >> 5, urow = tid & 31;
    auto fetch_u = [&](int kc) __attribute__((always_inline)) {
      const int col = 8 * kc + ucol;
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        const int row = c0 + urow + 32 * m;
        lreg[m] = (T)lc[(size_t)col * p + min(row, p - 1)];
      }
    };
    auto put_u = [&](int kc) __attribute__((always_inline)) {
      T* buf = lsh + (kc & 1) * SV_LBUF + ucol * SV_LROWS + urow;
#pragma unroll
      for (int m = 0; m < NH; ++m) buf[32 * m] = lreg[m];
    };
    // BF16 takes 16 k per product: the lanes with l/16 < 2 carry the
    // chunk's eight columns (4(l/16) + v), the others zeros
    constexpr int NA = PREC == 2 ? 4 : 2;
    auto load_a = [&](int kc, T* v) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        if (PREC == 2) v[u] = ga < 2 ? (T)x[(size_t)(8 * kc + 4 * ga + u) * ldx + ra] : (T)0;
        else v[u] = (T)x[(size_t)(8 * kc + ga + 4 * u) * ldx + ra];
      }
    };
    T an[NA];
    load_a(0, an);
    fetch_u(0);
    put_u(0);
    for (int kc = 0; kc < nkc; ++kc) {
      sv_lds_barrier();
      const T* lb = lsh + (kc & 1) * SV_LBUF;
      T af[NA];
#pragma unroll
      for (int u = 0; u < NA; ++u) af[u] = -an[u];
      if (kc + 1 < nkc) {
        load_a(kc + 1, an);
        fetch_u(kc + 1);
      }
#pragma unroll
      for (int k = 0; k < NBP; ++k) {
        if (k >= nb) continue;
        if constexpr (PREC == 2) {
          T bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) bv[u] = ga < 2 ? lb[(4 * ga + u) * SV_LROWS + 16 * k + c] : (T)0;
          acc[k] = A::mma16(af, bv, acc[k]);
        } else {
          const T b0 = lb[ga * SV_LROWS + 16 * k + c];
          const T b1 = lb[(4 + ga) * SV_LROWS + 16 * k + c];
          acc[k] = A::mma(af[0], b0, acc[k]);
          acc[k] = A::mma(af[1], b1, acc[k]);
        }
      }
      if (kc + 1 < nkc) put_u(kc + 1);
    }
    // every wave is done with both buffers before the panel's own blocks
    // are staged
    sv_lds_barrier();
  }
  T xn[4];
  load_x(0, xn);
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[0][q] += xn[q];
  if (nbe > 0) {
    fetch_l(0, 0);
    put_l(0, 0);
    fetch_l(0, 1);
    put_l(0, 1);
  }
  for (int b = 0; b < nb; ++b) {
    // block b's L' columns are in LDS (every thread's share); the other
    // buffer was last read in the previous iteration
    sv_lds_barrier();
    const T* lb = lsh + (b & 1) * SV_LBUF;
    if (b + 1 < nb) load_x(b + 1, xn);
    if (b + 1 < nbe) fetch_l(b + 1, 0);
    T xv[4] = {acc[0][0], acc[0][1], acc[0][2], acc[0][3]};
    if (b < nbe) {
      const int j0 = c0 + 16 * b;
      const int kkend = min(16, nelim - j0);
      const unsigned zmask = (unsigned)__ballot((zb >> b) & 1u) & 0xffffu;
      auto step = [&](auto kkc) __attribute__((always_inline)) {
        constexpr int kk = decltype(kkc)::value;
        if (kk >= kkend) return;
        if ((zmask >> kk) & 1u) {
          // a zero pivot: its column of L is zero
#pragma unroll
          for (int q = 0; q < 4; ++q) xv[q] = c == kk ? (T)0 : xv[q];
        }
        // L'(j0 + c, j0 + kk): zero above the diagonal, the unit diagonal
        // itself must not update
        const T lv = c == kk ? (T)0 : lb[kk * SV_LROWS + c];
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[q] = fma(-sv_share<kk>(xv[q]), lv, xv[q]);
      };
      step(std::integral_constant<int, 0>{});
      step(std::integral_constant<int, 1>{});
      step(std::integral_constant<int, 2>{});
      step(std::integral_constant<int, 3>{});
      step(std::integral_constant<int, 4>{});
      step(std::integral_constant<int, 5>{});
      step(std::integral_constant<int, 6>{});
      step(std::integral_constant<int, 7>{});
      step(std::integral_constant<int, 8>{});
      step(std::integral_constant<int, 9>{});
      step(std::integral_constant<int, 10>{});
      step(std::integral_constant<int, 11>{});
      step(std::integral_constant<int, 12>{});
      step(std::integral_constant<int, 13>{});
      step(std::integral_constant<int, 14>{});
      step(std::integral_constant<int, 15>{});
      if (b + 1 < nb) {
        // W of the block's eliminated columns as A fragments (row l % 16,
        // column l/16 + 4u), through the wave's staging area
        if (b + 1 < nbe) {
          put_l(b + 1, 0);
          fetch_l(b + 1, 1);
        }
        const bool elim = j0 + c < nelim;
#pragma unroll
        for (int q = 0; q < 4; ++q) stage[c * SV_LDW + A::row(ga, q)] = elim ? xv[q] : (T)0;
        // (BF16: row l % 16, columns 4(l/16) + v)
        T af[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          af[u] = PREC == 2 ? -stage[(4 * ga + u) * SV_LDW + c] : -stage[(4 * u + ga) * SV_LDW + c];
        // block b + k: B fragment L'(j0 + 16 k + l % 16, j0 + 4u + l/16)
        // (BF16: L'(j0 + 16 k + l % 16, j0 + 4(l/16) + v))
#pragma unroll
        for (int k = 1; k < NBP; ++k) {
          if (k >= nb - b) continue;
          T bf[4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            bf[u] = PREC == 2 ? lb[(4 * ga + u) * SV_LROWS + 16 * k + c] : lb[(4 * u + ga) * SV_LROWS + 16 * k + c];
          if constexpr (PREC == 2) {
            acc[k] = A::mma16(af, bf, acc[k]);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[k] = A::mma(af[u], bf[u], acc[k]);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k + 1 < NBP; ++k) acc[k] = acc[k + 1];
    acc[NBP - 1] = acc_t{0, 0, 0, 0};
    if (b + 1 < nb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[0][q] += xn[q];
      // here, not after the stores below: a wait for X placed after them
      // would wait for the stores too
      asm volatile("" ::"v"(acc[0][0]), "v"(acc[0][1]), "v"(acc[0][2]), "v"(acc[0][3]) : "memory");
    }
    if (b + 1 < nbe) put_l(b + 1, 1);
    store_x(b, xv);
  }
}

template <int PREC, int NBP>
__global__ __launch_bounds__(256, 2) void solve_diag_kernel(int r, int p, int c0, const int* __restrict__ piv,
                                                          const int* __restrict__ nelim_p, double* __restrict__ x,
                                                          int ldx, const double* __restrict__ lc,
                                                          const double* __restrict__ a21, int lda,
                                                          const int* __restrict__ perm) {
  using T = typename SvArith<PREC>::T;
  __shared__ T lsh[2 * SV_LBUF];
  __shared__ T stage[4][16 * SV_LDW];
  const int wave = threadIdx.x >> 6;
  if ((int)blockIdx.x * 64 >= r) return;
  // waves past the last row still take part in the staging and barriers
  const int r0 = (blockIdx.x * 4 + wave) * 16;
  solve_diag_wg<PREC, NBP>(r, p, c0, piv, min(max(*nelim_p, 0), p), x, ldx, lc, lsh, stage[wave], r0, a21, lda,
                           perm);
}

// Rows chunk*4096.. of column k: the workspace holds W (eliminated) or the
// final delayed column; the panel gets L21 = W D^-1 or the delayed column.
// The thread of the first column of a 2x2 pivot writes both columns.
CTP_DEV void solve_scale_body(int r, int p, double* __restrict__ a, int lda, const int* __restrict__ piv,
                              const double* __restrict__ d, const int* __restrict__ nelim_p,
                              const double* __restrict__ w, int ldw, int k, int chunk) {
  const int nelim = min(max(*nelim_p, 0), p);
  const int pk = piv[k];
  if (k < nelim && pk == PIV_2X2_SECOND) return;
  double* a21 = a + p;
  const int i0 = chunk * 4096;
  const int i1 = min(r, i0 + 4096);
  const double* wk = w + (size_t)k * ldw;
  double* ak = a21 + (size_t)k * lda;
  if (k >= nelim) {
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) ak[i] = wk[i];
  } else if (pk == PIV_1X1) {
    const double rd = 1.0 / d[2 * k];
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) ak[i] = wk[i] * rd;
  } else if (pk == PIV_ZERO) {
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) ak[i] = 0.0;
  } else {
    double i11, i21, i22;
    inv2x2(d[2 * k], d[2 * k + 1], d[2 * k + 2], i11, i21, i22);
    double* ak1 = ak + lda;
    const double* wk1 = wk + ldw;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const double w1 = wk[i], w2 = wk1[i];
      ak[i] = w1 * i11 + w2 * i21;
      ak1[i] = w1 * i21 + w2 * i22;
    }
  }
}

__global__ __launch_bounds__(256) void solve_scale_kernel(int r, int p, double* __restrict__ a, int lda,
                                                        const int* __restrict__ piv, const double* __restrict__ d,
                                                        const int* __restrict__ nelim_p, const double* __restrict__ w,
                                                        int ldw) {
  solve_scale_body(r, p, a, lda, piv, d, nelim_p, w, ldw, blockIdx.y, blockIdx.x);
}

// Batched: the node is blockIdx.z (L', scale) or blockIdx.y (diag).
__global__ __launch_bounds__(256) void solve_lc_batch_kernel(const BatchNode* __restrict__ nodes, int method) {
  const BatchNode& nd = nodes[blockIdx.z];
  if ((int)blockIdx.y >= nd.p || nd.n - nd.p <= 0) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  solve_lc_body(nd.p, nd.a, nd.lda, nd.piv, nd.nelim, reinterpret_cast<double*>(nd.work + ws.lc_off), blockIdx.y);
}

template <int PREC, int NBP>
__global__ __launch_bounds__(256, 2) void solve_diag_batch_kernel(const BatchNode* __restrict__ nodes, int method, int c0) {
  using T = typename SvArith<PREC>::T;
  __shared__ T lsh[2 * SV_LBUF];
  __shared__ T stage[4][16 * SV_LDW];
  const BatchNode& nd = nodes[blockIdx.y];
  const int r = nd.n - nd.p;
  const int wave = threadIdx.x >> 6;
  if ((int)blockIdx.x * 64 >= r || c0 >= nd.p) return;
  const int r0 = (blockIdx.x * 4 + wave) * 16;
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  // the node's panel may be narrower than NBP blocks: the extra blocks are
  // past p (their columns are neither read nor written)
  solve_diag_wg<PREC, NBP>(r, nd.p, c0, nd.piv, min(max(*nd.nelim, 0), nd.p), reinterpret_cast<double*>(nd.work + ws.w_off),
                     ws.ldw, reinterpret_cast<const double*>(nd.work + ws.lc_off), lsh, stage[wave], r0, nd.a + nd.p,
                     nd.lda, nd.perm);
}

__global__ __launch_bounds__(256) void solve_scale_batch_kernel(const BatchNode* __restrict__ nodes, int method) {
  const BatchNode& nd = nodes[blockIdx.z];
  const int r = nd.n - nd.p;
  if ((int)blockIdx.y >= nd.p || (int)blockIdx.x * 4096 >= r) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  solve_scale_body(r, nd.p, nd.a, nd.lda, nd.piv, nd.d, nd.nelim, reinterpret_cast<const double*>(nd.work + ws.w_off),
                   ws.ldw, blockIdx.y, blockIdx.x);
}


template <typename F>
static void solve_diag_dispatch(int nbp, F&& f) {
  if (nbp <= 4) f(std::integral_constant<int, 4>{});
  else if (nbp <= 8) f(std::integral_constant<int, 8>{});
  else f(std::integral_constant<int, 16>{});
}

// prec 0: FP64 throughout; 1 / 2: the triangular solve in FP32 on the FP32 /
// BF16 matrix cores (FP32 accumulation); the copy of L', the 2x2 inverses and
// D^-1 stay FP64.
int launch_solve(int n, int p, double* a, int lda, const int* perm, const int* piv, const double* d,
                 const int* nelim, double* w, int ldw, double* lc, int prec, hipStream_t stream) {
  const int r = n - p;
  if (r <= 0 || p <= 0) return 0;
  const dim3 cols((r + 4095) / 4096, p);
  // L' only: the diagonal kernels read X from A21 through perm themselves
  solve_lc_kernel<<<p, 256, 0, stream>>>(p, a, lda, piv, nelim, lc);
  const unsigned grid = (unsigned)((r + 63) / 64);
  const double* a21 = a + p;
  for (int c0 = 0; c0 < p; c0 += SV_PANEL) {
    const int nbp = (min(SV_PANEL, p - c0) + 15) / 16;
    solve_diag_dispatch(nbp, [&](auto k) {
      constexpr int NBP = decltype(k)::value;
      if (prec == 1)
        solve_diag_kernel<1, NBP><<<grid, 256, 0, stream>>>(r, p, c0, piv, nelim, w, ldw, lc, a21, lda, perm);
      else if (prec == 2)
        solve_diag_kernel<2, NBP><<<grid, 256, 0, stream>>>(r, p, c0, piv, nelim, w, ldw, lc, a21, lda, perm);
      else
        solve_diag_kernel<0, NBP><<<grid, 256, 0, stream>>>(r, p, c0, piv, nelim, w, ldw, lc, a21, lda, perm);
    });
  }
  solve_scale_kernel<<<cols, 256, 0, stream>>>(r, p, a, lda, piv, d, nelim, w, ldw);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

int launch_solve_batch(int count, const BatchNode* nodes, int method, int max_p, int max_r, int prec,
                       hipStream_t stream) {
  if (count <= 0 || max_r <= 0 || max_p <= 0) return 0;
  const dim3 cols((max_r + 4095) / 4096, max_p, count);
  solve_lc_batch_kernel<<<dim3(1, max_p, count), 256, 0, stream>>>(nodes, method);
  const dim3 grid((max_r + 63) / 64, count);
  for (int c0 = 0; c0 < max_p; c0 += SV_PANEL) {
    const int nbp = (min(SV_PANEL, max_p - c0) + 15) / 16;
    solve_diag_dispatch(nbp, [&](auto k) {
      constexpr int NBP = decltype(k)::value;
      if (prec == 1) solve_diag_batch_kernel<1, NBP><<<grid, 256, 0, stream>>>(nodes, method, c0);
      else if (prec == 2) solve_diag_batch_kernel<2, NBP><<<grid, 256, 0, stream>>>(nodes, method, c0);
      else solve_diag_batch_kernel<0, NBP><<<grid, 256, 0, stream>>>(nodes, method, c0);
    });
  }
  solve_scale_batch_kernel<<<cols, 256, 0, stream>>>(nodes, method);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
