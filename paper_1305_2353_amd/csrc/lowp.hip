// Reduced-precision trailing update of the dense factorization:
//     C(i, j) -= sum_k L21(i, k) W(j, k),  i >= j,
// C the FP32 trailing matrix, L21 and W = L21 D the FP64 outputs of the
// panel's Solve, rounded to FP32 or BF16 for the matrix cores, FP32
// accumulation.  (The pivot search, the 2x2 inverses, L21 and W stay in
// FP64; only this product, which holds almost all of the flops, is cut.)
//
// 1. convert: L21 and W (column-major FP64) -> operand rows with k
//    contiguous (row-major, K padded with zeros to a multiple of 64), so a
//    lane's MFMA fragment is a contiguous run of k;
// 2. product: 128 x 128 output tiles, 4 waves (2 x 2) of 64 x 64, each a
//    4 x 4 array of 16 x 16 MFMA blocks; K staged through LDS in chunks of
//    BK (16 for FP32, 64 for BF16) with register prefetch of the next chunk.
//    FP32: v_mfma_f32_16x16x4f32, lane l holds A(l%16, k0 + l/16) and
//          B(k0 + l/16, l%16);
//    BF16: v_mfma_f32_16x16x32_bf16, lane l holds A(l%16, k0 + 8(l/16) + v)
//          and B(k0 + 8(l/16) + v, l%16), v = 0..7;
//    both: accumulator element q of lane l is row 4(l/16) + q, column l%16.
//    The product is taken as C^T's block (W fragments as the A operand), so
//    16 lanes of an accumulator hold 16 consecutive rows i of one column j
//    of C and the read-modify-write of C touches 64-byte runs (with L21 as
//    the A operand the rows of a lane group were 4 apart).

// The same product serves the supernode Form in reduced precision (opts
// prec fp32 / bf16): S = L21 W^T stored as FP64 into rows row0..row0+nrows-1
// of the lower triangle (column-major, or as the 128 x 128 tiles of
// CTP_FLAG_S_TILED), from operand rows the Solve converted once.

#include "common.h"

namespace ctp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));   // 16 raw bytes

constexpr int LP_BM = 128;
constexpr int LP_THREADS = 256;
constexpr int LP_KPAD = 64;   // operand rows padded to a multiple of this
constexpr int LP_NXCD = 8;
constexpr int LP_GROUP = 8;

template <typename T> struct LowpTraits;
// k per LDS chunk: 64 bytes of each row for FP32, 128 bytes for BF16
template <> struct LowpTraits<float> { static constexpr int PREC = 1; static constexpr int BK = 16; };
template <> struct LowpTraits<__bf16> { static constexpr int PREC = 2; static constexpr int BK = 64; };

size_t lowp_ops_bytes(int r, int kmax) {
  const size_t kp = align_up((size_t)(kmax > 0 ? kmax : 1), LP_KPAD);
  return 2 * align_up((size_t)(r > 0 ? r : 1) * kp * sizeof(float), 256);
}

// dst(i, k) = (T) src(i, k) for k < K, 0 for K <= k < Kp; 64 rows x 64 k
// per workgroup, transposed through LDS.
template <typename T>
__global__ __launch_bounds__(256) void lowp_convert_kernel(const double* __restrict__ src, int lds, int r,
                                                           const int* __restrict__ nelim_p, int kcap,
                                                           T* __restrict__ dst, int kp) {
  __shared__ float t[64][65];
  const int K = min(max(*nelim_p, 0), kcap);
  const int i0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int kk = ty; kk < 64; kk += 4) {
    const int i = i0 + tx, k = k0 + kk;
    t[kk][tx] = (i < r && k < K) ? (float)src[(size_t)k * lds + i] : 0.0f;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int i = i0 + ii, k = k0 + tx;
    if (i < r && k < kp) dst[(size_t)i * kp + k] = (T)t[tx][ii];
  }
}

struct LowpArgs {
  int r;
  int kp;            // padded K of the operand rows
  const int* nelim_p;
  int kcap;
  const void* a;     // L21 rows
  const void* b;     // W rows
  float* c;          // trailing update: C -= L21 W^T (FP32)
  int ldc;
  double* s;         // Form: S = L21 W^T (FP64), rows row0..row0+nrows-1
  int lds, tiled, row0, nrows;
  int ntm, ntn;      // tiles down and across
  int per_xcd;
  int tn0;           // first tile column (trailing update over a range of tile columns)
};

// FORM = false: the dense trailing update; true: the supernode Form.
template <typename T, bool FORM>
__global__ __launch_bounds__(LP_THREADS, 2) void lowp_update_kernel(LowpArgs g) {
  constexpr int LP_BK = LowpTraits<T>::BK;
  constexpr int EPV = 16 / sizeof(T);            // elements per 16-byte vector
  constexpr int VPR = LP_BK / EPV;               // vectors per row per chunk
  constexpr int LDK = LP_BK + EPV;               // LDS row stride (elements), padded
  constexpr int NV = LP_BM * VPR / LP_THREADS;   // vectors per thread per operand
  __shared__ __attribute__((aligned(16))) T As[2][LP_BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][LP_BM * LDK];

  const int bid = blockIdx.x;
  const int tile = (bid % LP_NXCD) * g.per_xcd + bid / LP_NXCD;
  const int total = g.ntm * g.ntn;
  if (tile >= total) return;
  const int per_group = LP_GROUP * g.ntn;
  const int grp = tile / per_group;
  const int in_grp = tile % per_group;
  const int gm = min(LP_GROUP, g.ntm - grp * LP_GROUP);
  const int tm = grp * LP_GROUP + in_grp % gm;
  const int tn = in_grp / gm + g.tn0;
  const int i0 = g.row0 + tm * LP_BM, j0 = tn * LP_BM;
  if (j0 > i0 + LP_BM - 1) return;   // strictly above the diagonal
  const int iend = FORM ? g.row0 + g.nrows : g.r;   // rows of this call

  const int K = min(max(*g.nelim_p, 0), g.kcap);
  const int nk = (K + LP_BK - 1) / LP_BK;
  const T* A = static_cast<const T*>(g.a);
  const T* B = static_cast<const T*>(g.b);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // staging: vector v of this thread covers row (q / VPR), k vector (q % VPR)
  u4 ra[NV], rb[NV];
  auto load = [&](int kc) {
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const int q = tid + h * LP_THREADS;
      const int row = q / VPR, kv = q % VPR;
      const int ia = min(i0 + row, iend - 1), ib = min(j0 + row, g.r - 1);
      const size_t ko = (size_t)kc * LP_BK + kv * EPV;
      ra[h] = *reinterpret_cast<const u4*>(A + (size_t)ia * g.kp + ko);
      rb[h] = *reinterpret_cast<const u4*>(B + (size_t)ib * g.kp + ko);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const int q = tid + h * LP_THREADS;
      const int row = q / VPR, kv = q % VPR;
      *reinterpret_cast<u4*>(&As[buf][row * LDK + kv * EPV]) = ra[h];
      *reinterpret_cast<u4*>(&Bs[buf][row * LDK + kv * EPV]) = rb[h];
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};

  const int lrow = lane & 15, lk = lane >> 4;
  if (nk > 0) {
    load(0);
    store(0);
    __syncthreads();
  }
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load(kc + 1);
    if constexpr (LowpTraits<T>::PREC == 1) {
#pragma unroll
      for (int ks = 0; ks < LP_BK; ks += 4) {
        float af[4], bf[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) af[x] = As[buf][(wm * 64 + x * 16 + lrow) * LDK + ks + lk];
#pragma unroll
        for (int y = 0; y < 4; ++y) bf[y] = Bs[buf][(wn * 64 + y * 16 + lrow) * LDK + ks + lk];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[y], af[x], acc[x][y], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < LP_BK; ks += 32) {
        bf8 af[4], bf[4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
          af[x] = *reinterpret_cast<const bf8*>(&As[buf][(wm * 64 + x * 16 + lrow) * LDK + ks + 8 * lk]);
#pragma unroll
        for (int y = 0; y < 4; ++y)
          bf[y] = *reinterpret_cast<const bf8*>(&Bs[buf][(wn * 64 + y * 16 + lrow) * LDK + ks + 8 * lk]);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[y], af[x], acc[x][y], 0, 0, 0);
      }
    }
    if (kc + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wm * 64 + x * 16 + lrow;
        const int j = j0 + wn * 64 + y * 16 + 4 * lk + q;
        if (i < iend && j <= i) {
          if (!FORM) {
            g.c[(size_t)j * g.ldc + i] -= acc[x][y][q];
          } else if (g.tiled) {
            const size_t ti = (size_t)(i / LP_BM) * (i / LP_BM + 1) / 2 + j / LP_BM;
            g.s[ti * LP_BM * LP_BM + (size_t)(j % LP_BM) * LP_BM + i % LP_BM] = (double)acc[x][y][q];
          } else {
            g.s[(size_t)j * g.lds + (i - g.row0)] = (double)acc[x][y][q];
          }
        }
      }
}

// Operand rows (k contiguous, K padded to LP_KPAD) of L21 and W in ops, in
// FP32 (prec 1) or BF16 (prec 2).
int launch_lowp_convert(int r, int K, const double* l21, int lda, const double* w, int ldw, const int* nelim,
                        int prec, void* ops, hipStream_t stream) {
  if (r <= 0 || K <= 0) return 0;
  const int kp = (int)align_up((size_t)K, LP_KPAD);
  const size_t half = align_up((size_t)r * kp * sizeof(float), 256);
  void* opa = ops;
  void* opb = static_cast<unsigned char*>(ops) + half;
  const dim3 cg((r + 63) / 64, kp / 64);
  if (prec == 1) {
    lowp_convert_kernel<float><<<cg, 256, 0, stream>>>(l21, lda, r, nelim, K, static_cast<float*>(opa), kp);
    lowp_convert_kernel<float><<<cg, 256, 0, stream>>>(w, ldw, r, nelim, K, static_cast<float*>(opb), kp);
  } else {
    lowp_convert_kernel<__bf16><<<cg, 256, 0, stream>>>(l21, lda, r, nelim, K, static_cast<__bf16*>(opa), kp);
    lowp_convert_kernel<__bf16><<<cg, 256, 0, stream>>>(w, ldw, r, nelim, K, static_cast<__bf16*>(opb), kp);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

static LowpArgs lowp_args(int r, int K, const int* nelim, void* ops) {
  const int kp = (int)align_up((size_t)K, LP_KPAD);
  const size_t half = align_up((size_t)r * kp * sizeof(float), 256);
  LowpArgs g{};
  g.r = r;
  g.kp = kp;
  g.nelim_p = nelim;
  g.kcap = K;
  g.a = ops;
  g.b = static_cast<unsigned char*>(ops) + half;
  return g;
}

// The trailing update from operand rows already converted (by
// launch_lowp_convert with the same r and K), on the 128-wide tile columns
// [tc0, tc1) of C (rows from the first of them down); tc1 < 0: to the last.
int launch_lowp_update_ops(int r, int K, const int* nelim, float* c, int ldc, int prec, void* ops, int tc0,
                           int tc1, hipStream_t stream) {
  if (r <= 0 || K <= 0) return 0;
  const int nt = (r + LP_BM - 1) / LP_BM;
  if (tc1 < 0 || tc1 > nt) tc1 = nt;
  if (tc0 < 0) tc0 = 0;
  if (tc0 >= tc1) return 0;
  LowpArgs g = lowp_args(r, K, nelim, ops);
  g.c = c;
  g.ldc = ldc;
  g.row0 = tc0 * LP_BM;   // rows above the first tile column's diagonal are not touched
  g.tn0 = tc0;
  g.ntm = (r - g.row0 + LP_BM - 1) / LP_BM;
  g.ntn = tc1 - tc0;
  const int total = g.ntm * g.ntn;
  g.per_xcd = (total + LP_NXCD - 1) / LP_NXCD;
  const unsigned grid = g.per_xcd * LP_NXCD;
  if (prec == 1) lowp_update_kernel<float, false><<<grid, LP_THREADS, 0, stream>>>(g);
  else lowp_update_kernel<__bf16, false><<<grid, LP_THREADS, 0, stream>>>(g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// Supernode Form in reduced precision from the converted operand rows: rows
// row0..row0+nrows-1 of S (tiled: row0 a multiple of 128).
int launch_lowp_form(int r, int K, const int* nelim, int row0, int nrows, double* s, int lds, int tiled, int prec,
                     void* ops, hipStream_t stream) {
  if (r <= 0 || K <= 0 || nrows <= 0) return 0;
  LowpArgs g = lowp_args(r, K, nelim, ops);
  g.s = s;
  g.lds = lds;
  g.tiled = tiled;
  g.row0 = row0;
  g.nrows = nrows;
  g.ntm = (nrows + LP_BM - 1) / LP_BM;
  g.ntn = (row0 + nrows + LP_BM - 1) / LP_BM;
  const int total = g.ntm * g.ntn;
  g.per_xcd = (total + LP_NXCD - 1) / LP_NXCD;
  const unsigned grid = g.per_xcd * LP_NXCD;
  if (prec == 1) lowp_update_kernel<float, true><<<grid, LP_THREADS, 0, stream>>>(g);
  else lowp_update_kernel<__bf16, true><<<grid, LP_THREADS, 0, stream>>>(g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
