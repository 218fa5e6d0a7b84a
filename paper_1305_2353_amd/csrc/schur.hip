// Form task (Section 1): lower triangle of S = L21 D11 L21^T, a block of
// rows at a time, on the FP64 matrix cores of gfx950.
//
// S(i, j) = sum_k L21(i, k) W(j, k) with W = L21 D: the A operand is read
// straight from L21, the B operand is W, formed while the tile is staged
// (a 1x1 pivot scales one column of L21, a 2x2 pivot mixes two).
//
// Tiling: 128 x 128 output tile per workgroup of 4 waves (2 x 2), each wave
// a 64 x 64 block of 4 x 4 v_mfma_f64_16x16x4 accumulators; K streamed in
// chunks of 16 through double-buffered LDS with register prefetch.  The
// prefetch loads are issued unconditionally from clamped addresses and only
// consumed after the chunk's MFMAs, so their latency overlaps the matrix
// work (masking and the D scaling happen on the way into LDS).  Tiles
// are walked in groups of 8 row tiles (all column tiles of a group before
// the next group) and each XCD gets a contiguous range of that order, so
// the 64 tiles resident on one XCD share 8 row panels and 8 column panels
// in its L2.  Tiles strictly above the diagonal exit at once.

#include "common.h"

namespace ctp {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SC_BM = 128;
constexpr int SC_BN = 128;
constexpr int SC_THREADS = 256;
constexpr int SC_GROUP = 8;
constexpr int SC_NXCD = 8;

struct SchurArgs {
  int r;            // rows of A21 (order of S)
  int p;
  const double* l21;   // a + p
  int lda;
  const int* piv;
  const double* d;
  const int* nelim_p;
  int row0, nrows;
  double* s;
  int lds;
  int ntm, ntn;     // tile grid
  int per_xcd;      // tiles per XCD range
};

template <int BK, int RPT>
__global__ __launch_bounds__(SC_THREADS, 2) void schur_f64_kernel(SchurArgs g) {
  // RPT consecutive rows per thread; KPT k rows per thread and operand
  constexpr int TPK = SC_BM / RPT;        // threads per k row
  constexpr int KSTEP = SC_THREADS / TPK; // k rows covered by all threads at once
  constexpr int KPT = BK / KSTEP;
  __shared__ double As[2][BK][SC_BM];
  __shared__ double Bs[2][BK][SC_BN];
  __shared__ int piv_s[CTP_MAX_P + 1];
  __shared__ double d_s[2 * CTP_MAX_P + 2];

  // ---- tile index: XCD-contiguous ranges of a grouped order
  const int b = blockIdx.x;
  const int tile = (b % SC_NXCD) * g.per_xcd + b / SC_NXCD;
  const int total = g.ntm * g.ntn;
  if (tile >= total) return;
  const int per_group = SC_GROUP * g.ntn;
  const int grp = tile / per_group;
  const int in_grp = tile % per_group;
  const int gm = min(SC_GROUP, g.ntm - grp * SC_GROUP);
  const int tm = grp * SC_GROUP + in_grp % gm;
  const int tn = in_grp / gm;
  const int i0 = g.row0 + tm * SC_BM;       // first S row of the tile
  const int j0 = tn * SC_BN;                 // first S column
  const int iend = g.row0 + g.nrows;         // rows < iend
  if (j0 > min(i0 + SC_BM - 1, iend - 1)) return;   // strictly above the diagonal

  const int nelim = min(max(*g.nelim_p, 0), g.p);
  const int p = g.p;
  for (int k = threadIdx.x; k < p; k += SC_THREADS) {
    piv_s[k] = g.piv[k];
    d_s[2 * k] = g.d[2 * k];
    d_s[2 * k + 1] = g.d[2 * k + 1];
  }
  if (threadIdx.x == 0) { piv_s[p] = PIV_DELAYED; d_s[2 * p] = 0.0; d_s[2 * p + 1] = 0.0; }
  __syncthreads();

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // staging: consecutive threads take consecutive rows (one 1 KB column
  // segment per 128 threads); thread covers k rows kq, kq+2, ..., kq+BK-2
  const int ii = (tid % TPK) * RPT;
  const int kq = tid / TPK;

  // Prefetch registers: raw L21 values only.  Every load is issued
  // unconditionally from a clamped, in-bounds address so that none waits on
  // another; masks and the D scaling (W = L21 D) are applied when the
  // values are written to LDS, after the MFMAs of the current chunk.
  double ra[KPT][RPT], rb[KPT][RPT], rp[KPT][RPT];
  double c0[KPT], c1[KPT];
  bool kv[KPT];
  const int nk = (nelim + BK - 1) / BK;
  const int rmax = g.r - 1;

  auto load = [&](int kc) {
#pragma unroll
    for (int h = 0; h < KPT; ++h) {
      const int k = kc * BK + kq + KSTEP * h;
      const bool kval = k < nelim;
      const int pt = kval ? piv_s[k] : PIV_ZERO;
      const int kp = pt == PIV_2X2_FIRST ? k + 1 : (pt == PIV_2X2_SECOND ? k - 1 : k);
      const double dk = d_s[2 * (kval ? k : 0)];
      const double dk1 = d_s[2 * (kval ? k : 0) + 1];
      const double dm1 = d_s[2 * (kval ? kp : 0) + 1];
      c0[h] = (pt == PIV_ZERO) ? 0.0 : dk;
      c1[h] = pt == PIV_2X2_FIRST ? dk1 : (pt == PIV_2X2_SECOND ? dm1 : 0.0);
      kv[h] = kval;
      const double* colA = g.l21 + (size_t)(kval ? k : 0) * g.lda;
      const double* colP = g.l21 + (size_t)(kval ? kp : 0) * g.lda;
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int irow = min(i0 + ii + e, rmax), jrow = min(j0 + ii + e, rmax);
        ra[h][e] = colA[irow];
        rb[h][e] = colA[jrow];
        rp[h][e] = colP[jrow];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < KPT; ++h)
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const bool iv = kv[h] && (i0 + ii + e < iend);
        const bool jv = kv[h] && (j0 + ii + e < g.r);
        As[buf][kq + KSTEP * h][ii + e] = iv ? ra[h][e] : 0.0;
        Bs[buf][kq + KSTEP * h][ii + e] = jv ? fma(rp[h][e], c1[h], rb[h][e] * c0[h]) : 0.0;
      }
  };

  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  if (nk > 0) {
    load(0);
    store(0);
    __syncthreads();
  }
  const int lrow = lane & 15;
  const int lk = lane >> 4;
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load(kc + 1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = As[buf][ks + lk][wm * 64 + x * 16 + lrow];
#pragma unroll
      for (int y = 0; y < 4; ++y) bf[y] = Bs[buf][ks + lk][wn * 64 + y * 16 + lrow];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    if (kc + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: for v_mfma_f64_16x16x4, accumulator element q of lane l
  //      is row l/16 + 4q, column l%16 of the 16 x 16 block
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wm * 64 + x * 16 + lk + 4 * q;
        const int j = j0 + wn * 64 + y * 16 + lrow;
        if (i < iend && j <= i) g.s[(size_t)j * g.lds + (i - g.row0)] = acc[x][y][q];
      }
}

int launch_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
                 const int* nelim, int row0, int nrows, double* s, int lds, int tile,
                 hipStream_t stream) {
  SchurArgs g;
  g.r = n - p;
  g.p = p;
  g.l21 = a + p;
  g.lda = lda;
  g.piv = piv;
  g.d = d;
  g.nelim_p = nelim;
  g.row0 = row0;
  g.nrows = nrows;
  g.s = s;
  g.lds = lds;
  g.ntm = (nrows + SC_BM - 1) / SC_BM;
  g.ntn = (row0 + nrows + SC_BN - 1) / SC_BN;
  const int total = g.ntm * g.ntn;
  if (total == 0) return 0;
  g.per_xcd = (total + SC_NXCD - 1) / SC_NXCD;
  const unsigned grid = g.per_xcd * SC_NXCD;
  if (tile == 1) schur_f64_kernel<16, 2><<<grid, SC_THREADS, 0, stream>>>(g);
  else schur_f64_kernel<16, 4><<<grid, SC_THREADS, 0, stream>>>(g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
