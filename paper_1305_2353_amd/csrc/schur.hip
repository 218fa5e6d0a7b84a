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

#include <algorithm>

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

// ---------------------------------------------------------------------------
// Form from an explicit W = L21 D (the Solve leaves it in its workspace):
// S = L21 W^T is then a plain product of two row panels, so staging is two
// streams of raw values with no pivot lookups, no D arithmetic and no
// per-element masks.  Same 128 x 128 tiling, wave layout and tile order as
// above.  A thread stages 4 consecutive rows of one k column per operand;
// with VEC the 4 values come in as two 16-byte loads (needs 16-byte aligned
// columns).  Rows past the end are never masked: their products land only
// in rows / columns of the tile that the epilogue discards, so it is enough
// that their addresses stay inside the arrays (a group that straddles the
// last row falls back to clamped scalar loads).  Columns k >= nelim of the
// last chunk are read from column nelim-1 and zeroed.
// ---------------------------------------------------------------------------

struct SchurWArgs {
  int r;
  const double* l21;   // a + p
  int lda;
  const double* w;     // W = L21 D, r x nelim, column-major
  int ldw;
  const int* nelim_p;
  int p;
  int row0, nrows;
  double* s;
  int lds;
  int ntm, ntn;
  int per_xcd;
  int tiled;           // 1: s is this tile's own 128 x 128 block (ld 128)
  int tn0 = 0;         // first tile column (a range of tile columns)
};

// Main loop and epilogue of one tile.  VEC: every row of both operands
// that this tile stages exists and each column is 16-byte aligned, so a
// thread's 4 rows come in as two 16-byte loads; otherwise 4 clamped loads.
// VAR selects the schedule.  Register-staged tiles: bit 0 writes the next
// chunk into LDS after three of the four k steps (so a chunk ends with the
// barrier alone), bit 1 pads the LDS rows by 8 doubles (bit 2: by 16), bit
// 4 splits a thread's staging rows into two pairs 64 rows apart so that the
// lanes' 16-byte LDS stores are contiguous (VAR 17 is the fastest of these;
// a second register stage spills).  Bit 3 subtracts the product from the
// output instead of storing it (the trailing update of a right-looking
// factorization).  Bit 5 sends full, 16-byte aligned tiles to the
// direct-to-LDS pipeline below (chunks of 8 k, four buffers; with bit 6
// chunks of 16 k, three buffers, one workgroup per CU), and bit 8 takes the
// product as S^T = W L21^T there, which turns the tile's stores into whole
// 128-byte lines.  The default is bits 0, 4, 5 and 8 (VAR 305): 63.0
// against 56.8 TFLOP/s for VAR 17 on the 4096-row blocks of an n = 100000,
// p = 512 panel.  Measured without gain and not kept: LDS reads of the next
// chunk issued ahead of the current products (two waves per SIMD already
// hide them), two buffers of 16 k, non-temporal or paired 16-byte stores
// (the tiles of a launch finish together and their stores meet the HBM
// write bandwidth as one burst).  Every variant gives the same bits:
// each output is the same sequence of matrix-core steps over k, and the
// operands of a product commute exactly.
template <int VAR>
struct SchurWShape {
  static constexpr int LW = (VAR & 4) ? SC_BM + 16 : (VAR & 2) ? SC_BM + 8 : SC_BM;   // LDS row stride (doubles)
  static constexpr int STAGED_BYTES = 2 * 2 * 16 * LW * 8;    // two buffers, two operands
  static constexpr int DL_BK = (VAR & 64) ? 16 : 8;           // k per chunk of the pipeline
  static constexpr int DL_NBUF = (VAR & 64) ? 3 : 4;          // chunks resident in LDS
  static constexpr int DL_BYTES = (VAR & 32) ? DL_NBUF * 2 * DL_BK * SC_BM * 8 : 0;
  static constexpr int LDS_BYTES = STAGED_BYTES > DL_BYTES ? STAGED_BYTES : DL_BYTES;
};

// Lower-triangle part of a finished 128 x 128 tile to S (or subtracted from
// it).  Accumulator q of block (x, y) in lane l is row 16x + l/16 + 4q,
// column 16y + l%16 of the wave's 64 x 64 quarter; with bit 8 (the product
// taken as S^T = W L21^T) it is row 16x + l%16, column 16y + l/16 + 4q, so
// that 16 lanes store 16 consecutive rows of a column (one 128-byte line).
template <int VAR>
__device__ __forceinline__ void schur_w_epilogue(const SchurWArgs& g, int i0, int j0, const d4 (&acc)[4][4]) {
  constexpr bool TR = (VAR & 256) != 0;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 15;
  const int lk = lane >> 4;
  const int iend = g.row0 + g.nrows;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wm * 64 + x * 16 + (TR ? lrow : lk + 4 * q);
        const int j = j0 + wn * 64 + y * 16 + (TR ? lk + 4 * q : lrow);
        if (i < iend && j <= i) {
          double* dst = g.tiled ? g.s + (size_t)(j - j0) * SC_BM + (i - i0)
                                : g.s + (size_t)j * g.lds + (i - g.row0);
          if (VAR & 8) *dst -= acc[x][y][q];   // trailing update: C -= L21 W^T
          else *dst = acc[x][y][q];
        }
      }
}

#define SC_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// s_waitcnt immediate that waits until at most n vector-memory operations of
// the wave are outstanding (vmcnt bits 3:0 and 15:14; expcnt and lgkmcnt at
// their maxima, so they do not wait)
constexpr int sc_vmcnt(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Direct-to-LDS pipeline for a full tile whose operand columns are 16-byte
// aligned.  A chunk is BK k-rows of each operand, one 1 KB row (128 doubles)
// per wave instruction: lane l's 16 bytes land at row start + 16 l, so the
// rows arrive in LDS without passing through registers.  NBUF chunks are
// resident: at chunk kc every wave waits for its own loads of chunk kc
// (vmcnt counts only the later chunks still in flight), the barrier makes
// everyone's loads visible and certifies that chunk kc-1 has been read, and
// chunk kc+NBUF-1 is then issued into kc-1's buffer.  k rows past K load
// row K-1 and are zeroed in both operands before the product, so the
// matrix-core arithmetic is that of the staged variants.
template <int VAR>
__device__ __forceinline__ void schur_w_tile_dl(const SchurWArgs& g, int i0, int j0, int K, double* lds) {
  constexpr int BK = SchurWShape<VAR>::DL_BK;
  constexpr int NBUF = SchurWShape<VAR>::DL_NBUF;
  constexpr int NW = SC_THREADS / 64;
  constexpr int ROWS = 2 * BK;              // rows of both operands per chunk
  constexpr int PER_WAVE = ROWS / NW;       // load instructions per wave and chunk
  static_assert(BK % NW == 0 && BK % 4 == 0, "chunk rows must split evenly over the waves");
  static_assert(PER_WAVE * (NBUF - 2) < 64, "vmcnt immediate");
  constexpr int CHUNK = ROWS * SC_BM;       // doubles per buffer
  const int nk = (K + BK - 1) / BK;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 15;
  const int lk = lane >> 4;
  const double* const l21 = g.l21 + i0 + 2 * lane;
  const double* const wp = g.w + j0 + 2 * lane;

  auto issue = [&](int kc) {
    double* buf = lds + (kc % NBUF) * CHUNK;
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) {
      const int cr = wave + NW * j;         // chunk row: operand cr / BK, k row cr % BK
      const int kk = min(kc * BK + cr % BK, K - 1);
      const double* src = cr < BK ? l21 + (size_t)kk * g.lda : wp + (size_t)kk * g.ldw;
      __builtin_amdgcn_global_load_lds(src, SC_LDS_PTR(buf + cr * SC_BM), 16, 0, 0);
    }
  };

  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  // no earlier stores or loads of this wave may be counted by the waits below
  __builtin_amdgcn_s_waitcnt(sc_vmcnt(0));
#pragma unroll
  for (int c = 0; c < NBUF - 1; ++c)
    if (c < nk) issue(c);

  for (int kc = 0; kc < nk; ++kc) {
    // chunks issued after kc and still in flight: min(nk - 1, kc + NBUF - 2) - kc
    const int later = min(nk - 1 - kc, NBUF - 2);
    if (later >= 2) __builtin_amdgcn_s_waitcnt(sc_vmcnt(2 * PER_WAVE));
    else if (later == 1) __builtin_amdgcn_s_waitcnt(sc_vmcnt(PER_WAVE));
    else __builtin_amdgcn_s_waitcnt(sc_vmcnt(0));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (kc + NBUF - 1 < nk) issue(kc + NBUF - 1);
    const double* const As = lds + (kc % NBUF) * CHUNK;
    const double* const Bs = As + BK * SC_BM;
    const bool full = (kc + 1) * BK <= K;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double af[4], bf[4];
      const double* pa = As + (ks + lk) * SC_BM + wm * 64 + lrow;
      const double* pb = Bs + (ks + lk) * SC_BM + wn * 64 + lrow;
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = pa[x * 16];
#pragma unroll
      for (int y = 0; y < 4; ++y) bf[y] = pb[y * 16];
      if (!full) {
        const bool kv = kc * BK + ks + lk < K;
#pragma unroll
        for (int x = 0; x < 4; ++x) af[x] = kv ? af[x] : 0.0;
#pragma unroll
        for (int y = 0; y < 4; ++y) bf[y] = kv ? bf[y] : 0.0;
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = (VAR & 256) ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[y], af[x], acc[x][y], 0, 0, 0)
                                  : __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    asm volatile("" ::: "memory");
  }
  // every wave has read the last chunk before the workgroup moves on (the
  // persistent Form reuses the buffers for its next tile)
  __builtin_amdgcn_s_barrier();
  schur_w_epilogue<VAR>(g, i0, j0, acc);
}

template <bool VEC, int VAR>
__device__ __forceinline__ void schur_w_tile(const SchurWArgs& g, int i0, int j0, int K, double* lds) {
  if constexpr (VEC && (VAR & 32) != 0) {
    schur_w_tile_dl<VAR>(g, i0, j0, K, lds);
    return;
  }
  constexpr int BK = 16;
  constexpr int RPT = 4;
  constexpr int TPK = SC_BM / RPT;          // 32 threads per k column
  constexpr int KSTEP = SC_THREADS / TPK;   // 8 k columns at once
  constexpr int KPT = BK / KSTEP;           // 2 k columns per thread
  constexpr int LW = SchurWShape<VAR>::LW;
  // As(buf, k, i) and Bs(buf, k, j)
  double* const As = lds;
  double* const Bs = lds + 2 * BK * LW;
  const int iend = g.row0 + g.nrows;
  const int nk = (K + BK - 1) / BK;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // staging rows of this thread: 4 consecutive rows, or (VAR & 16) the
  // row pairs 2l, 2l+1 and 64+2l, 64+2l+1, l = tid % 32, so that the lanes'
  // 16-byte LDS stores are contiguous
  constexpr bool SPLIT = (VAR & 16) != 0;
  const int ii = SPLIT ? (tid % TPK) * 2 : (tid % TPK) * RPT;
  const int ii2 = SPLIT ? ii + SC_BM / 2 : ii + 2;
  const int kq = tid / TPK;
  const int ga = i0 + ii, gb = j0 + ii;
  const int ga2 = i0 + ii2, gb2 = j0 + ii2;
  int rowa[RPT], rowb[RPT];
#pragma unroll
  for (int e = 0; e < RPT; ++e) {
    const int oa = e < 2 ? ga + e : ga2 + (e - 2);
    const int ob = e < 2 ? gb + e : gb2 + (e - 2);
    rowa[e] = VEC ? oa : min(oa, g.r - 1);
    rowb[e] = VEC ? ob : min(ob, g.r - 1);
  }

  struct Stage {
    double ra[KPT][RPT], rb[KPT][RPT];
    bool kv[KPT];
  };
  Stage st0;
  auto load = [&](Stage& S, int kc) {
    auto& ra = S.ra;
    auto& rb = S.rb;
#pragma unroll
    for (int h = 0; h < KPT; ++h) {
      const int k = kc * BK + kq + KSTEP * h;
      S.kv[h] = k < K;
      const int kk = min(k, K - 1);
      const double* ca = g.l21 + (size_t)kk * g.lda;
      const double* cb = g.w + (size_t)kk * g.ldw;
      if (VEC) {
        const double2 x0 = *reinterpret_cast<const double2*>(ca + ga);
        const double2 x1 = *reinterpret_cast<const double2*>(ca + ga2);
        const double2 y0 = *reinterpret_cast<const double2*>(cb + gb);
        const double2 y1 = *reinterpret_cast<const double2*>(cb + gb2);
        ra[h][0] = x0.x; ra[h][1] = x0.y; ra[h][2] = x1.x; ra[h][3] = x1.y;
        rb[h][0] = y0.x; rb[h][1] = y0.y; rb[h][2] = y1.x; rb[h][3] = y1.y;
      } else {
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
          ra[h][e] = ca[rowa[e]];
          rb[h][e] = cb[rowb[e]];
        }
      }
    }
  };
  // masks are needed only in the last chunk when nelim is not a multiple of
  // BK; the branch is uniform across the workgroup
  auto store = [&](Stage& S, int buf, int kc) {
    const auto& ra = S.ra;
    const auto& rb = S.rb;
    const bool full = (kc + 1) * BK <= K;
#pragma unroll
    for (int h = 0; h < KPT; ++h) {
      const bool m = full || S.kv[h];
      double2 a0, a1, b0, b1;
      a0.x = m ? ra[h][0] : 0.0; a0.y = m ? ra[h][1] : 0.0;
      a1.x = m ? ra[h][2] : 0.0; a1.y = m ? ra[h][3] : 0.0;
      b0.x = m ? rb[h][0] : 0.0; b0.y = m ? rb[h][1] : 0.0;
      b1.x = m ? rb[h][2] : 0.0; b1.y = m ? rb[h][3] : 0.0;
      double* pa = As + (buf * BK + kq + KSTEP * h) * LW;
      double* pb = Bs + (buf * BK + kq + KSTEP * h) * LW;
      *reinterpret_cast<double2*>(pa + ii) = a0;
      *reinterpret_cast<double2*>(pa + ii2) = a1;
      *reinterpret_cast<double2*>(pb + ii) = b0;
      *reinterpret_cast<double2*>(pb + ii2) = b1;
    }
  };

  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  const int lrow = lane & 15;
  const int lk = lane >> 4;
  auto kstep = [&](int buf, int ks) {
    double af[4], bf[4];
    const double* pa = As + (buf * BK + ks + lk) * LW + wm * 64 + lrow;
    const double* pb = Bs + (buf * BK + ks + lk) * LW + wn * 64 + lrow;
#pragma unroll
    for (int x = 0; x < 4; ++x) af[x] = pa[x * 16];
#pragma unroll
    for (int y = 0; y < 4; ++y) bf[y] = pb[y * 16];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
  };
  // one chunk from LDS buffer buf; the next chunk (already in registers S)
  // goes to the other buffer after three of the four k steps
  auto chunk = [&](int buf, Stage& S, int kc) {
    if (VAR & 1) {
      kstep(buf, 0);
      kstep(buf, 4);
      kstep(buf, 8);
      __builtin_amdgcn_sched_barrier(0);
      if (kc + 1 < nk) store(S, buf ^ 1, kc + 1);
      __builtin_amdgcn_sched_barrier(0);
      kstep(buf, 12);
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) kstep(buf, ks);
      if (kc + 1 < nk) store(S, buf ^ 1, kc + 1);
    }
    __syncthreads();
  };
  if (nk > 0) {
    load(st0, 0);
    store(st0, 0, 0);
    __syncthreads();
  }
  for (int kc = 0; kc < nk; ++kc) {
    if (kc + 1 < nk) load(st0, kc + 1);
    chunk(kc & 1, st0, kc);
  }
  schur_w_epilogue<VAR & ~256>(g, i0, j0, acc);
}

extern __shared__ double sc_dyn[];

template <bool ALIGNED, int VAR>
__global__ __launch_bounds__(SC_THREADS, 2) void schur_w_kernel(SchurWArgs g) {
  const int b = blockIdx.x;
  const int tile = (b % SC_NXCD) * g.per_xcd + b / SC_NXCD;
  if (tile >= g.ntm * g.ntn) return;
  const int per_group = SC_GROUP * g.ntn;
  const int grp = tile / per_group;
  const int in_grp = tile % per_group;
  const int gm = min(SC_GROUP, g.ntm - grp * SC_GROUP);
  const int tm = grp * SC_GROUP + in_grp % gm;
  const int tn = in_grp / gm + g.tn0;
  const int i0 = g.row0 + tm * SC_BM;
  const int j0 = tn * SC_BN;
  const int iend = g.row0 + g.nrows;
  if (j0 > min(i0 + SC_BM - 1, iend - 1)) return;   // strictly above the diagonal
  const int K = min(max(*g.nelim_p, 0), g.p);
  // j0 may exceed i0 when row0 is not a multiple of the tile: check both
  if (ALIGNED && i0 + SC_BM <= g.r && j0 + SC_BN <= g.r) schur_w_tile<true, VAR>(g, i0, j0, K, sc_dyn);
  else schur_w_tile<false, VAR>(g, i0, j0, K, sc_dyn);
}

template <int VAR>
static int launch_schur_w_var(const SchurWArgs& g, bool vec, unsigned grid, hipStream_t stream) {
  constexpr int bytes = SchurWShape<VAR>::LDS_BYTES;
  auto kern = vec ? schur_w_kernel<true, VAR> : schur_w_kernel<false, VAR>;
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  kern<<<grid, SC_THREADS, bytes, stream>>>(g);
  return 0;
}

int launch_schur_w(int n, int p, const double* a, int lda, const double* w, int ldw,
                   const int* nelim, int row0, int nrows, double* s, int lds, int variant,
                   hipStream_t stream) {
  SchurWArgs g;
  g.r = n - p;
  g.l21 = a + p;
  g.lda = lda;
  g.w = w;
  g.ldw = ldw;
  g.nelim_p = nelim;
  g.p = p;
  g.row0 = row0;
  g.nrows = nrows;
  g.s = s;
  g.lds = lds;
  g.tiled = 0;
  g.ntm = (nrows + SC_BM - 1) / SC_BM;
  g.ntn = (row0 + nrows + SC_BN - 1) / SC_BN;
  const int total = g.ntm * g.ntn;
  if (total == 0 || p == 0) return 0;
  g.per_xcd = (total + SC_NXCD - 1) / SC_NXCD;
  const unsigned grid = g.per_xcd * SC_NXCD;
  // 16-byte loads need every column of both operands 16-byte aligned
  const bool vec = ((reinterpret_cast<uintptr_t>(a + p + row0) | reinterpret_cast<uintptr_t>(w)) % 16 == 0) &&
                   lda % 2 == 0 && ldw % 2 == 0;
  int rc;
  switch (variant) {
    case 1: rc = launch_schur_w_var<0>(g, vec, grid, stream); break;
    case 2: rc = launch_schur_w_var<1>(g, vec, grid, stream); break;
    case 3: rc = launch_schur_w_var<3>(g, vec, grid, stream); break;
    case 4: rc = launch_schur_w_var<19>(g, vec, grid, stream); break;
    case 5: rc = launch_schur_w_var<17>(g, vec, grid, stream); break;
    case 6: rc = launch_schur_w_var<49>(g, vec, grid, stream); break;
    default: rc = launch_schur_w_var<305>(g, vec, grid, stream); break;
  }
  if (rc) return rc;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// ---------------------------------------------------------------------------
// Batched Form: one persistent launch over every tile of every node.  Each
// workgroup takes the next tile number from a counter in the workspace,
// finds its node by binary search over the nodes' first tile numbers, and
// runs the same tile routine as the single-node Form on that node's L21 and
// stored W.  Every workgroup leaves once the counter passes the last tile.
// Tiles of a node are numbered along the rows of its lower triangle of
// 128 x 128 tiles: t = tm (tm + 1) / 2 + tn, tn <= tm.
// ---------------------------------------------------------------------------

template <int VAR>
__global__ __launch_bounds__(SC_THREADS, 2) void schur_queue_kernel(const BatchNode* __restrict__ nodes, int count,
                                                                   int method, long long total, int tiled,
                                                                   unsigned int* __restrict__ counter) {
  __shared__ long long s_t;
  for (;;) {
    if (threadIdx.x == 0) s_t = (long long)atomicAdd(counter, 1u);
    __syncthreads();
    const long long t = s_t;
    __syncthreads();
    if (t >= total) break;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (nodes[mid].tile_off <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchNode& nd = nodes[lo];
    const long long local = t - nd.tile_off;
    int tm = (int)((sqrt(8.0 * (double)local + 1.0) - 1.0) * 0.5);
    while ((long long)(tm + 1) * (tm + 2) / 2 <= local) ++tm;
    while ((long long)tm * (tm + 1) / 2 > local) --tm;
    const int tn = (int)(local - (long long)tm * (tm + 1) / 2);
    const Workspace ws = workspace_layout(nd.n, nd.p, method);
    SchurWArgs g;
    g.r = nd.n - nd.p;
    g.l21 = nd.a + nd.p;
    g.lda = nd.lda;
    g.w = reinterpret_cast<const double*>(nd.work + ws.w_off);
    g.ldw = ws.ldw;
    g.nelim_p = nd.nelim;
    g.p = nd.p;
    g.row0 = 0;
    g.nrows = g.r;
    g.tiled = tiled;
    g.s = tiled ? nd.s + (size_t)local * SC_BM * SC_BN : nd.s;
    g.lds = tiled ? SC_BM : nd.lds;
    const int i0 = tm * SC_BM, j0 = tn * SC_BN;
    const int K = min(max(*nd.nelim, 0), nd.p);
    const bool aligned = ((reinterpret_cast<uintptr_t>(g.l21) | reinterpret_cast<uintptr_t>(g.w)) % 16 == 0) &&
                         g.lda % 2 == 0 && g.ldw % 2 == 0;
    if (aligned && i0 + SC_BM <= g.r && j0 + SC_BN <= g.r) schur_w_tile<true, VAR>(g, i0, j0, K, sc_dyn);
    else schur_w_tile<false, VAR>(g, i0, j0, K, sc_dyn);
    __syncthreads();   // LDS is reused by the next tile
  }
}

__global__ void queue_reset_kernel(unsigned int* counter) { *counter = 0u; }

template <int VAR>
static int launch_schur_queue_var(const BatchNode* nodes, int count, int method, long long total, int tiled,
                                  unsigned int* counter, unsigned grid, hipStream_t stream) {
  constexpr int bytes = SchurWShape<VAR>::LDS_BYTES;
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(schur_queue_kernel<VAR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  schur_queue_kernel<VAR><<<grid, SC_THREADS, bytes, stream>>>(nodes, count, method, total, tiled, counter);
  return 0;
}

int launch_schur_batch(int count, const BatchNode* nodes, int method, long long total, int tiled,
                       int subtract, unsigned int* counter, int variant, int workgroups, hipStream_t stream) {
  if (count <= 0 || total <= 0) return 0;
  queue_reset_kernel<<<1, 1, 0, stream>>>(counter);
  const unsigned grid = (unsigned)std::min<long long>(total, workgroups > 0 ? workgroups : 512);
  int rc;
  if (subtract) {
    switch (variant) {
      case 1: rc = launch_schur_queue_var<8>(nodes, count, method, total, 0, counter, grid, stream); break;
      case 2: rc = launch_schur_queue_var<9>(nodes, count, method, total, 0, counter, grid, stream); break;
      case 3: rc = launch_schur_queue_var<25>(nodes, count, method, total, 0, counter, grid, stream); break;
      default: rc = launch_schur_queue_var<313>(nodes, count, method, total, 0, counter, grid, stream); break;
    }
  } else {
    switch (variant) {
      case 1: rc = launch_schur_queue_var<0>(nodes, count, method, total, tiled, counter, grid, stream); break;
      case 2: rc = launch_schur_queue_var<1>(nodes, count, method, total, tiled, counter, grid, stream); break;
      case 3: rc = launch_schur_queue_var<17>(nodes, count, method, total, tiled, counter, grid, stream); break;
      default: rc = launch_schur_queue_var<305>(nodes, count, method, total, tiled, counter, grid, stream); break;
    }
  }
  if (rc) return rc;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// ---------------------------------------------------------------------------
// Whole lower triangle of one node's S in one persistent launch (the Form
// of the fused supernode call).  Tiles are numbered in groups of SC_GROUP
// tile rows; inside a group column by column (the tiles of one column of
// the group share the W block, the group's rows share their L21 blocks), so
// consecutive numbers reuse operands.  The numbers are cut into SC_NXCD
// contiguous ranges, one per XCD (workgroup b runs on XCD b mod SC_NXCD),
// and the workgroups of an XCD stride through its range together.  Output:
// column-major S (ld lds) or, with tiled, the packed 128 x 128 tiles of the
// lower triangle, tile tm (tm + 1) / 2 + tn at s + 16384 t (ld 128).
// ---------------------------------------------------------------------------

// tiles before group G, every earlier group being full: sum over the
// SC_GROUP G rows before it of (tm + 1) = 32 G^2 + 4 G for SC_GROUP = 8
CTP_DEV long long sc_group_start(long long G) { return 32 * G * G + 4 * G; }

CTP_DEV void sc_persist_tile(long long t, int ntm, int& tm, int& tn) {
  long long G = (long long)((sqrt(16.0 + 128.0 * (double)t) - 4.0) / 64.0);
  while (sc_group_start(G + 1) <= t) ++G;
  while (G > 0 && sc_group_start(G) > t) --G;
  long long l = t - sc_group_start(G);
  const int r0 = (int)(G * SC_GROUP);
  const int gm = min(SC_GROUP, ntm - r0);
  const long long full = (long long)gm * (r0 + 1);   // columns tn <= r0 hold gm tiles each
  if (l < full) {
    tn = (int)(l / gm);
    tm = r0 + (int)(l % gm);
    return;
  }
  l -= full;
  int c = 1;
  while (l >= gm - c) {
    l -= gm - c;
    ++c;
  }
  tn = r0 + c;
  tm = r0 + c + (int)l;
}

template <int VAR>
__global__ __launch_bounds__(SC_THREADS, 2) void schur_persist_kernel(SchurWArgs g, long long total, int per_x,
                                                                     int aligned) {
  const int x = blockIdx.x % SC_NXCD, w = blockIdx.x / SC_NXCD;
  const long long per = (total + SC_NXCD - 1) / SC_NXCD;
  const long long t0 = (long long)x * per;
  const long long t1 = min(total, t0 + per);
  const int K = min(max(*g.nelim_p, 0), g.p);
  double* const base = g.s;
  for (long long t = t0 + w; t < t1; t += per_x) {
    int tm, tn;
    sc_persist_tile(t, g.ntm, tm, tn);
    const int i0 = tm * SC_BM, j0 = tn * SC_BN;
    SchurWArgs h = g;
    if (g.tiled) h.s = base + ((long long)tm * (tm + 1) / 2 + tn) * (SC_BM * SC_BN);
    if (aligned && i0 + SC_BM <= g.r && j0 + SC_BN <= g.r) schur_w_tile<true, VAR>(h, i0, j0, K, sc_dyn);
    else schur_w_tile<false, VAR>(h, i0, j0, K, sc_dyn);
    __syncthreads();   // LDS is reused by the next tile
  }
}

// Whole lower triangle of S = L21 W^T: column-major (lds) or packed tiles.
int launch_schur_full(int n, int p, const double* a, int lda, const double* w, int ldw, const int* nelim,
                      double* s, int lds, int tiled, int workgroups, hipStream_t stream) {
  SchurWArgs g;
  g.r = n - p;
  g.l21 = a + p;
  g.lda = lda;
  g.w = w;
  g.ldw = ldw;
  g.nelim_p = nelim;
  g.p = p;
  g.row0 = 0;
  g.nrows = g.r;
  g.s = s;
  g.lds = tiled ? SC_BM : lds;
  g.tiled = tiled;
  g.ntm = (g.r + SC_BM - 1) / SC_BM;
  g.ntn = g.ntm;
  g.per_xcd = 0;
  const long long total = (long long)g.ntm * (g.ntm + 1) / 2;
  if (total == 0 || p == 0) return 0;
  const int aligned = ((reinterpret_cast<uintptr_t>(a + p) | reinterpret_cast<uintptr_t>(w)) % 16 == 0) &&
                      lda % 2 == 0 && ldw % 2 == 0;
  long long nwg = workgroups > 0 ? workgroups : 512;
  nwg = std::min<long long>(nwg, (total + SC_NXCD - 1) / SC_NXCD * SC_NXCD);
  nwg = (nwg + SC_NXCD - 1) / SC_NXCD * SC_NXCD;
  constexpr int VAR = 305;
  constexpr int bytes = SchurWShape<VAR>::LDS_BYTES;
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(schur_persist_kernel<VAR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  }
  schur_persist_kernel<VAR><<<(unsigned)nwg, SC_THREADS, bytes, stream>>>(g, total, (int)(nwg / SC_NXCD), aligned);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// C(i, j) -= sum_k L21(i, k) W(j, k) for the lower triangle i >= j of the
// order-(n-p) matrix C (column-major, ldc): the trailing update of a
// right-looking factorization, rows of L21 = rows p..n-1 of the panel.  Only
// the 128-wide tile columns [tc0, tc1) of C (rows from the first of them
// down); tc1 < 0: to the last.
int launch_schur_w_sub(int n, int p, const double* a, int lda, const double* w, int ldw,
                       const int* nelim, double* c, int ldc, int tc0, int tc1, hipStream_t stream) {
  const int r = n - p;
  const int nt = (r + SC_BM - 1) / SC_BM;
  if (tc1 < 0 || tc1 > nt) tc1 = nt;
  if (tc0 < 0) tc0 = 0;
  if (tc0 >= tc1 || p == 0) return 0;
  SchurWArgs g;
  g.r = r;
  g.l21 = a + p;
  g.lda = lda;
  g.w = w;
  g.ldw = ldw;
  g.nelim_p = nelim;
  g.p = p;
  g.row0 = tc0 * SC_BM;          // rows above the first tile column's diagonal are not touched
  g.nrows = r - g.row0;
  g.s = c + g.row0;              // the subtracting epilogue indexes rows from row0
  g.lds = ldc;
  g.tiled = 0;
  g.tn0 = tc0;
  g.ntm = (g.nrows + SC_BM - 1) / SC_BM;
  g.ntn = tc1 - tc0;
  const int total = g.ntm * g.ntn;
  g.per_xcd = (total + SC_NXCD - 1) / SC_NXCD;
  const unsigned grid = g.per_xcd * SC_NXCD;
  const bool vec = ((reinterpret_cast<uintptr_t>(a + p) | reinterpret_cast<uintptr_t>(w)) % 16 == 0) &&
                   lda % 2 == 0 && ldw % 2 == 0;
  int rc = launch_schur_w_var<313>(g, vec, grid, stream);
  if (rc) return rc;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
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
