// Compression of A21 into the p x p matrix C (Section 4, Fig. 4.1 (a)-(b)).
//
// Both constructions use comparisons only, so C is exact.
//
// Strict (Section 4.1, eq. (4.2)): two streaming passes over A21.
//   pass 1: one thread per row finds the column of its largest |a(i,k)|
//           (first maximum) -> set index J[i];
//   pass 2: workgroups own (row chunk, 8 columns); each folds |a(i,k)| into
//           an LDS table indexed by (J[i], k) with 64-bit atomic max on the
//           IEEE bit patterns (monotone for values >= 0), then merges the
//           table into C in global memory with atomic max.
//   The paper reduces partial C matrices on a tree across processors; on
//   one GPU the reduction tree is lanes -> LDS -> L2 atomics.
//
// Relaxed (Section 4.2): row j of C is the largest unflagged entry's row
//   of column j, taken in column order with flagging.  The row chosen for
//   column j is the best of column j once at most j rows are excluded, so
//   it is among column j's top j+1 rows.  Panels of at most EXACT_MAX_R
//   rows give every column exactly that list (below, with the kernels that
//   build and walk it).  Taller panels: pass 1 keeps, per (column, row
//   chunk), the top RELAXED_TOPK (|a|, row) pairs in the total order
//   "larger value first, lower row first"; pass 2 (one workgroup) merges
//   them per column, walks the columns in order taking the first unflagged
//   candidate, rescans a column in full when all its candidates are taken
//   (rare on random panels; common on Schur complements dominated by a
//   low-rank term, whose columns all rank the rows alike).  Either walk
//   ends with the chosen signed rows gathered into C.

#include "common.h"

namespace ctp {

constexpr int STRICT_CG = 8;          // columns per workgroup in pass 2
constexpr int STRICT_ROWS = 4096;     // rows per workgroup in pass 2


__global__ void fill_u64_kernel(unsigned long long* x, size_t count, unsigned long long v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) x[i] = v;
}

__global__ void fill_i32_kernel(int* x, int count, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = v;
}

CTP_DEV void strict_rowset_body(int r, int p, const double* __restrict__ a21, int lda, int* __restrict__ J,
                                int* __restrict__ status, int i) {
  if (i >= r) return;
  const double* row = a21 + i;
  double best = -1.0;
  int bj = 0;
  bool finite = true;
  int k = 0;
  for (; k + 4 <= p; k += 4) {
    double v0 = fabs(row[(size_t)(k + 0) * lda]);
    double v1 = fabs(row[(size_t)(k + 1) * lda]);
    double v2 = fabs(row[(size_t)(k + 2) * lda]);
    double v3 = fabs(row[(size_t)(k + 3) * lda]);
    finite = finite && isfinite(v0) && isfinite(v1) && isfinite(v2) && isfinite(v3);
    if (v0 > best) { best = v0; bj = k; }
    if (v1 > best) { best = v1; bj = k + 1; }
    if (v2 > best) { best = v2; bj = k + 2; }
    if (v3 > best) { best = v3; bj = k + 3; }
  }
  for (; k < p; ++k) {
    double v = fabs(row[(size_t)k * lda]);
    finite = finite && isfinite(v);
    if (v > best) { best = v; bj = k; }
  }
  J[i] = bj;
  if (!finite) atomicOr(status, ST_NONFINITE);
}

__global__ __launch_bounds__(256) void strict_rowset_kernel(int r, int p, const double* __restrict__ a21,
                                                          int lda, int* __restrict__ J,
                                                          int* __restrict__ status) {
  strict_rowset_body(r, p, a21, lda, J, status, blockIdx.x * blockDim.x + threadIdx.x);
}

// Dynamic LDS: p * STRICT_CG u64 bins.
HIP_DYNAMIC_SHARED(unsigned long long, cmp_bins)

CTP_DEV void strict_colmax_body(int r, int p, const double* __restrict__ a21, int lda,
                                const int* __restrict__ J, unsigned long long* __restrict__ cbits, int ldc,
                                int bx, int by) {
  unsigned long long* bins = cmp_bins;
  const int k0 = by * STRICT_CG;
  const int ncol = min(STRICT_CG, p - k0);
  const int i0 = bx * STRICT_ROWS;
  const int i1 = min(r, i0 + STRICT_ROWS);
  for (int q = threadIdx.x; q < p * STRICT_CG; q += blockDim.x) bins[q] = 0ull;
  __syncthreads();
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int j = J[i];
    unsigned long long* b = bins + (size_t)j * STRICT_CG;
#pragma unroll
    for (int c = 0; c < STRICT_CG; ++c) {
      if (c < ncol) {
        unsigned long long v = abs_bits(a21[(size_t)(k0 + c) * lda + i]);
        if (v) atomicMax(b + c, v);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < p * STRICT_CG; q += blockDim.x) {
    unsigned long long v = bins[q];
    int j = q / STRICT_CG, c = q % STRICT_CG;
    if (v && c < ncol) atomicMax(cbits + (size_t)(k0 + c) * ldc + j, v);
  }
}

__global__ __launch_bounds__(256) void strict_colmax_kernel(int r, int p, const double* __restrict__ a21,
                                                          int lda, const int* __restrict__ J,
                                                          unsigned long long* __restrict__ cbits, int ldc) {
  strict_colmax_body(r, p, a21, lda, J, cbits, ldc, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Relaxed compression
// ---------------------------------------------------------------------------

struct Cand {
  double v;   // |a(i, j)|, or -1 for "none"
  int i;      // row of A21
};

__host__ __device__ inline size_t relaxed_flag_bytes(int r) { return (size_t)((r > 0 ? r : 1) + 31) / 32 * sizeof(unsigned); }

CTP_DEV bool better(double v1, int i1, double v2, int i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// Grid (column, chunk).  Writes RELAXED_TOPK candidates per (column, chunk)
// to cand[(col * nchunks + chunk) * K + q], best first; missing -> v = -1.
CTP_DEV void relaxed_topk_body(int r, int p, const double* __restrict__ a21, int lda, int nchunks,
                               Cand* __restrict__ cand, int* __restrict__ status, int col, int chunk) {
  constexpr int K = RELAXED_TOPK;
  const int i0 = chunk * RELAXED_CHUNK;
  const int i1 = min(r, i0 + RELAXED_CHUNK);
  const double* colp = a21 + (size_t)col * lda;

  double tv[K];
  int ti[K];
#pragma unroll
  for (int q = 0; q < K; ++q) { tv[q] = -1.0; ti[q] = 0x7fffffff; }
  bool finite = true;
  // eight loads in flight per thread (unconditional: rows past the chunk
  // read its last row and are skipped), then the insertions in row order
  constexpr int RU = 8;
  const int nt = blockDim.x;
  for (int ib = i0 + threadIdx.x; ib < i1; ib += RU * nt) {
    double vb[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) vb[u] = colp[min(ib + u * nt, i1 - 1)];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int i = ib + u * nt;
      const double v = fabs(vb[u]);
      if (i < i1) finite = finite && isfinite(v);
      if (i < i1 && better(v, i, tv[K - 1], ti[K - 1])) {
        // insertion into the sorted list (static indices only)
        double cv = v;
        int ci = i;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if (better(cv, ci, tv[q], ti[q])) {
            double sv = tv[q];
            int si = ti[q];
            tv[q] = cv; ti[q] = ci;
            cv = sv; ci = si;
          }
        }
      }
    }
  }
  if (!finite) atomicOr(status, ST_NONFINITE);

  // Workgroup merge: K rounds of "best head among all threads".
  __shared__ double sv[4];
  __shared__ int si[4];
  __shared__ double wv;
  __shared__ int wi;
  int head = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < K; ++q) {
    double hv = -1.0;
    int hi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < K; ++s)
      if (s == head) { hv = tv[s]; hi = ti[s]; }
    double bv = hv;
    int bi = hi;
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(bv, off, 64);
      int oi = __shfl_xor(bi, off, 64);
      if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { sv[wave] = bv; si[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double xv = sv[0];
      int xi = si[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (better(sv[w], si[w], xv, xi)) { xv = sv[w]; xi = si[w]; }
      wv = xv; wi = xi;
      Cand* out = cand + ((size_t)col * nchunks + chunk) * K + q;
      out->v = xv;
      out->i = (xv < 0.0) ? -1 : xi;
    }
    __syncthreads();
    if (wv >= 0.0 && hi == wi && hv == wv) ++head;   // the winner pops its head
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void relaxed_topk_kernel(int r, int p, const double* __restrict__ a21,
                                                         int lda, int nchunks, Cand* __restrict__ cand,
                                                         int* __restrict__ status) {
  relaxed_topk_body(r, p, a21, lda, nchunks, cand, status, blockIdx.x, blockIdx.y);
}

// One workgroup of 1024 threads.  Dynamic LDS: final candidate lists
// (p * K Cand) + chosen rows (p ints) + a bitmap of chosen rows (r bits).
HIP_DYNAMIC_SHARED(unsigned char, cmp_smem)

CTP_DEV void relaxed_select_body(int r, int p, const double* __restrict__ a21, int lda, int nchunks,
                                 const Cand* __restrict__ cand, double* __restrict__ c, int ldc,
                                 int* __restrict__ crow_out, int* __restrict__ status, bool gather) {
  constexpr int K = RELAXED_TOPK;
  Cand* lists = reinterpret_cast<Cand*>(cmp_smem);
  int* chosen = reinterpret_cast<int*>(lists + (size_t)p * K);
  unsigned* flags = reinterpret_cast<unsigned*>(chosen + p);   // one bit per A21 row
  __shared__ int s_pick;
  __shared__ int s_need_scan;
  __shared__ int s_taken;
  __shared__ double red_v[16];
  __shared__ int red_i[16];

  // 1. Merge the chunk lists of each column into its global top K.
  for (int col = threadIdx.x; col < p; col += blockDim.x) {
    double tv[K];
    int ti[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { tv[q] = -1.0; ti[q] = 0x7fffffff; }
    // a chunk's K candidates are requested together, and the next chunk's
    // while this one is merged (the loads do not wait for the comparisons)
    const Cand* src = cand + (size_t)col * nchunks * K;
    Cand nxt[K];
#pragma unroll
    for (int q = 0; q < K; ++q) nxt[q] = src[q];
    for (int ch = 0; ch < nchunks; ++ch) {
      Cand cur[K];
#pragma unroll
      for (int q = 0; q < K; ++q) cur[q] = nxt[q];
      if (ch + 1 < nchunks) {
#pragma unroll
        for (int q = 0; q < K; ++q) nxt[q] = src[(size_t)(ch + 1) * K + q];
      }
      bool live = true;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const Cand e = cur[q];
        // lists are sorted: the first missing or losing entry ends the chunk
        live = live && e.v >= 0.0 && better(e.v, e.i, tv[K - 1], ti[K - 1]);
        if (!live) continue;
        double cv = e.v;
        int ci = e.i;
#pragma unroll
        for (int s = 0; s < K; ++s) {
          if (better(cv, ci, tv[s], ti[s])) {
            double sv = tv[s];
            int si = ti[s];
            tv[s] = cv; ti[s] = ci;
            cv = sv; ci = si;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
      lists[(size_t)col * K + q].v = tv[q];
      lists[(size_t)col * K + q].i = tv[q] < 0.0 ? -1 : ti[q];
    }
  }
  __syncthreads();

  // 2. Column order with flagging.  A bitmap of the rows already chosen
  //    sits in LDS; wave 0 walks the columns on its own (lane q tests
  //    candidate q, the first free one wins), and the whole workgroup joins
  //    only to rescan a column whose K candidates are all taken.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int nwords = (r + 31) / 32;
  for (int q = threadIdx.x; q < nwords; q += blockDim.x) flags[q] = 0u;
  if (threadIdx.x == 0) s_taken = 0;
  __syncthreads();
  int j = 0;
  while (j < p) {
    if (wave == 0) {
      int taken = s_taken;
      int jj = j;
      int need = 0;
      // the next column's candidates are read while this one's flags are
      // tested (they do not depend on the flags)
      int ahead = lane < K && jj < p ? lists[(size_t)jj * K + lane].i : -1;
      for (; jj < p; ++jj) {
        const int row = ahead;
        ahead = lane < K && jj + 1 < p ? lists[(size_t)(jj + 1) * K + lane].i : -1;
        if (taken >= r) {
          if (lane == 0) chosen[jj] = -1;
          continue;
        }
        const bool ok = (unsigned)row < (unsigned)r;   // not a missing candidate
        const unsigned fw = flags[ok ? row >> 5 : 0];
        const unsigned long long m = __ballot((int)((unsigned)ok & ~(fw >> (row & 31)) & 1u));
        if (m == 0ull) {
          need = 1;
          break;
        }
        const int pick = __builtin_amdgcn_readlane(row, __ffsll((long long)m) - 1);
        if (lane == 0) {
          chosen[jj] = pick;
          atomicOr(&flags[pick >> 5], 1u << (pick & 31));
        }
        wave_sync();   // the flag is set before any lane tests the next column
        ++taken;
      }
      if (lane == 0) {
        s_pick = jj;          // first column not finished
        s_need_scan = need;
        s_taken = taken;
      }
    }
    __syncthreads();
    j = s_pick;
    if (!s_need_scan) break;
    // Full rescan of column j over the rows not yet chosen.
    // eight loads in flight per thread, the chosen rows masked afterwards
    // (the comparisons are a total order, so the result does not depend on
    // the order in which rows are visited)
    const double* colp = a21 + (size_t)j * lda;
    double bv = -1.0;
    int bi = 0x7fffffff;
    constexpr int RU = 8;
    for (int i0 = threadIdx.x; i0 < r; i0 += RU * (int)blockDim.x) {
      double v[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        v[u] = i < r ? colp[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        if (i < r && !((flags[i >> 5] >> (i & 31)) & 1u) && better(fabs(v[u]), i, bv, bi)) {
          bv = fabs(v[u]);
          bi = i;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
    __syncthreads();
    // every thread merges the waves' results (the same pick everywhere);
    // thread 0 records it, and wave 0, which walks next, is ordered after
    // that by a wave sync (the other waves read the flags again only after
    // the walk's barrier)
    double xv = red_v[0];
    int xi = red_i[0];
    for (int w = 1; w < nwaves; ++w)
      if (better(red_v[w], red_i[w], xv, xi)) { xv = red_v[w]; xi = red_i[w]; }
    const int pick = (xv >= 0.0) ? xi : -1;
    if (threadIdx.x == 0) {
      chosen[j] = pick;
      if (pick >= 0) {
        flags[pick >> 5] |= 1u << (pick & 31);
        ++s_taken;
      }
      atomicOr(status, ST_RELAXED_RESCAN);
    }
    wave_sync();
    ++j;
  }
  __syncthreads();

  // 3. Gather the chosen signed rows into C (zero rows when none), here or
  //    (gather == false) by relaxed_gather_kernel from crow_out.
  if (gather) {
    for (int q = threadIdx.x; q < p * p; q += blockDim.x) {
      int j = q % p, k = q / p;    // consecutive threads walk down a column of C
      int row = chosen[j];
      c[(size_t)k * ldc + j] = row >= 0 ? a21[(size_t)k * lda + row] : 0.0;
    }
  }
  if (crow_out)
    for (int j = threadIdx.x; j < p; j += blockDim.x) crow_out[j] = chosen[j];
}

// C(j, k) = A21(chosen[j], k) (0 when no row was left): one workgroup per
// column k and 256 rows of C, so the scattered reads of the chosen rows are
// spread over the whole GPU instead of queued in one workgroup.
__global__ __launch_bounds__(256) void relaxed_gather_kernel(int p, const double* __restrict__ a21, int lda,
                                                           const int* __restrict__ chosen, double* __restrict__ c,
                                                           int ldc) {
  const int k = blockIdx.x;
  for (int j = blockIdx.y * 256 + threadIdx.x; j < p; j += gridDim.y * 256) {
    const int row = chosen[j];
    c[(size_t)k * ldc + j] = row >= 0 ? a21[(size_t)k * lda + row] : 0.0;
  }
}

__global__ __launch_bounds__(1024) void relaxed_select_kernel(int r, int p, const double* __restrict__ a21,
                                                            int lda, int nchunks,
                                                            const Cand* __restrict__ cand,
                                                            double* __restrict__ c, int ldc,
                                                            int* __restrict__ crow_out,
                                                            int* __restrict__ status) {
  relaxed_select_body(r, p, a21, lda, nchunks, cand, c, ldc, crow_out, status, false);
}

// ---------------------------------------------------------------------------
// Relaxed compression with exact candidate lists (r <= EXACT_MAX_R rows).
//
// The row chosen for column j is column j's best row once at most j rows
// are excluded, so it is always among column j's top j+1 rows.  For panels
// of up to EXACT_MAX_R rows each column gets exactly those: min(j+1, r) row
// indices, best first, at offset j(j+1)/2 of a list array (16-bit rows).
// The walk then never runs out of candidates and never rescans a column,
// which matters on Schur complements dominated by a low-rank term, where
// every column ranks the rows alike and the top-8 lists above are
// exhausted from the ninth column on.
//
// Build (one workgroup per column, up to 16 rows per thread in registers,
// 64 to 1024 threads by the panel's height): the order "larger |a| first, lower row first" is the order of
// the 77-bit key (bits 62..0 of |a| as an integer, EXACT_MAX_R-1-row).  A
// most-significant-digit radix select narrows the key range that holds the
// (j+1)-th key, digit by digit (8-bit digits of |a|, then 7-bit digits of
// the row), until the keys at or above the range's lower end number at most
// EXACT_CAP; those are collected in LDS, sorted by a bitonic network and
// the first j+1 written out.  The keys are distinct, so after the last digit
// the range holds one key and at most j+1 <= EXACT_CAP are collected.
// ---------------------------------------------------------------------------

constexpr int EXACT_MAX_R = 16384;                     // rows of A21 the exact lists are built for
constexpr int EXACT_THREADS = 1024;
constexpr int EXACT_PER_THREAD = EXACT_MAX_R / EXACT_THREADS;
constexpr int EXACT_CAP = 1024;                        // keys sorted at the end (>= 2 * CTP_MAX_P)
constexpr size_t EXACT_WALK_LDS = 128 * 1024;          // lists copied to LDS for the walk up to this size

static_assert(EXACT_CAP >= 2 * CTP_MAX_P, "a column's list must fit the final sort");
static_assert(EXACT_MAX_R <= 65536, "rows are stored in 16 bits");

__host__ __device__ inline size_t exact_list_entries(int p, int r) {
  const size_t m = (size_t)(p < r ? p : r);
  return m * (m + 1) / 2;
}
// walk kernel's dynamic LDS: row bitmap, chosen rows, then the lists
__host__ __device__ inline size_t exact_walk_lists_off(int p, int r) {
  return align_up(relaxed_flag_bytes(r) + (size_t)p * sizeof(int), 16);
}
__host__ __device__ inline size_t exact_walk_lds(int p, int r, bool lds_lists) {
  return exact_walk_lists_off(p, r) + (lds_lists ? align_up(exact_list_entries(p, r) * sizeof(unsigned short), 16) : 0);
}

// key a before key b in the selection order
CTP_DEV bool key_before(unsigned long long ka, int ia, unsigned long long kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(EXACT_THREADS) void relaxed_exact_kernel(int r, int p, const double* __restrict__ a21,
                                                                     int lda, unsigned short* __restrict__ lists,
                                                                     int* __restrict__ status) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long sk[EXACT_CAP];
  __shared__ int si[EXACT_CAP];
  __shared__ unsigned s_digit, s_add, s_bin;
  __shared__ int s_cnt;
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
  const double* colp = a21 + (size_t)j * lda;

  unsigned long long key[EXACT_PER_THREAD];
  bool finite = true;
#pragma unroll
  for (int u = 0; u < EXACT_PER_THREAD; ++u) {
    const int i = tid + u * nthr;
    const double v = i < r ? fabs(colp[i]) : 0.0;
    finite = finite && isfinite(v);
    key[u] = (unsigned long long)__double_as_longlong(v);
  }
  if (!finite) atomicOr(status, ST_NONFINITE);
  if (j >= r) return;               // every row is taken before column j (uniform over the workgroup)
  const unsigned K = (unsigned)min(j + 1, r);

  // Range of the (j+1)-th key: keys whose masked fields equal (hp, lp).
  unsigned long long hp = 0, hm = 0;
  unsigned lp = 0, lm = 0;
  unsigned need = K;                // keys still to take from the range
  unsigned above = 0;               // keys above the range
  for (int pass = 0; pass < 10; ++pass) {
    const bool hi_field = pass < 8;
    const int shift = pass < 7 ? 55 - 8 * pass : pass == 7 ? 0 : pass == 8 ? 7 : 0;
    const unsigned wmask = pass < 7 ? 0xffu : 0x7fu;
    for (int q = tid; q < 256; q += nthr) hist[q] = 0u;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EXACT_PER_THREAD; ++u) {
      const int i = tid + u * nthr;
      const unsigned lo = (unsigned)(EXACT_MAX_R - 1 - i);
      const bool m = i < r && (key[u] & hm) == hp && (lo & lm) == lp;
      const unsigned dg = hi_field ? (unsigned)(key[u] >> shift) & wmask : (lo >> shift) & wmask;
      // one atomic per wave when its matching keys share the digit (the
      // leading digits of similar values), one per key otherwise
      const unsigned long long bal = __ballot(m);
      if (bal) {
        const int first = __ffsll((long long)bal) - 1;
        const unsigned d0 = __shfl(dg, first, 64);
        const unsigned long long same = __ballot(m && dg == d0);
        if (same == bal) {
          if (lane == first) atomicAdd(&hist[d0], (unsigned)__popcll(bal));
        } else if (m) {
          atomicAdd(&hist[dg], 1u);
        }
      }
    }
    __syncthreads();
    if (tid < 64) {
      // lane l owns digits 255-4l .. 252-4l (descending); an inclusive scan
      // over the lanes finds the digit that holds the need-th key
      const unsigned h0 = hist[255 - 4 * lane], h1 = hist[254 - 4 * lane];
      const unsigned h2 = hist[253 - 4 * lane], h3 = hist[252 - 4 * lane];
      const unsigned s = h0 + h1 + h2 + h3;
      unsigned inc = s;
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned o = __shfl(inc, lane >= off ? lane - off : lane, 64);
        if (lane >= off) inc += o;
      }
      const unsigned exc = inc - s;
      if (exc < need && need <= inc) {
        // the first of the lane's four digits whose running count reaches need
        const unsigned c1 = exc + h0, c2 = c1 + h1, c3 = c2 + h2;
        const int t = need <= c1 ? 0 : need <= c2 ? 1 : need <= c3 ? 2 : 3;
        s_digit = (unsigned)(255 - 4 * lane - t);
        s_add = t == 0 ? exc : t == 1 ? c1 : t == 2 ? c2 : c3;
        s_bin = t == 0 ? h0 : t == 1 ? h1 : t == 2 ? h2 : h3;
      }
    }
    __syncthreads();
    const unsigned d = s_digit;
    need -= s_add;
    above += s_add;
    if (hi_field) {
      hp |= (unsigned long long)d << shift;
      hm |= (unsigned long long)wmask << shift;
    } else {
      lp |= d << shift;
      lm |= wmask << shift;
    }
    if (above + s_bin <= (unsigned)EXACT_CAP) break;   // uniform: every thread read the same values
  }

  // Collect the keys at or above the range's lower end (above + s_bin of them).
  if (tid == 0) s_cnt = 0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < EXACT_PER_THREAD; ++u) {
    const int i = tid + u * nthr;
    const unsigned lo = (unsigned)(EXACT_MAX_R - 1 - i);
    bool ge;
    if (lm == 0u) ge = (key[u] & hm) >= hp;
    else ge = key[u] > hp || (key[u] == hp && (lo & lm) >= lp);
    if (i < r && ge) {
      const int slot = atomicAdd(&s_cnt, 1);
      if (slot < EXACT_CAP) { sk[slot] = key[u]; si[slot] = i; }
    }
  }
  __syncthreads();
  const int cnt = min(s_cnt, EXACT_CAP);
  int n2 = 1;
  while (n2 < cnt) n2 <<= 1;
  for (int q = cnt + tid; q < n2; q += nthr) { sk[q] = 0ull; si[q] = 0x7fffffff; }   // sorts last
  __syncthreads();
  // bitonic sort of n2 keys into selection order
  for (int k = 2; k <= n2; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = tid; t < n2; t += nthr) {
        const int o = t ^ jj;
        if (o > t) {
          const unsigned long long kt = sk[t], ko = sk[o];
          const int it = si[t], io = si[o];
          const bool fwd = (t & k) == 0;
          if (fwd ? key_before(ko, io, kt, it) : key_before(kt, it, ko, io)) {
            sk[t] = ko; si[t] = io;
            sk[o] = kt; si[o] = it;
          }
        }
      }
      __syncthreads();
    }
  }
  unsigned short* out = lists + (size_t)j * (j + 1) / 2;
  for (int q = tid; q < (int)K; q += nthr) out[q] = (unsigned short)si[q];
}

// One workgroup; wave 0 walks the columns in order and takes the first row
// of column j's list not taken yet (there is one: the list holds j+1
// distinct rows and j rows are taken); lanes test 4 x 64 list entries per
// step, four columns at a time.  The choices stay in LDS until the walk
// ends.  Dynamic LDS: a bitmap
// of the rows taken, the chosen rows (p ints), then (LDS_LISTS) the lists,
// 16-byte aligned.
template <bool LDS_LISTS>
__global__ __launch_bounds__(1024) void relaxed_walk_kernel(int r, int p, const unsigned short* __restrict__ lists,
                                                          int* __restrict__ crow_out) {
  unsigned* flags = reinterpret_cast<unsigned*>(cmp_smem);
  const int nwords = (r + 31) / 32;
  int* chosen = reinterpret_cast<int*>(flags + nwords);
  unsigned short* lcopy = reinterpret_cast<unsigned short*>(cmp_smem + exact_walk_lists_off(p, r));
  const int m = min(p, r);
  for (int q = threadIdx.x; q < nwords; q += blockDim.x) flags[q] = 0u;
  if (LDS_LISTS) {
    // 16-byte words (the list array starts 256-byte aligned in the workspace)
    const size_t nw = (exact_list_entries(p, r) * sizeof(unsigned short) + 15) / 16;
    const uint4* src4 = reinterpret_cast<const uint4*>(lists);
    uint4* dst4 = reinterpret_cast<uint4*>(lcopy);
    for (size_t q = threadIdx.x; q < nw; q += blockDim.x) dst4[q] = src4[q];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const unsigned short* src = LDS_LISTS ? lcopy : lists;
    // entries c0 + lane + 64t (t < 4) of column j's list; positions past its
    // end read the last entry and are masked when tested
    auto load4 = [&](int j, int c0, int (&row)[4]) {
      const unsigned short* L = src + (size_t)j * (j + 1) / 2;
#pragma unroll
      for (int t = 0; t < 4; ++t) row[t] = (int)L[min(c0 + 64 * t + lane, j)];
    };
    // Columns go in groups of four: the first 256 entries of the four lists
    // and their flag words are read together, then the picks are taken in
    // column order in registers, each excluding the rows picked before it
    // in the group (so the flags seen by column j + t are those before the
    // group plus the group's earlier picks, as in the sequential walk).  A
    // column with no free row among its first 256 entries ends the group and
    // continues through the rest of its list once the group's picks are set.
    for (int j0 = m + lane; j0 < p; j0 += 64) chosen[j0] = -1;   // every row is taken
    int j = 0;
    while (j < m) {
      const int g = min(4, m - j);
      int rows[4][4];
      unsigned fw[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) load4(min(j + t, m - 1), 0, rows[t]);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) fw[t][u] = flags[(unsigned)rows[t][u] < (unsigned)r ? rows[t][u] >> 5 : 0];
      int picks[4] = {-1, -1, -1, -1};
      int done = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= g || done < t) break;       // uniform: the previous column was resolved here
        unsigned long long bal[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int rw = rows[t][u];
          unsigned ok = (unsigned)(64 * u + lane <= j + t) & (unsigned)((unsigned)rw < (unsigned)r);
          ok &= ~(fw[t][u] >> (rw & 31)) & 1u;
          ok &= (unsigned)(rw != picks[0]) & (unsigned)(rw != picks[1]) & (unsigned)(rw != picks[2]);
          bal[u] = __ballot((int)ok);
        }
        const int u = bal[0] ? 0 : bal[1] ? 1 : bal[2] ? 2 : bal[3] ? 3 : -1;   // uniform
        if (u >= 0) {
          const unsigned long long b = u == 0 ? bal[0] : u == 1 ? bal[1] : u == 2 ? bal[2] : bal[3];
          const int rsel = u == 0 ? rows[t][0] : u == 1 ? rows[t][1] : u == 2 ? rows[t][2] : rows[t][3];
          picks[t] = __builtin_amdgcn_readlane(rsel, __ffsll((long long)b) - 1);
          done = t + 1;
        }
      }
      if (lane < done) {
        const int pk = lane == 0 ? picks[0] : lane == 1 ? picks[1] : lane == 2 ? picks[2] : picks[3];
        chosen[j + lane] = pk;
        atomicOr(&flags[pk >> 5], 1u << (pk & 31));
      }
      wave_sync();   // the group's flags are set before any lane tests a later column
      j += done;
      if (done < g) {
        // column j: its first 256 entries are taken; the rest of its list
        int pick = -1;
        int row[4];
        for (int c0 = 256; c0 <= j && pick < 0; c0 += 256) {
          load4(j, c0, row);
          unsigned f1[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) f1[t] = flags[(unsigned)row[t] < (unsigned)r ? row[t] >> 5 : 0];
          unsigned long long bal[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const unsigned ok = (unsigned)(c0 + 64 * t + lane <= j) & (unsigned)((unsigned)row[t] < (unsigned)r);
            bal[t] = __ballot((int)(ok & ~(f1[t] >> (row[t] & 31)) & 1u));
          }
          const int t = bal[0] ? 0 : bal[1] ? 1 : bal[2] ? 2 : bal[3] ? 3 : -1;   // uniform
          if (t >= 0) {
            const unsigned long long b = t == 0 ? bal[0] : t == 1 ? bal[1] : t == 2 ? bal[2] : bal[3];
            const int rsel = t == 0 ? row[0] : t == 1 ? row[1] : t == 2 ? row[2] : row[3];
            pick = __builtin_amdgcn_readlane(rsel, __ffsll((long long)b) - 1);
          }
        }
        if (lane == 0) {
          chosen[j] = pick;                  // -1 is not reached: the list holds a free row
          if (pick >= 0) atomicOr(&flags[pick >> 5], 1u << (pick & 31));
        }
        wave_sync();
        ++j;
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < p; j += blockDim.x) crow_out[j] = chosen[j];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

int launch_compress(int n, int p, const double* a, int lda, int method, double* c, int ldc,
                    int* crow, int* status, void* work, hipStream_t stream) {
  const int r = n - p;
  const double* a21 = a + p;
  if (p <= 0) return method == CTP_STRICT || method == CTP_RELAXED ? 0 : -5;   // C is empty
  Workspace ws = workspace_layout(n, p, method);
  unsigned char* base = static_cast<unsigned char*>(work);
  if (method == CTP_STRICT) {
    int* J = reinterpret_cast<int*>(base + ws.j_off);
    size_t cnt = (size_t)ldc * p;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, stream,
        reinterpret_cast<unsigned long long*>(c), cnt, 0ull);
    if (r > 0) {
      hipLaunchKernelGGL(strict_rowset_kernel, dim3((r + 255) / 256), dim3(256), 0, stream, r, p, a21, lda, J, status);
      dim3 grid((r + STRICT_ROWS - 1) / STRICT_ROWS, (p + STRICT_CG - 1) / STRICT_CG);
      size_t lds = (size_t)p * STRICT_CG * sizeof(unsigned long long);
      if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)strict_colmax_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
      }
      hipLaunchKernelGGL(strict_colmax_kernel, dim3(grid), dim3(256), lds, stream, r, p, a21, lda, J,
                                                       reinterpret_cast<unsigned long long*>(c), ldc);
    }
  } else if (method == CTP_RELAXED && r > 0 && r <= EXACT_MAX_R) {
    // exact lists in the solve's gather buffer, which is free until the solve
    unsigned short* lists = reinterpret_cast<unsigned short*>(base + ws.w_off);
    int* rows = crow ? crow : reinterpret_cast<int*>(base + ws.crow_off);
    const int per = (r + EXACT_PER_THREAD - 1) / EXACT_PER_THREAD;
    const int nthr = std::min(EXACT_THREADS, std::max(64, (per + 63) / 64 * 64));
    hipLaunchKernelGGL(relaxed_exact_kernel, dim3(p), dim3(nthr), 0, stream, r, p, a21, lda, lists, status);
    const bool lds_lists = exact_list_entries(p, r) * sizeof(unsigned short) <= EXACT_WALK_LDS;
    const size_t lds = exact_walk_lds(p, r, lds_lists);
    const void* walk = lds_lists ? (const void*)relaxed_walk_kernel<true> : (const void*)relaxed_walk_kernel<false>;
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute(walk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    }
    if (lds_lists)
      hipLaunchKernelGGL(relaxed_walk_kernel<true>, dim3(1), dim3(1024), lds, stream, r, p, lists, rows);
    else
      hipLaunchKernelGGL(relaxed_walk_kernel<false>, dim3(1), dim3(1024), lds, stream, r, p, lists, rows);
    hipLaunchKernelGGL(relaxed_gather_kernel, dim3(p, (p + 255) / 256), dim3(256), 0, stream, p, a21, lda, rows, c, ldc);
  } else if (method == CTP_RELAXED) {
    Cand* cand = reinterpret_cast<Cand*>(base + ws.cand_off);
    int nch = ws.relaxed_chunks;
    if (r > 0) {
      dim3 grid(p, nch);
      hipLaunchKernelGGL(relaxed_topk_kernel, dim3(grid), dim3(256), 0, stream, r, p, a21, lda, nch, cand, status);
    }
    size_t lds = (size_t)p * RELAXED_TOPK * sizeof(Cand) + (size_t)p * sizeof(int) + relaxed_flag_bytes(r);
    if (r > 0 && lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)relaxed_select_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    }
    if (r > 0) {
      int* rows = crow ? crow : reinterpret_cast<int*>(base + ws.crow_off);
      hipLaunchKernelGGL(relaxed_select_kernel, dim3(1), dim3(1024), lds, stream, r, p, a21, lda, nch, cand, c, ldc, rows, status);
      hipLaunchKernelGGL(relaxed_gather_kernel, dim3(p, (p + 255) / 256), dim3(256), 0, stream, p, a21, lda, rows, c, ldc);
    } else {
      size_t cnt = (size_t)ldc * p;
      hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, stream,
          reinterpret_cast<unsigned long long*>(c), cnt, 0ull);
      if (crow) hipLaunchKernelGGL(fill_i32_kernel, dim3((p + 255) / 256), dim3(256), 0, stream, crow, p, -1);
    }
  } else {
    return -5;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

// ---------------------------------------------------------------------------
// Batched compression: one grid over all supernodes of a batch (the node is
// blockIdx.z, or blockIdx.x for the one-workgroup select), each node's A21
// compressed into the C of its own workspace as by the single-node launches.
// ---------------------------------------------------------------------------

__global__ void batch_zero_c_kernel(const BatchNode* __restrict__ nodes, int method) {
  const BatchNode& nd = nodes[blockIdx.y];
  const Workspace ws = workspace_layout(nd.n, nd.p, method);
  unsigned long long* c = reinterpret_cast<unsigned long long*>(nd.work + ws.c_off);
  const int cnt = nd.p * nd.p;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) c[q] = 0ull;
}

__global__ __launch_bounds__(256) void strict_rowset_batch_kernel(const BatchNode* __restrict__ nodes) {
  const BatchNode& nd = nodes[blockIdx.y];
  const int r = nd.n - nd.p;
  const Workspace ws = workspace_layout(nd.n, nd.p, CTP_STRICT);
  strict_rowset_body(r, nd.p, nd.a + nd.p, nd.lda, reinterpret_cast<int*>(nd.work + ws.j_off), nd.status,
                     blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void strict_colmax_batch_kernel(const BatchNode* __restrict__ nodes) {
  const BatchNode& nd = nodes[blockIdx.z];
  const int r = nd.n - nd.p;
  if ((int)blockIdx.x * STRICT_ROWS >= r || (int)blockIdx.y * STRICT_CG >= nd.p) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, CTP_STRICT);
  strict_colmax_body(r, nd.p, nd.a + nd.p, nd.lda, reinterpret_cast<const int*>(nd.work + ws.j_off),
                     reinterpret_cast<unsigned long long*>(nd.work + ws.c_off), nd.p, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void relaxed_topk_batch_kernel(const BatchNode* __restrict__ nodes) {
  const BatchNode& nd = nodes[blockIdx.z];
  const int r = nd.n - nd.p;
  if (r <= 0 || (int)blockIdx.x >= nd.p || (int)blockIdx.y >= nd.nchunks) return;
  const Workspace ws = workspace_layout(nd.n, nd.p, CTP_RELAXED);
  relaxed_topk_body(r, nd.p, nd.a + nd.p, nd.lda, nd.nchunks, reinterpret_cast<Cand*>(nd.work + ws.cand_off),
                    nd.status, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(1024) void relaxed_select_batch_kernel(const BatchNode* __restrict__ nodes) {
  const BatchNode& nd = nodes[blockIdx.x];
  const int r = nd.n - nd.p;
  const Workspace ws = workspace_layout(nd.n, nd.p, CTP_RELAXED);
  double* c = reinterpret_cast<double*>(nd.work + ws.c_off);
  int* crow = reinterpret_cast<int*>(nd.work + ws.crow_off);
  if (r > 0) {
    relaxed_select_body(r, nd.p, nd.a + nd.p, nd.lda, nd.nchunks, reinterpret_cast<const Cand*>(nd.work + ws.cand_off),
                        c, nd.p, crow, nd.status, true);
  } else {
    for (int q = threadIdx.x; q < nd.p * nd.p; q += blockDim.x) c[q] = 0.0;
    for (int j = threadIdx.x; j < nd.p; j += blockDim.x) crow[j] = -1;
  }
}

int launch_compress_batch(int count, const BatchNode* nodes, int method, int max_p, int max_r, int max_chunks,
                          hipStream_t stream) {
  if (count <= 0) return 0;
  if (method == CTP_STRICT) {
    hipLaunchKernelGGL(batch_zero_c_kernel, dim3(16, count), dim3(256), 0, stream, nodes, method);
    if (max_r > 0) {
      hipLaunchKernelGGL(strict_rowset_batch_kernel, dim3((max_r + 255) / 256, count), dim3(256), 0, stream, nodes);
      const size_t lds = (size_t)max_p * STRICT_CG * sizeof(unsigned long long);
      if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)strict_colmax_batch_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
      }
      hipLaunchKernelGGL(strict_colmax_batch_kernel, dim3((max_r + STRICT_ROWS - 1) / STRICT_ROWS, (max_p + STRICT_CG - 1) / STRICT_CG,
                                        count), dim3(256), lds, stream, nodes);
    }
  } else if (method == CTP_RELAXED) {
    if (max_r > 0) hipLaunchKernelGGL(relaxed_topk_batch_kernel, dim3(max_p, max_chunks, count), dim3(256), 0, stream, nodes);
    const size_t lds =
        (size_t)max_p * RELAXED_TOPK * sizeof(Cand) + (size_t)max_p * sizeof(int) + relaxed_flag_bytes(max_r);
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)relaxed_select_batch_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
    }
    hipLaunchKernelGGL(relaxed_select_batch_kernel, dim3(count), dim3(1024), lds, stream, nodes);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
