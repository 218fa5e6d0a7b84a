// Scatter task (Section 1): extend-add of a factored front's contribution
// block into its parent front.
//
// After Factor + Solve (+ Form) of a front of order n with p panel columns
// and nelim eliminated, its contribution block is the trailing symmetric
// matrix over positions nelim..n-1:
//   * positions nelim..p-1 are the delayed pivots (Section 1: moved to a
//     later supernode): their rows and columns are the panel's lower
//     triangle after the eliminations (the delayed block in the A11 rows,
//     the updated delayed columns in the A21 rows);
//   * positions p..n-1 are the boundary: the Form's output, which the caller
//     produced as A22 - L21 D L21^T (the Form subtracting from the front's
//     own trailing entries).
// Position t stands for the child's original local index v(t) = perm[t]
// (t < p) or t (t >= p), and map[v] is its row in the parent front.  Every
// entry (ti >= tj >= nelim) is added into the parent's lower triangle at
// (max, min) of the two mapped rows: into the parent's panel when that
// column is below the parent's panel width pp, else into the parent's
// trailing block (its A22, the Form's input there).
//
// The contribution block is covered by 64 x 64 tiles of the lower triangle
// of the child's n x n index space (tiles entirely among eliminated
// positions do nothing); in a tile the 64 lanes of a wave take consecutive
// rows of one column, so the child's panel and S are read coalesced.  An
// injective map makes every parent entry receive at most one add per
// child, so no atomics are needed and the result is independent of the
// schedule.
//
// Batched form: one launch over the tiles of many children, each block
// finding its task by a binary search over the tasks' first tiles.  Tasks
// of one launch must write disjoint parent entries (distinct parents).

#include <cmath>

#include "common.h"

namespace ctp {

constexpr int EA_T = 64;   // tile side

struct ScatterArgs {
  int n, p, lda, lds, np, pp, ldf, ld22;
  const double* a;
  const double* s;
  const int* perm;
  const int* nelim;
  const int* map;
  double* f;
  double* f22;
};

__host__ __device__ inline long long ea_tiles(int n) {
  const long long nt = (n + EA_T - 1) / EA_T;
  return nt * (nt + 1) / 2;
}

// Tile t of the lower triangle, numbered row by row: (tm, tn), tn <= tm.
CTP_DEV void ea_tile(long long t, int& tm, int& tn) {
  int m = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((long long)m * (m + 1) / 2 > t) --m;
  while ((long long)(m + 1) * (m + 2) / 2 <= t) ++m;
  tm = m;
  tn = (int)(t - (long long)m * (m + 1) / 2);
}

CTP_DEV void ea_tile_body(const ScatterArgs& g, int tm, int tn, int* status) {
  const int nelim = min(max(*g.nelim, 0), g.p);
  const int i0 = tm * EA_T, j0 = tn * EA_T;
  if (i0 + EA_T <= nelim) return;                 // every row of the tile eliminated
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ti = i0 + lane;
  const bool row_ok = ti < g.n && ti >= nelim;
  const int vi = row_ok ? (ti < g.p ? g.perm[ti] : ti) : 0;
  const bool vi_ok = vi >= 0 && vi < g.n;
  const int pi = row_ok && vi_ok ? g.map[vi] : -1;
  bool bad = row_ok && !vi_ok;
  for (int k = wave; k < EA_T; k += 4) {
    const int tj = j0 + k;
    if (tj >= g.n) break;
    if (tj < nelim) continue;
    if (!row_ok || ti < tj) continue;
    const int vj = tj < g.p ? g.perm[tj] : tj;
    const int pj = vj >= 0 && vj < g.n ? g.map[vj] : -1;
    if (pi < 0 || pi >= g.np || pj < 0 || pj >= g.np) {
      bad = true;
      continue;
    }
    double v;
    if (tj < g.p) v = g.a[(size_t)tj * g.lda + ti];
    else v = g.s[(size_t)(tj - g.p) * g.lds + (ti - g.p)];
    const int R = max(pi, pj), C = min(pi, pj);
    if (C < g.pp) g.f[(size_t)C * g.ldf + R] += v;
    else g.f22[(size_t)(C - g.pp) * g.ld22 + (R - g.pp)] += v;
  }
  if (bad && status) atomicOr(status, CTP_STATUS_BAD_MAP);
}

__global__ __launch_bounds__(256) void extend_add_kernel(ScatterArgs g, int* status) {
  int tm, tn;
  ea_tile(blockIdx.x, tm, tn);
  ea_tile_body(g, tm, tn, status);
}

int launch_extend_add(int n, int p, const double* a, int lda, const double* s, int lds, const int* perm,
                      const int* nelim, const int* map, int np, int pp, double* f, int ldf, double* f22,
                      int ld22, int* status, hipStream_t stream) {
  if (n <= 0) return 0;
  const ScatterArgs g{n, p, lda, lds, np, pp, ldf, ld22, a, s, perm, nelim, map, f, f22};
  hipLaunchKernelGGL(extend_add_kernel, dim3((unsigned)ea_tiles(n)), dim3(256), 0, stream, g, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

long long scatter_tiles(int n) { return ea_tiles(n); }

__global__ __launch_bounds__(256) void extend_add_batch_kernel(const ctp_scatter_task* __restrict__ tasks, int count,
                                                               const double* panels, const double* s,
                                                               const int* perm, const int* nelim, const int* map,
                                                               double* fpanels, double* f22, int* status) {
  const long long b = blockIdx.x;
  int lo = 0, hi = count - 1;   // last task whose first tile is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_off <= b) lo = mid;
    else hi = mid - 1;
  }
  const ctp_scatter_task& t = tasks[lo];
  const long long local = b - t.tile_off;
  if (local >= ea_tiles(t.n)) return;
  const ScatterArgs g{t.n, t.p, t.lda, t.lds, t.np, t.pp, t.ldf, t.ld22,
                      panels + t.a_off, t.s_off >= 0 ? s + t.s_off : nullptr, perm + t.out_off,
                      nelim + t.node, map + t.map_off, fpanels + t.f_off,
                      t.f22_off >= 0 ? f22 + t.f22_off : nullptr};
  int tm, tn;
  ea_tile(local, tm, tn);
  ea_tile_body(g, tm, tn, status);
}

int launch_extend_add_batch(int count, const ctp_scatter_task* tasks, long long tiles, const double* panels,
                            const double* s, const int* perm, const int* nelim, const int* map, double* fpanels,
                            double* f22, int* status, hipStream_t stream) {
  if (count <= 0 || tiles <= 0) return 0;
  hipLaunchKernelGGL(extend_add_batch_kernel, dim3((unsigned)tiles), dim3(256), 0, stream, tasks, count, panels, s, perm, nelim, map, fpanels,
                                                               f22, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : CTP_ERR_HIP_BASE - (int)e;
}

}  // namespace ctp
