// Shared device/host helpers for the compressed-threshold-pivoting library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ctp.h"

#define CTP_DEV __device__ __forceinline__

// Column-major element (i, j) of an array with leading dimension ld.
#define CM(ptr, i, j, ld) ((ptr)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

namespace ctp {

// Pivot-type codes per final position (mirrored in ctp.h).
constexpr int PIV_ZERO = 0;
constexpr int PIV_1X1 = 1;
constexpr int PIV_2X2_FIRST = 2;
constexpr int PIV_2X2_SECOND = -2;
constexpr int PIV_DELAYED = -1;

// Device status bits (mirrored in ctp.h).
constexpr int ST_ZERO_PIVOT = CTP_STATUS_ZERO_PIVOT;
constexpr int ST_NONFINITE = CTP_STATUS_NONFINITE;
constexpr int ST_RELAXED_RESCAN = CTP_STATUS_RELAXED_RESCAN;
constexpr int ST_ROOT_FALLBACK = CTP_STATUS_ROOT_FALLBACK;

// Number of top candidates kept per column by the relaxed compression.
constexpr int RELAXED_TOPK = 8;

// For doubles known to be >= +0 (absolute values, not NaN) the IEEE bit
// pattern read as an unsigned integer orders exactly like the value.
CTP_DEV unsigned long long abs_bits(double x) {
  return (unsigned long long)__double_as_longlong(fabs(x));
}

CTP_DEV double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Orders one lane's LDS writes before the other lanes' later reads within
// a wave (release, wave barrier, acquire at wavefront scope).
CTP_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int RELAXED_CHUNK = 16384;  // rows per (column, chunk) block of the relaxed compression
constexpr int PIV_NSLOT = 8;          // pending eliminated columns per batch of the pivot search
constexpr int PIV_STATE_BYTES = 256;  // pivot-search state carried between launches
constexpr int TPP_MAX_GROUPS_WS = 4096; // grid-wide TPP: workgroups of a step (64 rows each)
constexpr int TPP_PART_WS = 6;          // grid-wide TPP: doubles of partial maxima per workgroup

// Workspace carve-up, shared by the size query and the launchers.
struct Workspace {
  size_t c_off = 0;       // p x p doubles: compressed matrix C (TPP: working A11)
  size_t j_off = 0;       // (n-p) ints: strict row -> set (TPP: p ints, variable -> position)
  size_t cand_off = 0;    // relaxed: per-chunk candidate keys (TPP: per-workgroup maxima)
  size_t crow_off = 0;    // relaxed: p ints, A21 row behind each C row
  size_t st_off = 0;      // pivot-search state carried between launches
  size_t wb_off = 0;      // pivot-search batch of pivot-column values
  size_t w_off = 0;       // compressed / restricted: (n-p) x p doubles, solve gather buffer
  int ldw = 1;
  size_t lc_off = 0;      // solve: L (masked, unit diagonal) after the pivot search (p x p, ld p)
  size_t misc_off = 0;    // 64 ints of counters / flags
  size_t total = 0;
  int relaxed_chunks = 0;
};

// One supernode of a batch as the kernels see it (built on the device from
// the caller's ctp_node array and the base pointers).
struct BatchNode {
  int n, p, lda, lds;
  int nchunks;            // relaxed compression chunks of its A21
  int ntiles;             // Form tiles of its S
  long long tile_off;     // first Form tile in the batch numbering
  double* a;              // panel
  double* s;              // S, or null
  int* perm;
  int* piv;
  double* d;
  int* nelim;
  int* status;
  unsigned char* work;    // this node's workspace (workspace_layout(n, p, method))
};

__host__ __device__ inline int relaxed_chunk_count(int rows) {
  return rows <= 0 ? 1 : (rows + RELAXED_CHUNK - 1) / RELAXED_CHUNK;
}
__host__ __device__ inline int pivot_state_bytes() { return PIV_STATE_BYTES; }
__host__ __device__ inline size_t pivot_wbuf_bytes(int p) {
  return align_up((size_t)PIV_NSLOT * (p > 0 ? p : 1) * sizeof(double), 256);
}

// Workspace carve-up of one supernode (host: size query and launchers;
// device: the batched kernels find each node's buffers).
__host__ __device__ inline Workspace workspace_layout(int n, int p, int method) {
  Workspace w;
  const int r = n > p ? n - p : 0;
  size_t off = 0;
  if (method == CTP_STRICT || method == CTP_RELAXED || method == CTP_TPP) {
    // compressed: C; TPP: the working copy of A11
    w.c_off = off;
    off = align_up(off + (size_t)p * p * sizeof(double), 256);
  }
  if (method == CTP_TPP) {
    // the grid-wide search: variable -> position, per-group column maxima
    w.j_off = off;
    off = align_up(off + (size_t)(p > 0 ? p : 1) * sizeof(int), 256);
    w.cand_off = off;   // then 64 ints of arrival counters
    off = align_up(off + (size_t)TPP_MAX_GROUPS_WS * TPP_PART_WS * sizeof(double) + 64 * sizeof(int), 256);
  }
  if (method == CTP_STRICT) {
    w.j_off = off;
    off = align_up(off + (size_t)r * sizeof(int), 256);
  }
  if (method == CTP_RELAXED) {
    w.relaxed_chunks = relaxed_chunk_count(r);
    w.cand_off = off;
    // Cand = {double, int} padded to 16 bytes
    off = align_up(off + (size_t)p * w.relaxed_chunks * RELAXED_TOPK * 16, 256);
    w.crow_off = off;
    off = align_up(off + (size_t)p * sizeof(int), 256);
  }
  w.st_off = off;
  off = align_up(off + (size_t)pivot_state_bytes(), 256);
  w.wb_off = off;
  off = align_up(off + pivot_wbuf_bytes(p), 256);
  if (r > 0) {
    w.ldw = (int)align_up((size_t)r, 32);
    w.w_off = off;
    off = align_up(off + (size_t)w.ldw * p * sizeof(double), 256);
    w.lc_off = off;
    off = align_up(off + (size_t)p * p * sizeof(double), 256);
  }
  w.misc_off = off;
  off = align_up(off + 64 * sizeof(int), 256);
  w.total = off;
  return w;
}


}  // namespace ctp
