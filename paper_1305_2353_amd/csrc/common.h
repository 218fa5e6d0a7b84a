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

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carve-up, shared by the size query and the launchers.
struct Workspace {
  size_t c_off = 0;       // p x p doubles: compressed matrix C
  size_t j_off = 0;       // (n-p) ints: strict row -> set, relaxed scratch
  size_t cand_off = 0;    // relaxed: per-chunk candidate keys
  size_t crow_off = 0;    // relaxed: p ints, A21 row behind each C row
  size_t st_off = 0;      // pivot-search state carried between launches
  size_t wb_off = 0;      // pivot-search batch of pivot-column values
  size_t w_off = 0;       // compressed / restricted: (n-p) x p doubles, solve gather buffer
  int ldw = 1;
  size_t misc_off = 0;    // 64 ints of counters / flags
  size_t total = 0;
  int relaxed_chunks = 0;
};

int relaxed_chunk_count(int rows);
int pivot_state_bytes();
size_t pivot_wbuf_bytes(int p);
Workspace workspace_layout(int n, int p, int method);

}  // namespace ctp
