// Roofline probes: micro-kernels that measure the peaks the library's
// kernels are compared against on the machine at hand, beside the
// datasheet figures.  Built into libctp_probe.so, apart from libctp.so.
//
//   ctp_probe_mfma: every wave of the grid issues `iters` rounds of NACC
//     independent matrix-core products on register operands (no memory
//     traffic in the loop): FP64 v_mfma_f64_16x16x4f64 (the Solve and Form
//     instruction, 2048 flop), FP32 v_mfma_f32_16x16x4f32 (2048 flop), BF16
//     v_mfma_f32_16x16x32_bf16 (16384 flop).  The accumulators are summed
//     into one word per wave at the end so that nothing is dead.
//   ctp_probe_copy: a grid-stride copy with 16-byte loads and stores (plain
//     or non-temporal), the HBM stream rate (bytes read + bytes written).
//
// The launchers only launch (on the given stream); the caller times them.

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int NACC = 8;   // independent accumulators per wave: enough to cover the MFMA latency

// The occupancy hint (256 threads, 2 workgroups per CU) keeps the
// accumulators in architectural registers; without it the compiler moves
// them through the accumulation registers on every iteration, which halves
// the rate.

__global__ __launch_bounds__(256, 2) void probe_mfma_f64_kernel(int iters, double* out) {
  const int lane = threadIdx.x & 63;
  double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  d4 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NACC; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (lane == 0) out[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = s;
}

__global__ __launch_bounds__(256, 2) void probe_mfma_f32_kernel(int iters, double* out) {
  const int lane = threadIdx.x & 63;
  float a = 1.0f + 1e-3f * lane, b = 1.0f - 1e-3f * lane;
  f4 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < NACC; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (lane == 0) out[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = s;
}

__global__ __launch_bounds__(256, 2) void probe_mfma_bf16_kernel(int iters, double* out) {
  const int lane = threadIdx.x & 63;
  bf8 a, b;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    a[v] = (__bf16)(1.0f + 1e-2f * ((lane + v) & 7));
    b[v] = (__bf16)(1.0f - 1e-2f * ((lane + 2 * v) & 7));
  }
  f4 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < NACC; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  if (lane == 0) out[blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)] = s;
}

// Eight 16-byte loads in flight per thread; NT: non-temporal loads and
// stores (streaming data that is not reused).
template <bool NT>
__global__ __launch_bounds__(256) void probe_copy_kernel(const u4* __restrict__ src, u4* __restrict__ dst, size_t n) {
  constexpr int U = 8;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    u4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else dst[i + u * stride] = v[u];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// Flop of one instruction of each kind, per wave.
long long ctp_probe_mfma_flop(int kind) {
  return kind == 0 ? 2048 : kind == 1 ? 2048 : kind == 2 ? 16384 : -1;
}

// kind 0 FP64, 1 FP32, 2 BF16.  grid x 256 threads (4 waves each), each
// wave `iters` x NACC instructions; out: one double per wave (device).
// Returns 0, -1 for a bad argument, or -(1000 + hipError).
int ctp_probe_mfma(int kind, int grid, int iters, double* out, hipStream_t stream) {
  if (kind < 0 || kind > 2 || grid < 1 || iters < 1 || !out) return -1;
  if (kind == 0) probe_mfma_f64_kernel<<<grid, 256, 0, stream>>>(iters, out);
  else if (kind == 1) probe_mfma_f32_kernel<<<grid, 256, 0, stream>>>(iters, out);
  else probe_mfma_bf16_kernel<<<grid, 256, 0, stream>>>(iters, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(1000 + (int)e);
}

int ctp_probe_nacc(void) { return NACC; }

// dst <- src, bytes a multiple of 16, 16-byte aligned device pointers;
// nontemporal != 0: non-temporal loads and stores.
int ctp_probe_copy(const void* src, void* dst, size_t bytes, int grid, int nontemporal, hipStream_t stream) {
  if (!src || !dst || bytes % 16 || grid < 1) return -1;
  if (reinterpret_cast<size_t>(src) % 16 || reinterpret_cast<size_t>(dst) % 16) return -1;
  if (nontemporal)
    probe_copy_kernel<true><<<grid, 256, 0, stream>>>(static_cast<const u4*>(src), static_cast<u4*>(dst), bytes / 16);
  else
    probe_copy_kernel<false><<<grid, 256, 0, stream>>>(static_cast<const u4*>(src), static_cast<u4*>(dst), bytes / 16);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(1000 + (int)e);
}

}  // extern "C"
