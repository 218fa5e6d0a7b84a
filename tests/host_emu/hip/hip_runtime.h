// Host emulation of the part of HIP that the one-workgroup kernels of the
// library use, so that their unchanged source can be compiled for the CPU
// with g++ and run under AddressSanitizer / UndefinedBehaviorSanitizer or
// ThreadSanitizer.  TEST INFRASTRUCTURE ONLY: nothing in the library
// includes this file; the tests put its directory first on the include path
// of a host build.
//
// Execution model:
//   * a launch runs its workgroups one after another (a valid schedule of
//     any kernel that does not wait for another workgroup); a workgroup's
//     threads are OS threads of a pool, one per work-item;
//   * __syncthreads() is a barrier of the workgroup's threads;
//   * cross-lane operations (__shfl*, __ballot, __any, DPP moves,
//     readfirstlane) are collectives of the 64 threads of a wave: each
//     publishes its value, the wave meets at a barrier, each reads its
//     source lane, the wave meets again.  All lanes of the wave must take
//     part (the kernels call them in wave-uniform code); a barrier that is
//     not reached by every thread within a time limit ends the run with a
//     message naming it, instead of hanging;
//   * dynamic LDS (HIP_DYNAMIC_SHARED) is a heap block of exactly the
//     launch's size, filled with 0xff bytes (NaN doubles) for every
//     workgroup, so AddressSanitizer sees any access past the size the host
//     asked for and a read before a write shows up as a NaN;
//   * static __shared__ variables are process globals (their values carry
//     over between workgroups, where the hardware would leave them
//     undefined);
//   * device memory is host memory; streams execute at once.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

using std::isfinite;
using std::isinf;
using std::isnan;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

// ---------------------------------------------------------------- runtime API
typedef enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorUnknown = 999 } hipError_t;
typedef struct ihipStream_t* hipStream_t;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 } hipFuncAttribute;

struct alignas(16) uint4 {
  unsigned x, y, z, w;
};

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};

inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipPeekAtLastError() { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int value) {
  return value <= 160 * 1024 ? hipSuccess : hipErrorInvalidValue;   // LDS of one CDNA4 workgroup
}
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (bytes) memmove(dst, src, bytes);
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k) {
  return hipMemcpyAsync(dst, src, bytes, k, nullptr);
}
inline hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) {
  if (bytes) memset(dst, v, bytes);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }

namespace emu {

constexpr int WAVE = 64;

[[noreturn]] inline void fail(const char* what) {
  fprintf(stderr, "host emulation: %s\n", what);
  fflush(stderr);
  abort();
}

[[noreturn]] void stuck(const char* what, int arrived, int expected);

// A reusable barrier with a time limit (a thread that never arrives is a
// kernel bug: a barrier or a collective in divergent code).
class Barrier {
 public:
  void reset(int n) {
    std::lock_guard<std::mutex> g(m_);
    n_ = n;
    count_ = 0;
  }
  void wait(const char* what) {
    std::unique_lock<std::mutex> l(m_);
    const unsigned long long gen = gen_;
    if (++count_ == n_) {
      count_ = 0;
      ++gen_;
      cv_.notify_all();
      return;
    }
    static const int limit = getenv("EMU_BARRIER_SECONDS") ? atoi(getenv("EMU_BARRIER_SECONDS")) : 120;
    // system_clock: its timed wait is one that ThreadSanitizer intercepts
    const auto until = std::chrono::system_clock::now() + std::chrono::seconds(limit);
    if (!cv_.wait_until(l, until, [&] { return gen_ != gen; })) {
      stuck(what, count_, n_);
    }
  }

 private:
  std::mutex m_;
  std::condition_variable cv_;
  int n_ = 0, count_ = 0;
  unsigned long long gen_ = 0;
};

struct WaveState {
  Barrier bar;
  uint64_t slot[WAVE];
  int active;
};

struct Launch {
  dim3 grid, block;
  int nthreads = 0;
  Barrier block_bar;
  std::vector<WaveState> waves;
  void* dyn = nullptr;
  const char* name = "";
  std::atomic<int> exited{0};
  int exit_barriers[1024];   // per thread: barriers passed when it left the kernel (-1: still running)
};

inline Launch& current() {
  static Launch L;
  return L;
}

struct ThreadIds {
  dim3 tid, bid;
  int lin = 0;
  int barriers = 0;   // __syncthreads passed in this workgroup
};
inline thread_local ThreadIds ids;

[[noreturn]] inline void stuck(const char* what, int arrived, int expected) {
  fprintf(stderr, "host emulation: %d of %d threads arrived, %d exited; kernel %s, block (%u, %u, %u)\n", arrived,
          expected, current().exited.load(), current().name, ids.bid.x, ids.bid.y, ids.bid.z);
  fprintf(stderr, "host emulation: waiting thread %d after %d barriers; exited threads (thread: barriers):", ids.lin,
          ids.barriers);
  for (int t = 0; t < current().nthreads; ++t)
    if (current().exit_barriers[t] >= 0) fprintf(stderr, " %d:%d", t, current().exit_barriers[t]);
  fprintf(stderr, "\n");
  fail(what);
}

// Persistent pool: worker t runs job(t) for t < count of each generation.
class Pool {
 public:
  static Pool& get() {
    static Pool p;
    return p;
  }
  void run(int count, const std::function<void(int)>& job) {
    while ((int)workers_.size() < count) {
      const int t = (int)workers_.size();
      workers_.emplace_back([this, t] { loop(t); });
    }
    {
      std::lock_guard<std::mutex> g(m_);
      job_ = &job;
      count_ = count;
      left_ = count;
      ++gen_;
    }
    cv_.notify_all();
    std::unique_lock<std::mutex> l(m_);
    done_cv_.wait(l, [&] { return left_ == 0; });
    job_ = nullptr;
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& w : workers_) w.join();
  }

 private:
  void loop(int t) {
    unsigned long long seen = 0;
    for (;;) {
      const std::function<void(int)>* job;
      {
        std::unique_lock<std::mutex> l(m_);
        cv_.wait(l, [&] { return gen_ != seen; });
        seen = gen_;
        if (stop_) return;
        if (t >= count_) continue;
        job = job_;
      }
      (*job)(t);
      std::lock_guard<std::mutex> g(m_);
      if (--left_ == 0) done_cv_.notify_all();
    }
  }
  std::vector<std::thread> workers_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* job_ = nullptr;
  int count_ = 0, left_ = 0;
  unsigned long long gen_ = 0;
  bool stop_ = false;
};

template <typename... P, typename... A>
void launch(const char* name, void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, A&&... args) {
  Launch& L = current();
  L.name = name;
  const int nt = (int)(block.x * block.y * block.z);
  if (nt <= 0 || nt > 1024) fail("workgroup size out of range");
  if (lds > 160 * 1024) fail("dynamic LDS beyond 160 KiB");
  L.grid = grid;
  L.block = block;
  L.nthreads = nt;
  L.block_bar.reset(nt);
  const int nw = (nt + WAVE - 1) / WAVE;
  L.waves = std::vector<WaveState>(nw);
  for (int w = 0; w < nw; ++w) {
    L.waves[w].active = std::min(WAVE, nt - w * WAVE);
    L.waves[w].bar.reset(L.waves[w].active);
  }
  const std::tuple<std::decay_t<P>...> params(std::forward<A>(args)...);
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        L.exited = 0;
        for (int t = 0; t < nt; ++t) L.exit_barriers[t] = -1;
        L.dyn = lds ? malloc(lds) : nullptr;
        if (lds) memset(L.dyn, 0xff, lds);
        const std::function<void(int)> job = [&](int t) {
          ids.lin = t;
          ids.tid = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
          ids.bid = dim3(bx, by, bz);
          ids.barriers = 0;
          std::apply(kernel, params);
          L.exit_barriers[t] = ids.barriers;
          L.exited.fetch_add(1);
        };
        Pool::get().run(nt, job);
        free(L.dyn);
        L.dyn = nullptr;
      }
}

inline int lane() { return ids.lin % WAVE; }

// Collective: every lane publishes `bits`, then reads lane src(lane) (or
// keeps `keep` when src < 0).
inline uint64_t exchange(uint64_t bits, int src, uint64_t keep) {
  WaveState& w = current().waves[ids.lin / WAVE];
  w.slot[lane()] = bits;
  w.bar.wait("cross-lane operation not reached by every lane of the wave");
  const uint64_t v = (src >= 0 && src < w.active) ? w.slot[src] : keep;
  w.bar.wait("cross-lane operation not reached by every lane of the wave");
  return v;
}

template <typename T>
inline uint64_t to_bits(T v) {
  static_assert(sizeof(T) <= 8, "cross-lane value wider than 64 bits");
  uint64_t b = 0;
  memcpy(&b, &v, sizeof(T));
  return b;
}

template <typename T>
inline T from_bits(uint64_t b) {
  T v;
  memcpy(&v, &b, sizeof(T));
  return v;
}

template <typename T>
inline T shuffle(T v, int src) {
  return from_bits<T>(exchange(to_bits(v), src, to_bits(v)));
}

// Source lane of a DPP move (the controls the kernels use, and their
// relatives), or -1 where the move has no source.
inline int dpp_src(int ctrl, int l) {
  const int row = l & ~15, r = l & 15;
  if (ctrl >= 0 && ctrl <= 0xff) return (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);   // quad_perm
  if (ctrl >= 0x101 && ctrl <= 0x10f) return r + (ctrl & 15) < 16 ? l + (ctrl & 15) : -1;   // row_shl
  if (ctrl >= 0x111 && ctrl <= 0x11f) return r - (ctrl & 15) >= 0 ? l - (ctrl & 15) : -1;   // row_shr
  if (ctrl >= 0x121 && ctrl <= 0x12f) return row | ((r - (ctrl & 15)) & 15);                 // row_ror
  if (ctrl == 0x140) return row | (15 - r);                                                 // row_mirror
  if (ctrl == 0x141) return (l & ~7) | (7 - (l & 7));                                       // row_half_mirror
  if (ctrl >= 0x150 && ctrl <= 0x15f) return row | (ctrl & 15);                             // row_share
  if (ctrl >= 0x160 && ctrl <= 0x16f) return row | (r ^ (ctrl & 15));                       // row_xmask
  fail("DPP control not emulated");
}

}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
  ::emu::launch(#kernel, kernel, dim3(grid), dim3(block), (size_t)(lds), __VA_ARGS__)

#define threadIdx (::emu::ids.tid)
#define blockIdx (::emu::ids.bid)
#define blockDim (::emu::current().block)
#define gridDim (::emu::current().grid)

// The array name becomes a reference to the launch's dynamic-LDS pointer
// (the build uses -fno-strict-aliasing for this view of a void*).
#define HIP_DYNAMIC_SHARED(type, var) \
  static type* const& var = reinterpret_cast<type* const&>(::emu::current().dyn);

inline void __syncthreads() {
  ::emu::current().block_bar.wait("__syncthreads not reached by every thread of the workgroup");
  ++::emu::ids.barriers;
}
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }

inline int __lane_id() { return ::emu::lane(); }

// HIP's device min / max for same-typed integer and floating operands.
template <typename T, typename = std::enable_if_t<std::is_arithmetic<T>::value>>
inline T min(T a, T b) {
  return b < a ? b : a;
}
template <typename T, typename = std::enable_if_t<std::is_arithmetic<T>::value>>
inline T max(T a, T b) {
  return a < b ? b : a;
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  const int l = ::emu::lane();
  int src = l ^ mask;
  if (src >= ((l + width) & ~(width - 1))) src = l;
  return ::emu::shuffle(v, src);
}

template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  const int l = ::emu::lane();
  return ::emu::shuffle(v, (l & ~(width - 1)) + (src & (width - 1)));
}

inline unsigned long long __ballot(int pred) {
  unsigned long long m = 0;
  const int l = ::emu::lane();
  auto& w = ::emu::current().waves[::emu::ids.lin / ::emu::WAVE];
  w.slot[l] = pred ? 1 : 0;
  w.bar.wait("__ballot not reached by every lane of the wave");
  for (int i = 0; i < w.active; ++i) m |= (unsigned long long)(w.slot[i] & 1) << i;
  w.bar.wait("__ballot not reached by every lane of the wave");
  return m;
}
inline int __any(int pred) { return __ballot(pred) != 0; }
inline int __all(int pred) {
  const auto& w = ::emu::current().waves[::emu::ids.lin / ::emu::WAVE];
  const unsigned long long full = w.active == 64 ? ~0ull : ((1ull << w.active) - 1);
  return __ballot(pred) == full;
}

// A wave barrier is a meeting of the wave's lanes (which also orders their
// memory operations); fences need nothing more here.
inline void emu_wave_barrier() {
  auto& w = ::emu::current().waves[::emu::ids.lin / ::emu::WAVE];
  w.bar.wait("wave barrier not reached by every lane of the wave");
}
#define __builtin_amdgcn_wave_barrier emu_wave_barrier
#define __builtin_amdgcn_fence(order, scope) ((void)0)

inline int emu_readfirstlane(int v) { return ::emu::shuffle(v, 0); }
#define __builtin_amdgcn_readfirstlane emu_readfirstlane
inline int emu_readlane(int v, int src) { return ::emu::shuffle(v, src); }
#define __builtin_amdgcn_readlane emu_readlane

inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  if (row_mask != 0xf || bank_mask != 0xf) ::emu::fail("DPP row/bank masks not emulated");
  const int s = ::emu::dpp_src(ctrl, ::emu::lane());
  const int moved = ::emu::shuffle(src, s < 0 ? 0 : s);
  return s < 0 ? (bound_ctrl ? 0 : old) : moved;
}
#define __builtin_amdgcn_update_dpp emu_update_dpp

inline long long __double_as_longlong(double x) {
  long long b;
  memcpy(&b, &x, 8);
  return b;
}
inline double __longlong_as_double(long long b) {
  double x;
  memcpy(&x, &b, 8);
  return x;
}
inline int __ffsll(unsigned long long x) { return x ? __builtin_ctzll(x) + 1 : 0; }
inline int __ffsll(long long x) { return __ffsll((unsigned long long)x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

template <typename T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}
template <typename T>
inline T atomicOr(T* p, T v) {
  return __atomic_fetch_or(p, v, __ATOMIC_RELAXED);
}
template <typename T>
inline T atomicAnd(T* p, T v) {
  return __atomic_fetch_and(p, v, __ATOMIC_RELAXED);
}
template <typename T>
inline T atomicMax(T* p, T v) {
  T old = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (old < v && !__atomic_compare_exchange_n(p, &old, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
  }
  return old;
}
template <typename T>
inline T atomicMin(T* p, T v) {
  T old = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (old > v && !__atomic_compare_exchange_n(p, &old, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
  }
  return old;
}
template <typename T>
inline T atomicExch(T* p, T v) {
  return __atomic_exchange_n(p, v, __ATOMIC_RELAXED);
}
template <typename T>
inline T atomicCAS(T* p, T cmp, T v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
  return cmp;
}
