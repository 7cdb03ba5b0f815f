// hip_runtime.h stand-in for the CPU emulation of the batched kernel
// (tests/test_batched_emulation.py).  A workgroup is blockDim.x host threads:
// __syncthreads is a barrier over them, a wavefront is 64 of them, and the
// wave collectives (ballot, shuffles) exchange values through a per-wave slot
// array between two wave barriers.  Atomics are the GCC builtins.  Only what
// the batched kernel uses is provided.  Not part of the library.
#pragma once
#include <assert.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <barrier>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __shared__
#define __launch_bounds__(x)

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorUnknown = 999 };
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

namespace emu {
struct Wave {
  std::barrier<> bar{64};
  uint64_t slot[64];
};
struct Block {
  explicit Block(unsigned threads) : bar(threads), waves(threads / 64) {}
  std::barrier<> bar;
  std::vector<Wave> waves;
  std::vector<char> smem;
};
struct Thread {
  unsigned tid, bid, bdim, gdim;
  Block* blk;
};
inline thread_local Thread t_self;
}  // namespace emu

#define threadIdx (emu_idx_tid())
#define blockIdx (emu_idx_bid())
#define blockDim (emu_idx_bdim())
#define gridDim (emu_idx_gdim())
inline dim3 emu_idx_tid() { return dim3(emu::t_self.tid); }
inline dim3 emu_idx_bid() { return dim3(emu::t_self.bid); }
inline dim3 emu_idx_bdim() { return dim3(emu::t_self.bdim); }
inline dim3 emu_idx_gdim() { return dim3(emu::t_self.gdim); }

inline void __syncthreads() { emu::t_self.blk->bar.arrive_and_wait(); }

inline emu::Wave& emu_wave() { return emu::t_self.blk->waves[emu::t_self.tid / 64]; }
inline unsigned emu_lane() { return emu::t_self.tid % 64; }

inline unsigned long long __ballot(int pred) {
  emu::Wave& w = emu_wave();
  w.slot[emu_lane()] = pred ? 1 : 0;
  w.bar.arrive_and_wait();
  unsigned long long m = 0;
  for (int l = 0; l < 64; ++l) m |= (unsigned long long)w.slot[l] << l;
  w.bar.arrive_and_wait();
  return m;
}

template <typename T>
inline T emu_exchange(T v, int src) {
  static_assert(sizeof(T) <= 8, "64-bit lanes");
  emu::Wave& w = emu_wave();
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  w.slot[emu_lane()] = bits;
  w.bar.arrive_and_wait();
  T out = v;
  if (src >= 0 && src < 64) memcpy(&out, &w.slot[src], sizeof(T));
  w.bar.arrive_and_wait();
  return out;
}
template <typename T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  assert(width == 64);
  const int lane = (int)emu_lane();
  return emu_exchange(v, lane >= (int)delta ? lane - (int)delta : lane);
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  assert(width == 64);
  return emu_exchange(v, src);
}

inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __popc(unsigned x) { return __builtin_popcount(x); }
inline int __clzll(long long x) { return x == 0 ? 64 : __builtin_clzll((unsigned long long)x); }

template <typename T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T atomicMin(T* p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}

inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }

// Runs all grid.x workgroups at once, each as block.x host threads (the
// batched kernel's workgroups share a work queue, so they run concurrently).
template <typename... KArgs, typename... Args>
inline void emu_launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shm, Args... args) {
  std::vector<std::unique_ptr<emu::Block>> blks;
  for (unsigned b = 0; b < grid.x; ++b) {
    blks.emplace_back(new emu::Block(block.x));
    blks.back()->smem.assign(shm, (char)0xA5);
  }
  std::vector<std::thread> th;
  for (unsigned b = 0; b < grid.x; ++b)
    for (unsigned t = 0; t < block.x; ++t)
      th.emplace_back([&, b, t]() {
        emu::t_self = emu::Thread{t, b, block.x, grid.x, blks[b].get()};
        kernel(args...);
      });
  for (auto& x : th) x.join();
}
#define hipLaunchKernelGGL(k, grid, block, shm, stream, ...) emu_launch(k, grid, block, shm, __VA_ARGS__)
// Dynamic LDS of the running workgroup.
inline char* emu_block_smem() { return emu::t_self.blk->smem.data(); }
