// rank_emit.hip -- step 3 (dense grades: the 1-based index of an edge's
// distance in the duplicate-free list D, Section 2) over the sorted prefix
// that the reduction used, and step 5 (Section 4: "get the barcode
// interval"): each pivot row r gets the grade of the column stored for it;
// the canonical barcode lists the deaths ascending with the infinite bar last.
//
// The grade of sorted position p is 1 + the number of positions q in 1..p
// where the distance changes; only positions below E_eff are ever needed,
// because no pivot lies beyond the last one.
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kRankThreads = 256;
constexpr int kRankPer = 16;
constexpr int kRankBlock = kRankThreads * kRankPer;  // positions per block

__device__ uint32_t block_sum_256(uint32_t v, uint32_t* tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) tmp[wave] = v;
  __syncthreads();
  uint32_t s = tmp[0] + tmp[1] + tmp[2] + tmp[3];
  __syncthreads();
  return s;
}

__device__ uint32_t block_excl_256(uint32_t v, uint32_t* tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += tmp[w];
  __syncthreads();
  return base + x - v;
}

__device__ inline uint32_t change_flags(const uint64_t* __restrict__ k, int64_t p0, int64_t count,
                                        int shift, uint32_t* bits) {
  uint32_t m = 0, c = 0;
  uint64_t prev = p0 > 0 && p0 - 1 < count ? k[p0 - 1] >> shift : ~0ull;
#pragma unroll
  for (int q = 0; q < kRankPer; ++q) {
    const int64_t p = p0 + q;
    if (p < count) {
      const uint64_t v = k[p] >> shift;
      if (p > 0 && v != prev) {
        m |= 1u << q;
        ++c;
      }
      prev = v;
    }
  }
  *bits = m;
  return c;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_count(const uint64_t* __restrict__ k,
                                                             const RedCtl* ctl, int shift,
                                                             uint32_t* blockcnt) {
  __shared__ uint32_t tmp[4];
  const int64_t count = ctl->E_eff;
  const int64_t nb = (count + kRankBlock - 1) / kRankBlock;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint32_t bits;
    const uint32_t c = change_flags(k, b * kRankBlock + threadIdx.x * kRankPer, count, shift, &bits);
    const uint32_t s = block_sum_256(c, tmp);
    if (threadIdx.x == 0) blockcnt[b] = s;
  }
}

__global__ __launch_bounds__(kRankThreads) void k_rank_scan(const RedCtl* ctl, uint32_t* blockcnt) {
  __shared__ uint32_t tmp[4];
  const int64_t count = ctl->E_eff;
  const int64_t nb = (count + kRankBlock - 1) / kRankBlock;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kRankThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? blockcnt[b] : 0;
    const uint32_t ex = block_excl_256(v, tmp);
    const uint32_t tot = block_sum_256(v, tmp);
    if (b < nb) blockcnt[b] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kRankThreads) void k_rank_write(const uint64_t* __restrict__ k,
                                                             const RedCtl* ctl, int shift,
                                                             const uint32_t* blockcnt,
                                                             uint32_t* __restrict__ rank) {
  __shared__ uint32_t tmp[4];
  const int64_t count = ctl->E_eff;
  const int64_t nb = (count + kRankBlock - 1) / kRankBlock;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int64_t p0 = b * kRankBlock + threadIdx.x * kRankPer;
    uint32_t bits;
    const uint32_t c = change_flags(k, p0, count, shift, &bits);
    uint32_t run = 1 + blockcnt[b] + block_excl_256(c, tmp);
#pragma unroll
    for (int q = 0; q < kRankPer; ++q) {
      run += (bits >> q) & 1u;
      if (p0 + q < count) rank[p0 + q] = run;
    }
  }
}

__global__ void k_vertex_deaths(const int64_t* __restrict__ killer,
                                const uint32_t* __restrict__ rank, int64_t n,
                                uint32_t* __restrict__ dbv) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = killer[r];
    dbv[r] = p >= 0 ? rank[p] : kInf;
  }
}

// Bitonic sort of up to kSmallSortMax deaths in LDS; writes (0, death) bars.
__global__ __launch_bounds__(1024) void k_sort_bars_small(const uint32_t* __restrict__ dbv,
                                                          int64_t n,
                                                          uint32_t* __restrict__ bars) {
  __shared__ uint32_t s[kSmallSortMax];
  int P = 1;
  while (P < n) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) s[i] = i < n ? dbv[i] : kInf;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t x = s[lo], y = s[hi];
        if ((x > y) == up) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    bars[2 * i] = 0;
    bars[2 * i + 1] = s[i];
  }
}

__global__ void k_u32_to_keys(const uint32_t* __restrict__ v, int64_t n,
                              uint64_t* __restrict__ keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = v[i];
}

__global__ void k_keys_to_bars(const uint64_t* __restrict__ keys, int64_t n,
                               uint32_t* __restrict__ bars) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bars[2 * i] = 0;
    bars[2 * i + 1] = (uint32_t)keys[i];
  }
}

__global__ void k_pairs_detail(const int64_t* __restrict__ killer,
                               const uint64_t* __restrict__ skeys, int ib,
                               const uint64_t* __restrict__ table, int64_t LW, int64_t n,
                               int64_t* killer_pos, uint64_t* killer_edge,
                               int64_t* killer_sqdist, int32_t* partner) {
  const uint64_t imask = (1ull << ib) - 1ull;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = killer[r];
    int64_t pos = -1, sq = -1;
    uint64_t edge = ~0ull;
    int32_t other = -1;
    if (p >= 0) {
      const uint64_t key = skeys[p];
      pos = p;
      sq = (int64_t)(key >> (2 * ib));
      edge = (((key >> ib) & imask) << 32) | (key & imask);
      const uint64_t* row = table + r * LW;
      for (int64_t w = r >> 6; w >= 0 && other < 0; --w) {
        uint64_t x = row[w];
        if (w == (r >> 6)) x &= ~(1ull << (r & 63));
        if (x) other = (int32_t)(w * 64 + 63 - __clzll(x));
      }
    }
    if (killer_pos) killer_pos[r] = pos;
    if (killer_edge) killer_edge[r] = edge;
    if (killer_sqdist) killer_sqdist[r] = sq;
    if (partner) partner[r] = other;
  }
}

int grid_for(int64_t count, int per_block, int cap) {
  int64_t g = (count + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

int64_t rank_blocks(int64_t count) { return (count + kRankBlock - 1) / kRankBlock; }

hipError_t launch_rank(const uint64_t* skeys, const RedCtl* ctl, int shift, uint32_t* blockcnt,
                       int64_t max_count, uint32_t* rank_out, hipStream_t s) {
  const int g = grid_for(max_count, kRankBlock, 4096);
  hipLaunchKernelGGL(k_rank_count, dim3(g), dim3(kRankThreads), 0, s, skeys, ctl, shift,
                     blockcnt);
  hipLaunchKernelGGL(k_rank_scan, dim3(1), dim3(kRankThreads), 0, s, ctl, blockcnt);
  hipLaunchKernelGGL(k_rank_write, dim3(g), dim3(kRankThreads), 0, s, skeys, ctl, shift,
                     blockcnt, rank_out);
  return hipGetLastError();
}

hipError_t launch_vertex_deaths(const int64_t* killer, const uint32_t* rank, int64_t n,
                                uint32_t* dbv, hipStream_t s) {
  hipLaunchKernelGGL(k_vertex_deaths, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, killer, rank,
                     n, dbv);
  return hipGetLastError();
}

hipError_t launch_sort_bars_small(const uint32_t* dbv, int64_t n, uint32_t* out_bars,
                                  hipStream_t s) {
  if (n > kSmallSortMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sort_bars_small, dim3(1), dim3(1024), 0, s, dbv, n, out_bars);
  return hipGetLastError();
}

hipError_t launch_u32_to_keys(const uint32_t* v, int64_t n, uint64_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(k_u32_to_keys, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, v, n, keys);
  return hipGetLastError();
}

hipError_t launch_keys_to_bars(const uint64_t* keys, int64_t n, uint32_t* out_bars,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_keys_to_bars, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, keys, n,
                     out_bars);
  return hipGetLastError();
}

hipError_t launch_pairs_detail(const int64_t* killer, const uint64_t* skeys, int ib,
                               const uint64_t* table, int64_t LW, int64_t n,
                               int64_t* killer_pos, uint64_t* killer_edge,
                               int64_t* killer_sqdist, int32_t* partner, hipStream_t s) {
  hipLaunchKernelGGL(k_pairs_detail, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, killer,
                     skeys, ib, table, LW, n, killer_pos, killer_edge, killer_sqdist, partner);
  return hipGetLastError();
}

}  // namespace ph0
