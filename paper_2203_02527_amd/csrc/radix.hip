// radix.hip -- step 2 of the GPU pipeline (Section 4, step 2: sort the edges):
// stable least-significant-digit radix passes over 64-bit keys.
//
// Each pass is reduce-then-scan, with no workgroup ever waiting on another:
//   count   -- every 2048-key tile histograms its digits in LDS;
//   scan    -- one workgroup per digit scans that digit's tile counts
//              (exclusive, in place) and leaves the digit's total;
//   scatter -- every tile scans the 256 digit totals for the digits' first
//              output positions, ranks its keys among equal digits and
//              writes them.
// Inside a tile (4 waves x 8 rounds x 64 lanes) each wave owns a contiguous
// quarter; a key's rank among equal digits comes from wave ballots on the
// digit bits, so equal digits keep their order.  That stability is what turns
// sorting on the distance bits alone into the (delta, j, i) order.  The tile
// is reordered by digit in LDS before it is written, so each digit's run
// leaves as consecutive addresses.
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 8;
constexpr int kTileKeys = kThreads * kRounds;  // 2048
constexpr int kScanBlock = 4096;                // counts scanned per block

// Exclusive scan of one value per thread over a 256-thread block (the block
// total goes to *total when given).
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch /* >= 4 */,
                                         uint32_t* total = nullptr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += scratch[w];
  if (total) *total = scratch[0] + scratch[1] + scratch[2] + scratch[3];
  __syncthreads();
  return base + x - v;
}

// Whether a key passes the pass's range filter (the first pass of a chunk
// picks the chunk's distance range out of all keys).
__device__ inline bool kept(uint64_t key, const KeyFilter& f) {
  const uint64_t v = key >> f.fshift;
  return v >= f.flo && v < f.fhi;
}

// Load this wave's kRounds x 64 keys of the tile and rank each among equal
// digits inside the wave (running counts per wave in wcnt).

__device__ inline void load_and_rank(const uint64_t* __restrict__ in, int64_t count, int64_t base,
                                     int shift, int bits, uint32_t dmask, const KeyFilter& f,
                                     uint64_t (&key)[kRounds], uint32_t (&rank)[kRounds],
                                     uint32_t* wcnt_wave) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int64_t idx = base + k * 64 + lane;
    const bool valid = idx < count;
    key[k] = valid ? in[idx] : 0;
  }
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const bool valid = base + k * 64 + lane < count && kept(key[k], f);
    const uint32_t dg = (uint32_t)(key[k] >> shift) & dmask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t bb = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    uint32_t before = 0, cnt = 0;
    if (valid) {
      before = __popcll(peers & lt_mask);
      cnt = wcnt_wave[dg];
    }
    rank[k] = cnt + before;
    // Every lane has read the running count before the first lane of each
    // digit group advances it (LDS operations of one wave complete in order).
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcnt_wave[dg] = cnt + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(kThreads) void k_radix_count(const uint64_t* __restrict__ in,
                                                          int64_t count, int shift, int bits,
                                                          int64_t ntiles,
                                                          uint32_t* __restrict__ counts,
                                                          KeyFilter f) {
  __shared__ uint32_t h[kWaves][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nbins = 1u << bits, dmask = nbins - 1u;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) h[w][tid] = 0;
  __syncthreads();
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kTileKeys + (int64_t)wave * 64 * kRounds;
  uint64_t key[kRounds];
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int64_t idx = base + k * 64 + lane;
    key[k] = idx < count ? in[idx] : 0;
  }
#pragma unroll
  for (int k = 0; k < kRounds; ++k)
    if (base + k * 64 + lane < count && kept(key[k], f))
      atomicAdd(&h[wave][(uint32_t)(key[k] >> shift) & dmask], 1u);
  __syncthreads();
  if ((uint32_t)tid < nbins)
    counts[(int64_t)tid * ntiles + tile] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

// One 1024-thread workgroup per digit: exclusive scan, in place, of that
// digit's tile counts (tile order); the digit's total goes to totals[digit].
// (Also any set of short count arrays laid end to end.)
constexpr int kDigitScanThreads = 1024;
__global__ __launch_bounds__(kDigitScanThreads) void k_radix_digit_scan(
    uint32_t* __restrict__ counts, int64_t ntiles, uint32_t* __restrict__ totals) {
  constexpr int kW = kDigitScanThreads / 64;
  constexpr int kPer = 8;  // consecutive counts per thread
  constexpr int kSpan = kPer * kDigitScanThreads;
  __shared__ uint32_t wsum[kW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* c = counts + (int64_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += kSpan) {
    const int64_t p0 = b0 + threadIdx.x * kPer;
    uint32_t x[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      x[q] = p0 + q < ntiles ? c[p0 + q] : 0;
      sum += x[q];
    }
    // exclusive scan of the thread sums over the block
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
      before += w < wave ? wsum[w] : 0u;
      all += wsum[w];
    }
    __syncthreads();
    uint32_t run = carry + before + incl - sum;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (p0 + q < ntiles) c[p0 + q] = run;
      run += x[q];
    }
    carry += all;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Exclusive scan of `len` counts: per-block totals, a scan of the totals,
// then each block scans its part with its offset.
__global__ __launch_bounds__(kThreads) void k_scan_totals(const uint32_t* __restrict__ v,
                                                          int64_t len,
                                                          uint32_t* __restrict__ totals) {
  __shared__ uint32_t tmp[4];
  const int64_t b0 = blockIdx.x * (int64_t)kScanBlock;
  uint32_t s = 0;
  for (int k = threadIdx.x; k < kScanBlock; k += kThreads)
    if (b0 + k < len) s += v[b0 + k];
  const uint32_t ex = block_exclusive_scan(s, tmp);
  if (threadIdx.x == kThreads - 1) totals[blockIdx.x] = ex + s;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(uint32_t* totals, int64_t nblocks) {
  __shared__ uint32_t tmp[4];
  __shared__ uint32_t last;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += kThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t x = b < nblocks ? totals[b] : 0;
    const uint32_t ex = block_exclusive_scan(x, tmp);
    if (threadIdx.x == kThreads - 1) last = ex + x;
    __syncthreads();
    if (b < nblocks) totals[b] = carry + ex;
    carry += last;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(uint32_t* __restrict__ v, int64_t len,
                                                         const uint32_t* __restrict__ totals) {
  __shared__ uint32_t tmp[4];
  constexpr int kPer = kScanBlock / kThreads;  // 16 consecutive counts per thread
  const int64_t p0 = blockIdx.x * (int64_t)kScanBlock + threadIdx.x * kPer;
  uint32_t x[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    x[q] = p0 + q < len ? v[p0 + q] : 0;
    s += x[q];
  }
  uint32_t run = (totals ? totals[blockIdx.x] : 0u) + block_exclusive_scan(s, tmp);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (p0 + q < len) v[p0 + q] = run;
    run += x[q];
  }
}

// k_scan_apply for a scan of at most kScanDirectBlocks blocks: each block
// sums the raw totals of the blocks before it itself (no separate scan of
// the totals).
constexpr int64_t kScanDirectBlocks = 1024;
__global__ __launch_bounds__(kThreads) void k_scan_apply_direct(uint32_t* __restrict__ v,
                                                                int64_t len,
                                                                const uint32_t* __restrict__ sums) {
  __shared__ uint32_t tmp[4];
  uint32_t before = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kThreads) before += sums[b];
  uint32_t all = 0;
  (void)block_exclusive_scan(before, tmp, &all);
  constexpr int kPer = kScanBlock / kThreads;
  const int64_t p0 = blockIdx.x * (int64_t)kScanBlock + threadIdx.x * kPer;
  uint32_t x[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    x[q] = p0 + q < len ? v[p0 + q] : 0;
    s += x[q];
  }
  uint32_t run = all + block_exclusive_scan(s, tmp);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (p0 + q < len) v[p0 + q] = run;
    run += x[q];
  }
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                            uint64_t* __restrict__ out,
                                                            int64_t count, int shift, int bits,
                                                            int64_t ntiles,
                                                            const uint32_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ totals,
                                                            int32_t* err, KeyFilter f,
                                                            int64_t out_count) {
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t tile_start[256];  // first LDS slot of each digit in the tile
  __shared__ uint32_t gbase[256];       // output position of the digit's first key here
  __shared__ uint32_t scan_tmp[kWaves];
  __shared__ uint64_t skeys[kTileKeys];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nbins = 1u << bits, dmask = nbins - 1u;
  // The digit's first output position: the totals of the smaller digits.
  const uint32_t dstart = block_exclusive_scan((uint32_t)tid < nbins ? totals[tid] : 0u, scan_tmp);
  for (int b = tid; b < 256; b += kThreads)
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][b] = 0;
  __syncthreads();
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kTileKeys + (int64_t)wave * 64 * kRounds;
  uint64_t key[kRounds];
  uint32_t rank[kRounds];
  load_and_rank(in, count, base, shift, bits, dmask, f, key, rank, wcnt[wave]);
  __syncthreads();

  // Per digit: prefix over waves, the tile total, its start in the tile.
  uint32_t total = 0;
  {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][tid];
      wcnt[w][tid] = run;
      run += c;
    }
    total = (uint32_t)tid < nbins ? run : 0;
  }
  uint32_t tile_kept;
  const uint32_t start = block_exclusive_scan(total, scan_tmp, &tile_kept);
  tile_start[tid] = start;
  gbase[tid] = (uint32_t)tid < nbins ? dstart + offsets[(int64_t)tid * ntiles + tile] : 0;
  __syncthreads();

#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    if (base + k * 64 + lane < count && kept(key[k], f)) {
      const uint32_t dg = (uint32_t)(key[k] >> shift) & dmask;
      skeys[tile_start[dg] + wcnt[wave][dg] + rank[k]] = key[k];
    }
  }
  __syncthreads();
  bool oob = false;
  for (int pos = tid; pos < (int)tile_kept; pos += kThreads) {
    const uint64_t k = skeys[pos];
    const uint32_t dg = (uint32_t)(k >> shift) & dmask;
    const uint64_t dst = (uint64_t)gbase[dg] + (uint64_t)(pos - tile_start[dg]);
    if (dst < (uint64_t)out_count)
      out[dst] = k;
    else
      oob = true;  // inconsistent counts: report, never write outside
  }
  if (oob) atomicOr(err, 2);
}

}  // namespace

int64_t radix_tiles(int64_t count) { return (count + kTileKeys - 1) / kTileKeys; }

int64_t radix_count_entries(int64_t count) { return 256 * radix_tiles(count) + 256; }

hipError_t launch_radix_pass(const uint64_t* in, uint64_t* out, int64_t count, int shift,
                             int bits, uint32_t* counts, int32_t* err, hipStream_t s,
                             KeyFilter f, int64_t expect) {
  const int64_t out_count = expect >= 0 ? expect : count;
  const int64_t tiles = radix_tiles(count);
  if (tiles == 0) return hipSuccess;
  const unsigned nbins = 1u << bits;
  uint32_t* totals = counts + 256 * tiles;
  hipLaunchKernelGGL(k_radix_count, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, count,
                     shift, bits, tiles, counts, f);
  hipLaunchKernelGGL(k_radix_digit_scan, dim3(nbins), dim3(kDigitScanThreads), 0, s, counts,
                     tiles, totals);
  hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out,
                     count, shift, bits, tiles, (const uint32_t*)counts,
                     (const uint32_t*)totals, err, f, out_count);
  return hipGetLastError();
}

hipError_t launch_scan_columns(uint32_t* v, int64_t len, int cols, uint32_t* totals,
                               hipStream_t s) {
  if (len <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_radix_digit_scan, dim3((unsigned)cols), dim3(kDigitScanThreads), 0, s, v,
                     len, totals);
  return hipGetLastError();
}

int64_t scan_totals_len(int64_t len) { return (len + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan_u32(uint32_t* v, int64_t len, uint32_t* totals, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int64_t nblocks = (len + kScanBlock - 1) / kScanBlock;
  if (nblocks == 1) {  // one block: its base is 0, no totals pass needed
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kThreads), 0, s, v, len,
                       (const uint32_t*)nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nblocks), dim3(kThreads), 0, s, v, len, totals);
  if (nblocks <= kScanDirectBlocks) {  // two launches: the apply sums the totals before it
    hipLaunchKernelGGL(k_scan_apply_direct, dim3((unsigned)nblocks), dim3(kThreads), 0, s, v, len,
                       (const uint32_t*)totals);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, totals, nblocks);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblocks), dim3(kThreads), 0, s, v, len, totals);
  return hipGetLastError();
}

}  // namespace ph0
