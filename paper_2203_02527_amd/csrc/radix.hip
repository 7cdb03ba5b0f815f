// radix.hip -- step 2 of the GPU pipeline (Section 4, step 2: sort the edges):
// one stable least-significant-digit radix pass over 64-bit keys.
//
// A pass reads every key once and writes it once.  Global digit counts come
// precomputed (from the distance kernel), so each workgroup only needs the
// counts of the tiles before it: tiles take their index from an atomic
// ticket, publish their own digit counts, and look back over earlier tiles'
// published counts (decoupled look-back).  A tile waits only on tiles with
// smaller tickets, which have already started, so every wait ends.
//
// Inside a tile (4 waves x 16 rounds x 64 lanes = 4096 keys) each wave owns a
// contiguous quarter; a key's rank among equal digits comes from wave ballots
// on the digit bits, so the order of equal digits is preserved (stability is
// what turns sorting on the distance bits into the (delta, j, i) order).  The
// tile is reordered by digit in LDS before it is written, so that each digit's
// run leaves as consecutive addresses.
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 16;
constexpr int kTileKeys = kThreads * kRounds;  // 4096

constexpr uint64_t kFlagShift = 54;  // descriptor: epoch (8b) | state (2b) | value (54b)
constexpr uint64_t kValueMask = (1ull << kFlagShift) - 1;
constexpr uint64_t kAggregate = 1;
constexpr uint64_t kInclusive = 2;
constexpr int64_t kSpinLimit = 1ll << 26;

__device__ inline uint64_t desc_make(uint32_t epoch, uint64_t state, uint64_t value) {
  return ((uint64_t)(epoch & 0xFF) << 56) | (state << kFlagShift) | value;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch /* >= 4 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += scratch[w];
  __syncthreads();
  return base + x - v;
}

__global__ __launch_bounds__(kThreads) void k_radix_pass(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int64_t count, int shift,
    int bits, const uint32_t* __restrict__ ghist, uint64_t* desc, uint32_t* ticket,
    int32_t* err, uint32_t epoch) {
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t tile_start[256];  // first LDS slot of each digit in the tile
  __shared__ uint64_t gbase[256];       // global position of the digit's first key here
  __shared__ uint32_t scan_tmp[kWaves];
  __shared__ uint64_t skeys[kTileKeys];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nbins = 1u << bits, dmask = nbins - 1u;
  if (tid == 0) s_ticket = atomicAdd(ticket, 1u);
  for (int b = tid; b < 256; b += kThreads)
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][b] = 0;
  __syncthreads();
  const int64_t tile = s_ticket;
  const int64_t base = tile * kTileKeys + (int64_t)wave * 64 * kRounds;

  uint64_t key[kRounds];
  uint32_t rank[kRounds];
  const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int64_t idx = base + k * 64 + lane;
    const bool valid = idx < count;
    key[k] = valid ? in[idx] : 0;
    const uint32_t dg = (uint32_t)(key[k] >> shift) & dmask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t bb = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    uint32_t before = 0, cnt = 0;
    if (valid) {
      before = __popcll(peers & lt_mask);
      cnt = wcnt[wave][dg];
    }
    rank[k] = cnt + before;
    // All lanes have read the running count; the first lane of each digit
    // group advances it (LDS operations of one wave complete in order).
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcnt[wave][dg] = cnt + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // Per digit: prefix over waves, the tile total, and its start in the tile.
  uint32_t total = 0;
  if (tid < 256) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][tid];
      wcnt[w][tid] = run;
      run += c;
    }
    total = (uint32_t)tid < nbins ? run : 0;
  }
  const uint32_t start = block_exclusive_scan(total, scan_tmp);
  const uint32_t gh = (uint32_t)tid < nbins ? ghist[tid] : 0;
  const uint32_t gexcl = block_exclusive_scan(gh, scan_tmp);
  if (tid < 256) tile_start[tid] = start;

  // Decoupled look-back: thread `tid` owns digit `tid`.
  if ((uint32_t)tid < nbins) {
    uint64_t* mine = desc + tile * 256 + tid;
    uint64_t prefix = 0;
    if (tile == 0) {
      __hip_atomic_store(mine, desc_make(epoch, kInclusive, total), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(mine, desc_make(epoch, kAggregate, total), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      int64_t t = tile - 1;
      int64_t spins = 0;
      while (t >= 0) {
        const uint64_t v = __hip_atomic_load(desc + t * 256 + tid, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t state = (v >> kFlagShift) & 3u;
        if ((uint32_t)(v >> 56) != (epoch & 0xFF) || state == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(err, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        prefix += v & kValueMask;
        if (state == kInclusive) break;
        --t;
      }
      __hip_atomic_store(mine, desc_make(epoch, kInclusive, prefix + total), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    gbase[tid] = (uint64_t)gexcl + prefix;
  }
  __syncthreads();

  // Reorder the tile by digit in LDS.
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int64_t idx = base + k * 64 + lane;
    if (idx < count) {
      const uint32_t dg = (uint32_t)(key[k] >> shift) & dmask;
      skeys[tile_start[dg] + wcnt[wave][dg] + rank[k]] = key[k];
    }
  }
  __syncthreads();
  const int64_t tile_base = tile * kTileKeys;
  const int64_t valid_n = count - tile_base < kTileKeys ? count - tile_base : kTileKeys;
  bool oob = false;
  for (int pos = tid; pos < valid_n; pos += kThreads) {
    const uint64_t k = skeys[pos];
    const uint32_t dg = (uint32_t)(k >> shift) & dmask;
    const uint64_t dst = gbase[dg] + (uint64_t)(pos - tile_start[dg]);
    if (dst < (uint64_t)count)
      out[dst] = k;
    else
      oob = true;  // inconsistent digit counts: report, never write outside
  }
  if (oob) atomicOr(err, 2);
}

}  // namespace

int64_t radix_tiles(int64_t count) { return (count + kTileKeys - 1) / kTileKeys; }

hipError_t launch_radix_pass(const uint64_t* in, uint64_t* out, int64_t count, int shift,
                             int bits, const uint32_t* hist_pass, uint64_t* desc,
                             uint32_t* ticket, int32_t* err, uint32_t epoch, hipStream_t s) {
  const int64_t tiles = radix_tiles(count);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_radix_pass, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out, count,
                     shift, bits, hist_pass, desc, ticket, err, epoch);
  return hipGetLastError();
}

}  // namespace ph0
