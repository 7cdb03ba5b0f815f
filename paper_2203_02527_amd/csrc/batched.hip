// batched.hip -- many small clouds in one persistent launch.
//
// Each 512-thread workgroup takes the next cloud from an atomic queue (the
// host orders clouds largest first) and runs the whole barcode algorithm of
// Section 2 for it, the five GPU steps of Section 4 fused in one workgroup:
//   * points and the pivot table live in LDS: every stored column is
//     2-sparse, {x, r}, so row r keeps only x (part[r], -1 while free; at
//     most 512 entries);
//   * distances are recomputed from LDS as needed: a histogram of the
//     squared distances picks chunks of whole histogram bins, lowest first;
//     a chunk's edges are compacted in colex order into per-workgroup scratch
//     and sorted by stable LSD radix passes on the distance bits, which gives
//     the (delta, j, i) order; grades continue across chunks (chunks are
//     disjoint distance ranges);
//   * the chunk is reduced with the same exact round scheme as the large
//     path (walk every active column against the table, commit the survivors
//     no earlier column can pre-empt, carry the rest), with the window state
//     in LDS and __syncthreads as the round barrier;
//   * once N-1 pivots exist the cloud is done (later columns reduce to zero);
//     usually the first chunk suffices and most edges are never sorted;
//   * the N deaths are sorted in LDS and written as the canonical barcode.
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kMaxN = kBatchMaxN;
constexpr int kMaxPts = kBatchMaxPts;
constexpr int kBins = 1024;
constexpr int kWindow = 2048;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kActiveB = 0, kFinal = 1;

// Per-workgroup LDS; kWaves waves per workgroup (the radix pass keeps one
// digit histogram per wave).
template <int kWaves>
struct Shared {
  int16_t pts[kMaxPts];
  int16_t part[kMaxN];
  uint32_t hist[kBins];
  uint32_t wcnt[kWaves][256];
  uint32_t digit_base[256];
  uint32_t tile_tot[256];
  int16_t wa[kWindow], wr[kWindow], wrlo[kWindow];
  int32_t wpos[kWindow];
  uint8_t wst[kWindow];
  uint32_t death[kMaxN];
  uint32_t lowc[kMaxN], touch[kMaxN];
  uint32_t scan_tmp[kWaves];
  int32_t dmin[64], dmax[64];
  uint32_t s_cloud, s_fd, s_pivots, s_count, s_keep, s_bin_hi;
  uint64_t s_bound;
};

template <int kWaves>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t t = tmp[w];
    base += w < wave ? t : 0;
    all += t;
  }
  __syncthreads();
  if (total) *total = all;
  return base + x - v;
}

// Edge e (colex) -> (j, i): e = j(j-1)/2 + i, i < j.
__device__ inline void edge_ij(int64_t e, int* j, int* i) {
  int jj = (int)((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);
  while ((int64_t)jj * (jj - 1) / 2 > e) --jj;
  while ((int64_t)(jj + 1) * jj / 2 <= e) ++jj;
  *j = jj;
  *i = (int)(e - (int64_t)jj * (jj - 1) / 2);
}

// Step a colex position (j, i) forward by `step` edges (j only grows).
__device__ inline void edge_advance(int* j, int* i, int step) {
  int ii = *i + step, jj = *j;
  while (ii >= jj) {
    ii -= jj;
    ++jj;
  }
  *i = ii;
  *j = jj;
}

template <class SH>
__device__ inline uint64_t sqdist(const SH& S, int d, int i, int j) {
  uint64_t s = 0;
  for (int k = 0; k < d; ++k) {
    const int64_t df = (int64_t)S.pts[i * d + k] - (int64_t)S.pts[j * d + k];
    s += (uint64_t)(df * df);
  }
  return s;
}

// One stable LSD pass of `cnt` keys in src -> dst on digit (key >> shift)
// of `bits` <= 8 bits.
template <int kThreads>
__device__ void block_radix_pass(Shared<kThreads / 64>& S, const uint64_t* src, uint64_t* dst,
                                 int64_t cnt, int shift, int bits) {
  constexpr int kWaves = kThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nb = 1u << bits, dmask = nb - 1u;
  if (tid < 256) S.digit_base[tid] = 0;
  __syncthreads();
  for (int64_t p = tid; p < cnt; p += kThreads)
    atomicAdd(&S.digit_base[(uint32_t)(src[p] >> shift) & dmask], 1u);
  __syncthreads();
  {
    const uint32_t v = tid < 256 ? S.digit_base[tid] : 0;
    const uint32_t ex = block_excl_scan<kWaves>(v, S.scan_tmp, nullptr);
    if (tid < 256) S.digit_base[tid] = ex;
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int64_t t0 = 0; t0 < cnt; t0 += kThreads) {
    for (int k = tid; k < kWaves * 256; k += kThreads) (&S.wcnt[0][0])[k] = 0;
    __syncthreads();
    const int64_t p = t0 + tid;
    const bool valid = p < cnt;
    const uint64_t key = valid ? src[p] : 0;
    const uint32_t dg = (uint32_t)(key >> shift) & dmask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t bb = __ballot((dg >> b) & 1u);
      peers &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t before = __popcll(peers & lt);
    if (valid && before == 0) S.wcnt[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    // per digit: exclusive prefix over waves (thread = digit)
    if (tid < 256) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = S.wcnt[w][tid];
        S.wcnt[w][tid] = run;
        run += c;
      }
      S.tile_tot[tid] = run;
    }
    __syncthreads();
    if (valid) dst[S.digit_base[dg] + S.wcnt[wave][dg] + before] = key;
    __syncthreads();
    if (tid < 256) S.digit_base[tid] += S.tile_tot[tid];
    __syncthreads();
  }
}

__device__ inline uint32_t benc(int round, int pos) {
  return ((uint32_t)(0x7FFF - (round & 0x7FFF)) << 17) | (uint32_t)pos;
}

// Reduce the sorted chunk keys[0..cnt) (grades in gr) against the LDS table.
// `round` runs on across the chunks of one cloud: the per-row minima are
// tagged with it, so a value left by an earlier round never matches.
template <int kThreads>
__device__ void reduce_chunk(Shared<kThreads / 64>& S, const uint64_t* keys, const uint32_t* gr,
                             int64_t cnt, int n, int ib, int* err, int& round) {
  const int tid = threadIdx.x;
  const uint64_t imask = (1ull << ib) - 1ull;
  int64_t next = 0;
  int nwin = 0;
  int64_t rounds_here = 0;
  while (true) {
    // Refill the window with the next columns in sorted order.
    const int64_t room = kWindow - nwin;
    const int64_t take = cnt - next < room ? cnt - next : room;
    for (int t = tid; t < take; t += kThreads) {
      const uint64_t key = keys[next + t];
      S.wa[nwin + t] = (int16_t)(key & imask);
      S.wr[nwin + t] = (int16_t)((key >> ib) & imask);
      S.wrlo[nwin + t] = S.wa[nwin + t];
      S.wpos[nwin + t] = (int32_t)(next + t);
      S.wst[nwin + t] = kActiveB;
    }
    nwin += (int)take;
    next += take;
    if (tid == 0) {
      S.s_fd = kNone;
      S.s_keep = kNone;
      S.s_count = 0;
    }
    if ((round & 0x7FFF) == 0 && round > 0) {  // the 15-bit round tag wraps: clear
      for (int k = tid; k < n; k += kThreads) {
        S.lowc[k] = kNone;
        S.touch[k] = kNone;
      }
    }
    __syncthreads();
    if (nwin == 0) break;

    // Walk every window column against the table, one thread per column.  A
    // column is 2-sparse, {a, r}; adding the stored column {x, r} of row r
    // (x = part[r]) leaves {a, x}, and a free row (part[r] < 0) stops it.
    for (int s = tid; s < nwin; s += kThreads) {
      int a = S.wa[s], r = S.wr[s], rlo = S.wrlo[s];
      int moved = 0;
      bool zero = false;
      while (true) {
        const int x = S.part[r];
        if (x < 0) break;  // row r is free
        ++moved;
        if (x == a || x >= r) {  // zero column (or a corrupt table)
          if (x >= r) *err = 1;
          zero = true;
          break;
        }
        const int lo = x < a ? x : a;
        r = x < a ? a : x;
        a = lo;
      }
      if (zero) {
        S.wst[s] = kFinal;
        continue;
      }
      // Root of row a in the current forest: follow stored columns down.
      int v = moved ? a : rlo;
      while (true) {
        const int c = S.part[v];
        if (c < 0) break;
        if (c >= v) {
          *err = 1;
          break;
        }
        v = c;
      }
      rlo = v;
      S.wa[s] = (int16_t)a;
      S.wr[s] = (int16_t)r;
      S.wrlo[s] = (int16_t)rlo;
      const uint32_t e = benc(round, S.wpos[s]);
      atomicMin(&S.lowc[r], e);
      atomicMin(&S.touch[rlo], e);
    }
    __syncthreads();
    // First survivor whose low repeats an earlier survivor's low, and the
    // first survivor of all (it must finalize: it commits; a round in which
    // it does not reports and stops).
    for (int s = tid; s < nwin; s += kThreads) {
      if (S.wst[s] != kActiveB) continue;
      const uint32_t pos = (uint32_t)S.wpos[s];
      atomicMin(&S.s_keep, pos);
      if (S.lowc[S.wr[s]] != benc(round, S.wpos[s])) atomicMin(&S.s_fd, pos);
    }
    __syncthreads();
    const uint32_t fd = S.s_fd;
    const uint32_t first_active = S.s_keep;
    for (int s = tid; s < nwin; s += kThreads) {
      if (S.wst[s] != kActiveB) continue;
      const int r = S.wr[s], a = S.wa[s];
      const uint32_t e = benc(round, S.wpos[s]);
      if ((uint32_t)S.wpos[s] < fd || (S.lowc[r] == e && S.touch[r] > e)) {
        S.part[r] = (int16_t)a;  // the stored column {a, r}
        S.death[r] = gr[S.wpos[s]];
        S.wst[s] = kFinal;
        atomicAdd(&S.s_pivots, 1u);
      }
    }
    __syncthreads();
    // Compact the window to its still-active columns (order is irrelevant:
    // the commit rule compares sorted positions).
    int16_t ka = 0, kr = 0, krlo = 0;
    int32_t kpos = 0;
    uint32_t keep = 0;
    for (int s0 = 0; s0 < nwin; s0 += kThreads) {
      const int s = s0 + tid;
      const bool k = s < nwin && S.wst[s] == kActiveB;
      if (k) {
        ka = S.wa[s];
        kr = S.wr[s];
        krlo = S.wrlo[s];
        kpos = S.wpos[s];
      }
      uint32_t tot;
      const uint32_t ex = block_excl_scan<kThreads / 64>(k ? 1u : 0u, S.scan_tmp, &tot);
      __syncthreads();
      if (k) {
        const int dsts = (int)(keep + ex);
        if ((uint32_t)kpos == first_active) S.s_count = 1;  // it did not finalize
        S.wa[dsts] = ka;
        S.wr[dsts] = kr;
        S.wrlo[dsts] = krlo;
        S.wpos[dsts] = kpos;
        S.wst[dsts] = kActiveB;
      }
      keep += tot;
      __syncthreads();
    }
    nwin = (int)keep;
    ++round;
    if (S.s_pivots >= (uint32_t)(n - 1)) break;
    // Progress guard: the first active column must be gone (flagged during
    // the compaction above).
    const bool stuck = S.s_count != 0;
    if (stuck || ++rounds_here > cnt + 2) {
      *err = 5;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
}

template <typename T, int kThreads>
__global__ __launch_bounds__(kThreads) void k_batched(BatchArgs A) {
  constexpr int kWaves = kThreads / 64;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  Shared<kWaves>& S = *reinterpret_cast<Shared<kWaves>*>(smem);
  const int tid = threadIdx.x;
  const int d = A.d;
  uint64_t* bufA = A.scratch + (int64_t)blockIdx.x * 2 * A.emax;
  uint64_t* bufB = bufA + A.emax;
  uint32_t* gr = A.grades + (int64_t)blockIdx.x * A.emax;
  const T* X = static_cast<const T*>(A.pts);
  // One cloud (single_n > 0): rows 0 .. single_n - 1, one workgroup, its
  // status always written to errs[0]; otherwise clouds from the queue.
  bool single_done = false;
  while (true) {
    uint32_t ci;
    if (A.single_n > 0) {
      if (single_done) break;
      single_done = true;
      ci = 0;
    } else {
      if (tid == 0) S.s_cloud = atomicAdd(A.queue, 1u);
      __syncthreads();
      ci = S.s_cloud;
      __syncthreads();
      if (ci >= (uint32_t)A.nclouds) break;
    }
    const int c = A.single_n > 0 ? 0 : A.order[ci];
    const int64_t row0 = A.single_n > 0 ? 0 : A.offsets[c];
    const int n = A.single_n > 0 ? (int)A.single_n : (int)(A.offsets[c + 1] - row0);
    if (A.single_n > 0 && tid == 0) A.errs[0] = 0;
    uint32_t* bars = A.bars + 2 * row0;
    if (n < 1) continue;
    if (n > kMaxN || (int64_t)n * d > kMaxPts || d > 64) {
      if (tid == 0) A.errs[c] = 2;
      continue;
    }
    if (n == 1) {
      if (tid == 0) {
        bars[0] = 0;
        bars[1] = kInf;
      }
      continue;
    }
    // Points into LDS; coordinate ranges -> squared-distance bound.
    for (int k = tid; k < n * d; k += kThreads) S.pts[k] = (int16_t)X[row0 * d + k];
    __syncthreads();
    if (tid < d) {
      int lo = 1 << 30, hi = -(1 << 30);
      for (int i = 0; i < n; ++i) {
        const int v = S.pts[i * d + tid];
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
      }
      S.dmin[tid] = lo;
      S.dmax[tid] = hi;
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t b = 0;
      for (int k = 0; k < d; ++k) {
        const uint64_t w = (uint64_t)(S.dmax[k] - S.dmin[k]);
        b += w * w;
      }
      S.s_bound = b;
      S.s_pivots = 0;
    }
    const int ib = 64 - __clzll((uint64_t)(n - 1));
    for (int k = tid; k < n; k += kThreads) S.part[k] = -1;
    for (int k = tid; k < n; k += kThreads) {
      S.death[k] = kInf;
      S.lowc[k] = kNone;
      S.touch[k] = kNone;
    }
    for (int k = tid; k < kBins; k += kThreads) S.hist[k] = 0;
    __syncthreads();
    const uint64_t bound = S.s_bound;
    int dbits = 0;
    while (dbits < 64 && (bound >> dbits) != 0) ++dbits;
    if (dbits + 2 * ib > 64) {
      if (tid == 0) A.errs[c] = 3;
      continue;
    }
    const int hs = dbits > 10 ? dbits - 10 : 0;
    const int64_t E = (int64_t)n * (n - 1) / 2;
    // Histogram of delta >> hs over all edges (each thread steps through
    // colex positions tid, tid + kThreads, ...).
    {
      int j, i;
      edge_ij(tid < E ? tid : 0, &j, &i);
      for (int64_t e = tid; e < E; e += kThreads) {
        atomicAdd(&S.hist[(uint32_t)(sqdist(S, d, i, j) >> hs)], 1u);
        edge_advance(&j, &i, kThreads);
      }
    }
    __syncthreads();
    const int bucket = n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3;
    const int64_t target = (int64_t)A.chunk_mult[bucket] * n;
    uint32_t bin_lo = 0, distinct = 0;
    int err = 0, round = 0;
    while (S.s_pivots < (uint32_t)(n - 1) && bin_lo < (uint32_t)kBins) {
      if (tid == 0) {
        int64_t cum = 0;
        uint32_t b = bin_lo;
        while (b < (uint32_t)kBins && (cum == 0 || cum < target)) cum += S.hist[b++];
        S.s_bin_hi = b;
      }
      __syncthreads();
      const uint32_t bin_hi = S.s_bin_hi;
      // Stable compaction of the chunk's edges, in colex order.
      uint32_t cnt = 0;
      int cj, ci;
      edge_ij(tid < E ? tid : 0, &cj, &ci);
      for (int64_t e0 = 0; e0 < E; e0 += kThreads) {
        const int64_t e = e0 + tid;
        uint64_t key = 0;
        bool in = false;
        if (e < E) {
          const int j = cj, i = ci;
          edge_advance(&cj, &ci, kThreads);
          const uint64_t dl = sqdist(S, d, i, j);
          const uint32_t b = (uint32_t)(dl >> hs);
          in = b >= bin_lo && b < bin_hi;
          key = (dl << (2 * ib)) | ((uint64_t)j << ib) | (uint64_t)i;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>(in ? 1u : 0u, S.scan_tmp, &tot);
        if (in) bufA[cnt + ex] = key;
        cnt += tot;
      }
      __syncthreads();
      // LSD passes over the distance bits that vary inside the chunk.
      uint64_t* src = bufA;
      uint64_t* dst = bufB;
      const int db = A.digit_bits;
      for (int sh = 0; sh < dbits; sh += db) {
        const int bits = dbits - sh < db ? dbits - sh : db;
        block_radix_pass<kThreads>(S, src, dst, cnt, 2 * ib + sh, bits);
        uint64_t* t = src;
        src = dst;
        dst = t;
      }
      // Grades: the chunk's distances all exceed the previous chunks'.
      uint32_t run = distinct;
      for (int64_t p0 = 0; p0 < cnt; p0 += kThreads) {
        const int64_t p = p0 + tid;
        uint32_t f = 0;
        if (p < cnt) f = (p == 0) || ((src[p] >> (2 * ib)) != (src[p - 1] >> (2 * ib)));
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kWaves>(f, S.scan_tmp, &tot);
        if (p < cnt) gr[p] = run + ex + f;
        run += tot;
      }
      distinct = run;
      __syncthreads();
      reduce_chunk<kThreads>(S, src, gr, cnt, n, ib, &err, round);
      bin_lo = bin_hi;
    }
    if (err) A.errs[c] = err;
    // Canonical barcode: bitonic sort of the n deaths in LDS.
    int P = 1;
    while (P < n) P <<= 1;
    uint32_t* sd = S.hist;  // reuse (P <= 512 <= kBins)
    for (int k = tid; k < P; k += kThreads) sd[k] = k < n ? S.death[k] : kInf;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int k = tid; k < P / 2; k += kThreads) {
          const int lo = 2 * k - (k & (stride - 1)), hi = lo + stride;
          const bool up = (lo & size) == 0;
          const uint32_t x = sd[lo], y = sd[hi];
          if ((x > y) == up) {
            sd[lo] = y;
            sd[hi] = x;
          }
        }
        __syncthreads();
      }
    for (int k = tid; k < n; k += kThreads) {
      bars[2 * k] = 0;
      bars[2 * k + 1] = sd[k];
    }
    if (tid == 0 && S.s_pivots != (uint32_t)(n - 1)) A.errs[c] = 4;
    __syncthreads();
  }
}

}  // namespace

size_t batched_shared_bytes(int threads) {
  return threads == 1024 ? sizeof(Shared<16>) : sizeof(Shared<8>);
}

namespace {
template <typename T, int kThreads>
hipError_t launch_batched_t(const BatchArgs& a, int blocks, hipStream_t s) {
  const size_t shm = sizeof(Shared<kThreads / 64>);
  const hipError_t e = hipFuncSetAttribute((const void*)k_batched<T, kThreads>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batched<T, kThreads>), dim3(blocks), dim3(kThreads), shm, s, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_batched(const BatchArgs& a, int blocks, hipStream_t s) {
  if (a.digit_bits < 1 || a.digit_bits > 8 || (a.threads != 512 && a.threads != 1024))
    return hipErrorInvalidValue;
  if (a.elem_bytes == 1)
    return a.threads == 1024 ? launch_batched_t<int8_t, 1024>(a, blocks, s)
                             : launch_batched_t<int8_t, 512>(a, blocks, s);
  return a.threads == 1024 ? launch_batched_t<int16_t, 1024>(a, blocks, s)
                           : launch_batched_t<int16_t, 512>(a, blocks, s);
}

}  // namespace ph0
