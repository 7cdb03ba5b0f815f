// keys.hip -- step 1 of the GPU pipeline (Section 4, step 1: the N(N-1)/2
// pairwise distances): one packed 64-bit sort key per edge,
//     key = delta << 2b | j << b | i        (i < j, b = index bits)
// written at the edge's colex position j(j-1)/2 + i, so that the array is
// already in (j, i) order and a stable sort on the delta bits alone yields the
// (delta, j, i) order.  delta is the exact squared Euclidean distance of two
// integer points.  Each workgroup also counts its distances into a histogram
// of `delta >> hist_shift` (kHistBins bins, LDS across all the workgroup's
// tiles, one flush per workgroup), from which the host picks the distance
// ranges the sort has to order.
//
// Two paths:
//  * vector ALU, direct differences (any d, int8 or int16; int64 sums);
//  * int8 MFMA Gram: delta = |x_i|^2 + |x_j|^2 - 2 <x_i, x_j>, the inner
//    products from v_mfma_i32_32x32x32_i8 (exact int32 for d <= 32768).
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kTile = 64;  // points per tile side; a tile covers 64 x 64 edges
constexpr int kSegTiles = 4;  // tiles per count segment of the MFMA passes

__device__ inline void tile_coords(int64_t t, int64_t* jb, int64_t* ib) {
  // Tiles with ib <= jb, numbered row by row: t = jb(jb+1)/2 + ib.
  int64_t j = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  *jb = j;
  *ib = t - j * (j + 1) / 2;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Workgroup k copies entry k of the list.
__global__ __launch_bounds__(256) void k_gather(Gather g) {
  const int k = blockIdx.x;
  for (int i = threadIdx.x; i < g.words[k]; i += blockDim.x) g.dst[k][i] = g.src[k][i];
}

// Per-dimension coordinate ranges: lo[k] = min x_ik, hi[k] = max x_ik
// (minmax = lo[0..d) then hi[0..d)).  A coalesced grid-stride pass over all
// coordinates folds each into LDS per-dimension minima and maxima (d <= kRangeLds),
// then one global atomic pair per dimension and workgroup.
constexpr int kRangeLds = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_coord_range(const T* __restrict__ x, int64_t n,
                                                     int32_t d, int32_t* __restrict__ minmax) {
  __shared__ int32_t lo[kRangeLds], hi[kRangeLds];
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    lo[k] = 0x7FFFFFFF;
    hi[k] = (int32_t)0x80000000;
  }
  __syncthreads();
  const int64_t total = n * d;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int k = (int)(e % d);
  const int kstep = (int)(stride % d);
  for (; e < total; e += stride) {
    const int32_t v = x[e];
    atomicMin(&lo[k], v);
    atomicMax(&hi[k], v);
    k += kstep;
    if (k >= d) k -= d;
  }
  __syncthreads();
  for (int kk = threadIdx.x; kk < d; kk += blockDim.x) {
    if (lo[kk] != 0x7FFFFFFF) atomicMin(&minmax[kk], lo[kk]);
    if (hi[kk] != (int32_t)0x80000000) atomicMax(&minmax[d + kk], hi[kk]);
  }
}

// The same for d > kRangeLds: one dimension per workgroup row of the grid.
template <typename T>
__global__ void k_coord_range_wide(const T* __restrict__ x, int64_t n, int32_t d,
                                   int32_t* __restrict__ minmax) {
  for (int k = blockIdx.y; k < d; k += gridDim.y) {
    int lo = 0x7FFFFFFF, hi = (int32_t)0x80000000;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const int v = x[i * d + k];
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const int l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&minmax[k], lo);
      atomicMax(&minmax[d + k], hi);
    }
  }
}

// Squared norms and per-dimension coordinate ranges of int8 points in one
// pass, for rows made of 16-byte pieces (d = 16 * 2^k <= kRangeLds, 16-byte
// aligned).  The pieces of a row sit in adjacent lanes, which sum the row's
// norm; each thread keeps the running range of its piece's 16 dimensions
// (two rows per step, their loads issued together), folded into LDS and
// then one global atomic pair per dimension and workgroup.
constexpr int kPrepMaxBlocks = 64;

__global__ __launch_bounds__(256) void k_prep_i8(const int8_t* __restrict__ x, int64_t n,
                                                 int32_t d, int32_t* __restrict__ minmax,
                                                 int32_t* __restrict__ norms) {
  __shared__ int32_t lo[kRangeLds], hi[kRangeLds];
  const int segs = d >> 4, seg = threadIdx.x & (segs - 1);
  const int rows = 256 / segs;  // rows per workgroup step
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    lo[k] = 0x7FFFFFFF;
    hi[k] = (int32_t)0x80000000;
  }
  __syncthreads();
  int32_t mn[16], mx[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn[i] = 127;
    mx[i] = -128;
  }
  // Every lane runs the same steps (the bound depends on the workgroup
  // only), so the row sums below see whole rows; rows past n load row n - 1
  // and are not counted.
  auto take = [&](const int4 v, bool ok, int64_t row) {
    const int32_t w[4] = {v.x, v.y, v.z, v.w};
    int32_t sq = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int32_t e = (int32_t)(int8_t)(w[q] >> (8 * b));
        sq += e * e;
        const int i = 4 * q + b;
        mn[i] = ok && e < mn[i] ? e : mn[i];
        mx[i] = ok && e > mx[i] ? e : mx[i];
      }
    for (int o = 1; o < segs; o <<= 1) sq += __shfl_xor(sq, o, 64);
    if (ok && seg == 0) norms[row] = sq;
  };
  const int64_t step = (int64_t)gridDim.x * rows;
  for (int64_t r0 = blockIdx.x * (int64_t)rows; r0 < n; r0 += 2 * step) {
    const int64_t ra = r0 + threadIdx.x / segs, rb = ra + step;
    const bool oka = ra < n, okb = rb < n;
    const int4 va = *reinterpret_cast<const int4*>(x + (oka ? ra : n - 1) * d + seg * 16);
    const int4 vb = *reinterpret_cast<const int4*>(x + (okb ? rb : n - 1) * d + seg * 16);
    take(va, oka, ra);
    take(vb, okb, rb);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    atomicMin(&lo[seg * 16 + i], mn[i]);
    atomicMax(&hi[seg * 16 + i], mx[i]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    atomicMin(&minmax[k], lo[k]);
    atomicMax(&minmax[d + k], hi[k]);
  }
}

// lo[0..d) = INT_MAX, hi[0..d) = INT_MIN, and zero[0..zero_len) = 0.
__global__ void k_range_init(int32_t* __restrict__ minmax, int32_t d, uint32_t* __restrict__ zero,
                             int64_t zero_len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 2 * (int64_t)d + zero_len;
       k += stride) {
    if (k < 2 * (int64_t)d)
      minmax[k] = k < d ? 0x7FFFFFFF : (int32_t)0x80000000;
    else
      zero[k - 2 * (int64_t)d] = 0u;
  }
}

// ---- vector ALU path ----
constexpr int kChunk = 32;  // dimensions staged per LDS round

__device__ inline void hist_zero(uint32_t* lh) {
  for (int b = threadIdx.x; b < kHistBins; b += blockDim.x) lh[b] = 0;
}

__device__ inline void hist_flush(const uint32_t* lh, uint32_t* hist) {
  __syncthreads();
  for (int b = threadIdx.x; b < kHistBins; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// Counts of the count pass are kept per (64-row band J, row of the band,
// segment s): segment s of band J covers its tiles I in [sS, min(sS + S,
// J + 1)), S tiles per segment (S = 1: one count per tile).  Flattened
// bands in order, then rows, then segments, so that an exclusive scan of the
// counts gives each (row, segment) the colex position of its first kept key
// among all kept keys.
__host__ __device__ inline int32_t seg_count(int64_t J, int S) { return (int32_t)(J / S) + 1; }
// Segments of the bands before J: sum over J' < J of (J' / S + 1).
__host__ __device__ inline int64_t seg_base(int64_t J, int S) {
  const int64_t q = J / S, r = J - q * S;
  return J + S * (q * (q - 1) / 2) + q * r;
}
__device__ inline int64_t key_count_index(int64_t J, int jl, int64_t s, int S) {
  return 64 * seg_base(J, S) + (int64_t)jl * seg_count(J, S) + s;
}

// Tiles a pass visits: all, or every kp.sample-th one for the sampled
// histogram.  The full passes stride over the tiles by the grid; the sampled
// pass gives each workgroup a contiguous run of the visited tiles (tile
// t = v * sample for v in [v0, v1)), so that it runs with few workgroups,
// each flushing its LDS histogram once.
struct TileRange {
  int64_t v0, v1, step, sample;
};
__device__ inline TileRange tile_range(const KeyPass& kp, int mode, int64_t ntiles) {
  TileRange r;
  if (mode == kKeysHist) {
    r.sample = kp.sample;
    const int64_t visited = (ntiles + r.sample - 1) / r.sample;
    const int64_t per = (visited + gridDim.x - 1) / gridDim.x;
    r.v0 = blockIdx.x * per;
    r.v1 = r.v0 + per < visited ? r.v0 + per : visited;
    r.step = 1;
  } else {
    r.sample = 1;
    r.v0 = blockIdx.x;
    r.v1 = ntiles;
    r.step = gridDim.x;
  }
  return r;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_keys_alu(const T* __restrict__ x, int64_t n, int32_t d,
                                                  int ib, int64_t ntiles, KeyPass kp) {
  __shared__ int32_t xs[2][kTile][kChunk + 1];
  __shared__ uint32_t lh[kHistBins];
  constexpr bool kHist = MODE == kKeysFull || MODE == kKeysHist;
  if (kHist) hist_zero(lh);
  const int hs = kHist && kp.hist_shift_dev ? *kp.hist_shift_dev : kp.hist_shift;

  const int il = threadIdx.x & 63;   // i inside the tile (one per lane)
  const int jl0 = threadIdx.x >> 6;  // first j of this wave; j = jl0 + 4q
  const TileRange tr = tile_range(kp, MODE, ntiles);
  for (int64_t v = tr.v0; v < tr.v1; v += tr.step) {
    const int64_t t = v * tr.sample;
    int64_t jb, ibk;
    tile_coords(t, &jb, &ibk);
    const int64_t i0 = ibk * kTile, j0 = jb * kTile;
    int64_t acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0;
    for (int k0 = 0; k0 < d; k0 += kChunk) {
      const int kc = d - k0 < kChunk ? d - k0 : kChunk;
      __syncthreads();
      for (int e = threadIdx.x; e < kTile * kc; e += blockDim.x) {
        const int pt = e / kc, kk = e - pt * kc;
        const int64_t gi = i0 + pt, gj = j0 + pt;
        xs[0][pt][kk] = gi < n ? (int32_t)x[gi * d + k0 + kk] : 0;
        xs[1][pt][kk] = gj < n ? (int32_t)x[gj * d + k0 + kk] : 0;
      }
      __syncthreads();
      for (int kk = 0; kk < kc; ++kk) {
        const int32_t xi = xs[0][il][kk];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int64_t df = (int64_t)(xi - xs[1][jl0 + 4 * q][kk]);
          acc[q] += df * df;
        }
      }
    }
    const int64_t i = i0 + il;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int jl = jl0 + 4 * q;
      const int64_t j = j0 + jl;
      const bool valid = j < n && i < j;
      const uint64_t delta = (uint64_t)acc[q];
      const uint64_t key = (delta << (2 * ib)) | ((uint64_t)j << ib) | (uint64_t)i;
      if constexpr (kHist) {
        if (valid) {
          if (MODE == kKeysFull) kp.keys[j * (j - 1) / 2 + i] = key;
          atomicAdd(&lh[delta >> hs], 1u);
        }
      } else {
        // One wave covers the 64 i of row j: a ballot counts and ranks.
        const bool kept = valid && delta >= kp.dlo && delta < kp.dhi;
        const uint64_t m = __ballot(kept);
        const int64_t ci = key_count_index(jb, jl, ibk, 1);
        if (MODE == kKeysCount) {
          if (il == 0) kp.cnt[ci] = (uint32_t)__popcll(m);
        } else if (kept) {
          const uint32_t below = __popcll(m & ((1ull << il) - 1ull));
          kp.keys[kp.cnt[ci] + below] = key;
        }
      }
    }
  }
  if (kHist) hist_flush(lh, kp.hist);
}

// ---- int8 MFMA Gram path ----
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

constexpr int kMaxDpad = 256;  // int8 dims staged per LDS round (multiple of 32)

// Squared norms |x_i|^2 of int8 points (exact int32 for d <= 32768).
__global__ void k_norms_i8(const int8_t* __restrict__ x, int64_t n, int32_t d,
                           int32_t* __restrict__ norms) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = 0;
    for (int32_t k = 0; k < d; ++k) {
      const int32_t v = x[i * d + k];
      s += v * v;
    }
    norms[i] = s;
  }
}

// Rows of one tile for the single-stage path (d <= 64, 16-byte aligned rows):
// at most 2 x 64 rows x 4 segments of 16 bytes, two per thread.  Loaded into
// registers one tile ahead, so the loads of the next tile overlap the
// current tile's MFMA and epilogue.
struct TileRegs {
  int4 v[2];
};

__device__ inline void tile_regs_load(TileRegs& r, const int8_t* __restrict__ x, int64_t n,
                                      int32_t d, int64_t i0, int64_t j0, int segs) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * 256;
    r.v[q] = make_int4(0, 0, 0, 0);
    if (e < 2 * 64 * segs) {
      const int side = e / (64 * segs), rem = e - side * 64 * segs;
      const int pt = rem / segs, sg = rem - pt * segs;
      const int64_t g = (side ? j0 : i0) + pt;
      if (g < n && 16 * sg < d) r.v[q] = *reinterpret_cast<const int4*>(x + g * d + 16 * sg);
    }
  }
}

template <int KROW>
__device__ inline void tile_regs_store(const TileRegs& r, int8_t (*xs)[64][KROW], int segs) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < 2 * 64 * segs) {
      const int side = e / (64 * segs), rem = e - side * 64 * segs;
      const int pt = rem / segs, sg = rem - pt * segs;
      *reinterpret_cast<int4*>(&xs[side][pt][16 * sg]) = r.v[q];
    }
  }
}

// KMAX int8 dimensions are staged per LDS round (64 for d <= 64, else 256);
// rows are padded by 16 bytes so that the 32 row reads of a half-wave spread
// over the LDS banks.  With vec16 (d a multiple of 16 and 16-byte aligned
// points) the rows are copied with 16-byte loads.  AHEAD (d <= 64, vec16)
// loads each tile's rows, norms and (emit) row bases while the previous tile
// computes; it is an instantiation of its own so that no wait of the general
// path's loads lands in its loop.
//
// Work is handed out in items: a count segment (up to kSegTiles consecutive
// tiles I of one band J) for the full, count and emit passes, one sampled
// tile for the histogram pass.  The count pass leaves one count per (row,
// segment), the emit pass starts each segment's rows at their scanned counts
// and advances them tile by tile.
//
// Waves per SIMD each pass is compiled for at least: four for the emit pass
// with d <= 64 (a few bytes spill), three for the others (the count and
// histogram passes then fit five).
constexpr int keys_waves(int mode, int kmax) { return mode == kKeysEmit && kmax == 64 ? 4 : 3; }

// The tile being worked on and the item it belongs to (ok = 0 past the
// workgroup's last item).
struct Cursor {
  int64_t item;
  int32_t J, I, I0, I1;  // band, tile, the item's first tile and its end
  int32_t ok;
};

// The item's band and tiles: a sampled tile (sample > 0), else count
// segment `item` of the nb bands.
__device__ inline Cursor item_cursor(int64_t item, int64_t item_end, int64_t sample, int32_t nb,
                                     int S) {
  Cursor cu;
  cu.item = item;
  cu.ok = item < item_end;
  cu.J = cu.I = cu.I0 = cu.I1 = 0;
  if (!cu.ok) return cu;
  if (sample > 0) {
    int64_t jb, ibk;
    tile_coords(item * sample, &jb, &ibk);
    cu.J = (int32_t)jb;
    cu.I0 = cu.I = (int32_t)ibk;
    cu.I1 = cu.I + 1;
  } else {
    // the band: seg_base(J) <= item < seg_base(J + 1)
    int32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (seg_base(mid, S) <= item) lo = mid; else hi = mid;
    }
    cu.J = lo;
    cu.I0 = cu.I = (int32_t)(item - seg_base(lo, S)) * S;
    cu.I1 = cu.I0 + S < lo + 1 ? cu.I0 + S : lo + 1;
  }
  return cu;
}

template <int MODE, int KMAX, bool AHEAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(keys_waves(MODE, KMAX)))) void k_keys_mfma(const int8_t* __restrict__ x, int64_t n,
                                                   int32_t d, int ib, int64_t ntiles,
                                                   const int32_t* __restrict__ norms,
                                                   bool vec16, KeyPass kp) {
  constexpr int kRow = KMAX + 16;
  constexpr bool kHist = MODE == kKeysFull || MODE == kKeysHist;
  constexpr int S = kSegTiles;
  __shared__ __attribute__((aligned(16))) int8_t xs[2][kTile][kRow];
  __shared__ __attribute__((aligned(16))) int32_t nrm[2][kTile];
  __shared__ uint32_t lh[kHist ? kHistBins : 1];
  // Kept keys of each wave's rows in the tile: hcp[wave][r] holds the count
  // of accumulator r's lower half-wave row in its low 16 bits and that of
  // its upper half-wave row in its high 16 bits (32 i each).
  __shared__ __attribute__((aligned(16))) uint32_t hcp[4][16];
  __shared__ __attribute__((aligned(16))) uint32_t rbase[kTile];  // emit: colex base of each row's kept keys
  // emit: each wave's queue of kept keys (delta << 32 | r << 6 | lane) for
  // one half of its accumulators, and where each r's entries start
  constexpr int kQueue = MODE == kKeysEmit ? 512 : 1;
  __shared__ uint64_t q_keys[4][kQueue];
  __shared__ __attribute__((aligned(16))) uint32_t q_start[4][16];
  // Kept keys of tile row jl (0..63) in the i-half `sub` (the wave jl / 32 * 2 + sub).
  auto row_count = [&](int jl, int sub) -> uint32_t {
    const int o = jl & 31, r = 4 * (o >> 3) + (o & 3);
    return (hcp[(jl >> 5) * 2 + sub][r] >> (16 * ((o >> 2) & 1))) & 0xFFFFu;
  };
  if (kHist) hist_zero(lh);
  const int hs = kHist && kp.hist_shift_dev ? *kp.hist_shift_dev : kp.hist_shift;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int jsub = wave >> 1, isub = wave & 1;  // 32 x 32 sub-tile of this wave
  // The kept range [dlo, dhi) clamped to 32 bits (delta < 2^31 here).
  const uint32_t dlo32 = kp.dlo < 0xFFFFFFFFull ? (uint32_t)kp.dlo : 0xFFFFFFFFu;
  const uint32_t dhi32 = kp.dhi < 0xFFFFFFFFull ? (uint32_t)kp.dhi : 0xFFFFFFFFu;
  const uint32_t span32 = dhi32 > dlo32 ? dhi32 - dlo32 : 0u;
  constexpr bool ahead = AHEAD && KMAX == 64;
  const int segs1 = ((d + 31) & ~31) >> 4;
  const int32_t nb = (int32_t)((n + kTile - 1) / kTile);

  // Items of this workgroup: a contiguous run of sampled tiles, or the
  // segments blockIdx.x, blockIdx.x + gridDim.x, ...
  int64_t item_end, item_step, item0;
  if (MODE == kKeysHist) {
    const int64_t visited = (ntiles + kp.sample - 1) / kp.sample;
    const int64_t per = (visited + gridDim.x - 1) / gridDim.x;
    item0 = blockIdx.x * per;
    item_end = item0 + per < visited ? item0 + per : visited;
    item_step = 1;
  } else {
    item0 = blockIdx.x;
    item_end = seg_base(nb, S);
    item_step = gridDim.x;
  }
  const int64_t sample = MODE == kKeysHist ? kp.sample : 0;
  auto next_of = [&](Cursor cu) {
    if (cu.I + 1 < cu.I1) {
      ++cu.I;
      return cu;
    }
    return item_cursor(cu.item + item_step, item_end, sample, nb, S);
  };
  // The count slot of (band, row, segment) for the tile's segment.
  auto count_slot = [&](const Cursor& cu, int row) {
    return key_count_index(cu.J, row, cu.I0 / S, S);
  };

  TileRegs pre;
  int32_t pre_nrm = 0;
  uint32_t pre_rb = 0;
  auto side_load = [&](const Cursor& cu) {
    if (threadIdx.x < 2 * kTile) {
      const int side = threadIdx.x >> 6, pt = threadIdx.x & 63;
      const int64_t g = (int64_t)(side ? cu.J : cu.I) * kTile + pt;
      pre_nrm = g < n ? norms[g] : 0;
    }
    if (MODE == kKeysEmit && threadIdx.x < kTile && cu.I == cu.I0)
      pre_rb = kp.cnt[count_slot(cu, threadIdx.x)];
  };
  Cursor cur = item_cursor(item0, item_end, sample, nb, S);
  if (ahead && cur.ok) {
    tile_regs_load(pre, x, n, d, (int64_t)cur.I * kTile, (int64_t)cur.J * kTile, segs1);
    side_load(cur);
  }
  uint32_t row_acc = 0;  // count / emit: thread tid < 64's row, over the segment so far
  while (cur.ok) {
    const int64_t i0 = (int64_t)cur.I * kTile, j0 = (int64_t)cur.J * kTile;
    const bool seg_first = cur.I == cur.I0, seg_last = cur.I + 1 == cur.I1;
    v16i c;
    if constexpr (!ahead) {
#pragma unroll
      for (int r = 0; r < 16; ++r) c[r] = 0;
    }
    __syncthreads();  // the previous tile's readers of LDS are done
    if constexpr (MODE == kKeysEmit) {
      // The row's next output position: its segment base, advanced by the
      // previous tile's kept keys (still in hcp).
      if (threadIdx.x < kTile) {
        if (seg_first)
          row_acc = ahead ? pre_rb : kp.cnt[count_slot(cur, threadIdx.x)];
        else
          row_acc += row_count(threadIdx.x, 0) + row_count(threadIdx.x, 1);
        rbase[threadIdx.x] = row_acc;
      }
    }
    if constexpr (ahead) {
      if (threadIdx.x < 2 * kTile) nrm[threadIdx.x >> 6][threadIdx.x & 63] = pre_nrm;
    } else {
      if (threadIdx.x < 2 * kTile) {
        const int side = threadIdx.x >> 6, pt = threadIdx.x & 63;
        const int64_t g = (side ? j0 : i0) + pt;
        nrm[side][pt] = g < n ? norms[g] : 0;
      }
    }
    const Cursor nxt = next_of(cur);
    if constexpr (ahead) {
      tile_regs_store<kRow>(pre, xs, segs1);
      if (nxt.ok) {
        tile_regs_load(pre, x, n, d, (int64_t)nxt.I * kTile, (int64_t)nxt.J * kTile, segs1);
        side_load(nxt);
      }
      __syncthreads();
      // d <= 64: one or two 32-deep products, the first from a zero accumulator.
      const v16i zero = {};
      const v4i a0 = *reinterpret_cast<const v4i*>(&xs[1][jsub * 32 + (lane & 31)][16 * (lane >> 5)]);
      const v4i b0 = *reinterpret_cast<const v4i*>(&xs[0][isub * 32 + (lane & 31)][16 * (lane >> 5)]);
      c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, zero, 0, 0, 0);
      if (segs1 > 2) {
        const v4i a1 =
            *reinterpret_cast<const v4i*>(&xs[1][jsub * 32 + (lane & 31)][32 + 16 * (lane >> 5)]);
        const v4i b1 =
            *reinterpret_cast<const v4i*>(&xs[0][isub * 32 + (lane & 31)][32 + 16 * (lane >> 5)]);
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, c, 0, 0, 0);
      }
    }
    for (int k0 = 0; k0 < (ahead ? 0 : d); k0 += KMAX) {
      const int kc = d - k0 < KMAX ? d - k0 : KMAX;
      const int kpad = (kc + 31) & ~31;
      if (k0 > 0) __syncthreads();
      if (vec16) {
        const int segs = kpad >> 4;  // 16-byte segments per row
        for (int e = threadIdx.x; e < 2 * kTile * segs; e += blockDim.x) {
          const int side = e / (kTile * segs), rem = e - side * kTile * segs;
          const int pt = rem / segs, sg = rem - pt * segs;
          const int64_t g = (side ? j0 : i0) + pt;
          int4 v = make_int4(0, 0, 0, 0);
          if (g < n && 16 * sg < kc) v = *reinterpret_cast<const int4*>(x + g * d + k0 + 16 * sg);
          *reinterpret_cast<int4*>(&xs[side][pt][16 * sg]) = v;
        }
      } else {
        for (int e = threadIdx.x; e < kTile * kpad; e += blockDim.x) {
          const int pt = e / kpad, kk = e - pt * kpad;
          const int64_t gi = i0 + pt, gj = j0 + pt;
          xs[0][pt][kk] = (gi < n && kk < kc) ? x[gi * d + k0 + kk] : (int8_t)0;
          xs[1][pt][kk] = (gj < n && kk < kc) ? x[gj * d + k0 + kk] : (int8_t)0;
        }
      }
      __syncthreads();
      // A = rows j (m = lane % 32), B = rows i (n = lane % 32); each lane
      // supplies 16 consecutive k of its row: k = 16 * (lane / 32) + 0..15.
      for (int kk = 0; kk < kpad; kk += 32) {
        const v4i a = *reinterpret_cast<const v4i*>(
            &xs[1][jsub * 32 + (lane & 31)][kk + 16 * (lane >> 5)]);
        const v4i b = *reinterpret_cast<const v4i*>(
            &xs[0][isub * 32 + (lane & 31)][kk + 16 * (lane >> 5)]);
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
      }
    }
    // D layout of a 32x32 MFMA: lane holds column n = lane % 32 and rows
    // m = 8 * (r / 4) + 4 * (lane / 32) + r % 4 for r = 0..15.  So for one
    // r, each half-wave holds one row j and 32 consecutive i.
    //
    // delta < 2^31 on this path (d <= 32768 int8 coordinates: at most
    // 32768 * 255^2), so it is formed in wrapping 32-bit arithmetic, exact,
    // and compared against the range clamped to 32 bits.  Tiles strictly
    // below the diagonal and inside the cloud need no per-edge validity test.
    const int il = isub * 32 + (lane & 31);
    const int64_t i = i0 + il;
    const uint32_t ni = (uint32_t)nrm[0][il];
    const int half = lane >> 5;
    const int jrow = jsub * 32 + 4 * half;  // row of r = 0; r adds 8 (r / 4) + r % 4
    // delta of accumulator r, from the four row norms of its group r / 4
    auto delta_of = [&](const int4& nj, int r) -> uint32_t {
      const int t = r & 3;
      const int32_t nv = t == 0 ? nj.x : t == 1 ? nj.y : t == 2 ? nj.z : nj.w;
      return (uint32_t)nv + ni - 2u * (uint32_t)c[r];
    };
    const bool interior = j0 >= i0 + kTile && j0 + kTile <= n;
    auto epilogue = [&](auto full_tile) {
      constexpr bool kInterior = decltype(full_tile)::value;
      // Two halves of the accumulators (r < 8, r >= 8: disjoint rows).  The
      // emit pass queues each half's kept keys per wave in LDS (r by r, each
      // r's lower half-wave first, lanes in order), then writes the queue
      // out 64 keys per store, each key at its row's base plus its rank.
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        uint32_t wq = 0;  // emit: this wave's queued keys of this half
        uint32_t pk[8], qs[8];  // packed row counts and queue starts of r = 8 hf + 0..7
#pragma unroll
        for (int qq = 0; qq < 2; ++qq) {
          const int q = 2 * hf + qq;
          const int4 nj = *reinterpret_cast<const int4*>(&nrm[1][jrow + 8 * q]);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int r = 4 * q + t;
            const int jl = jrow + 8 * q + t;
            const int64_t j = j0 + jl;
            const bool valid = kInterior || (j < n && i < j);
            const uint32_t delta = delta_of(nj, r);
            if constexpr (kHist) {
              if (valid) {
                if (MODE == kKeysFull)
                  kp.keys[j * (j - 1) / 2 + i] =
                      ((uint64_t)delta << (2 * ib)) | ((uint64_t)j << ib) | (uint64_t)i;
                atomicAdd(&lh[(uint32_t)((uint64_t)delta >> hs)], 1u);
              }
            } else {
              const bool kept = valid && delta - dlo32 < span32;
              const uint64_t m = __ballot(kept);
              pk[r - 8 * hf] = (uint32_t)__popc((uint32_t)m) |
                               ((uint32_t)__popc((uint32_t)(m >> 32)) << 16);
              qs[r - 8 * hf] = wq;
              if constexpr (MODE == kKeysEmit) {
                if (kept) {
                  const uint32_t at =
                      wq + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                  q_keys[wave][at] = ((uint64_t)delta << 32) | (uint32_t)((r << 6) | lane);
                }
                wq += (uint32_t)__popcll(m);
              }
            }
          }
        }
        if constexpr (!kHist) {
          if (lane == 0) {
            uint4* hp = reinterpret_cast<uint4*>(&hcp[wave][8 * hf]);
            hp[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
            hp[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
            if (MODE == kKeysEmit) {
              uint4* qp = reinterpret_cast<uint4*>(&q_start[wave][8 * hf]);
              qp[0] = make_uint4(qs[0], qs[1], qs[2], qs[3]);
              qp[1] = make_uint4(qs[4], qs[5], qs[6], qs[7]);
            }
          }
        }
        if constexpr (MODE == kKeysEmit) {
          __syncthreads();  // every wave's counts of this half are in LDS
          for (uint32_t e = lane; e < wq; e += 64) {
            const uint64_t qk = q_keys[wave][e];
            const uint32_t meta = (uint32_t)qk;
            const int r = (int)(meta >> 6), ln = (int)(meta & 63), h = ln >> 5;
            const int row0 = jsub * 32 + 8 * (r >> 2) + (r & 3);  // row of r's lower half-wave
            const int jl = row0 + 4 * h;
            // rank among the kept keys of its half-row in this wave
            uint32_t rank = e - q_start[wave][r];
            if (h) rank -= hcp[wave][r] & 0xFFFFu;
            // after the lower i-half's keys of the row (the other wave)
            const uint32_t pos = rbase[jl] + (isub ? row_count(jl, 0) : 0u) + rank;
            const uint64_t jj = (uint64_t)(j0 + jl), ii = (uint64_t)(i0 + isub * 32 + (ln & 31));
            kp.keys[pos] = ((qk >> 32) << (2 * ib)) | (jj << ib) | ii;
          }
        }
      }
      if constexpr (MODE == kKeysCount) {
        __syncthreads();
        if (threadIdx.x < kTile) {
          row_acc = (seg_first ? 0u : row_acc) + row_count(threadIdx.x, 0) +
                    row_count(threadIdx.x, 1);
          if (seg_last) kp.cnt[count_slot(cur, threadIdx.x)] = row_acc;
        }
      }
    };
    if (interior)
      epilogue(std::true_type{});
    else
      epilogue(std::false_type{});
    cur = nxt;
  }
  if (kHist) hist_flush(lh, kp.hist);
}

// Histogram shift from the coordinate ranges (lo[0..d) then hi[0..d)): the
// bit length b of sum_k (hi_k - lo_k)^2 (64 if the sum overflows), then
// max(b - 11, 0), the same rule the host applies to the ranges it reads.
__global__ __launch_bounds__(256) void k_dist_shift(const int32_t* __restrict__ minmax,
                                                    int32_t d, int32_t* shift) {
  __shared__ unsigned long long s_sum;
  __shared__ int s_over;
  if (threadIdx.x == 0) {
    s_sum = 0;
    s_over = 0;
  }
  __syncthreads();
  unsigned long long b = 0;
  int over = 0;
  for (int32_t k = threadIdx.x; k < d; k += blockDim.x) {
    const unsigned long long w = (unsigned long long)((int64_t)minmax[d + k] - minmax[k]);
    const unsigned long long q = w * w;
    over |= b + q < b;
    b += q;
  }
  const unsigned long long before = atomicAdd(&s_sum, b);
  over |= before + b < before;
  if (over) atomicOr(&s_over, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int bits = 64;
    if (!s_over) {
      bits = 0;
      while (bits < 64 && (s_sum >> bits) != 0) ++bits;
    }
    shift[0] = bits > 11 ? bits - 11 : 0;
  }
}

int grid_for(int64_t count, int per_block, int cap) {
  int64_t g = (count + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_gather(const Gather& g, hipStream_t s) {
  if (g.count <= 0) return hipSuccess;
  if (g.count > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather, dim3(g.count), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_coord_range(const void* pts, int elem_bytes, int64_t n, int32_t d,
                              int32_t* minmax, hipStream_t s, int32_t* norms, bool* norms_done,
                              uint32_t* zero, int64_t zero_len) {
  if (norms_done) *norms_done = false;
  if (!zero) zero_len = 0;
  hipLaunchKernelGGL(k_range_init, dim3(grid_for(2 * (int64_t)d + zero_len, 256, 64)), dim3(256),
                     0, s, minmax, d, zero, zero_len);
  const int segs = d / 16;
  if (norms && norms_done && elem_bytes == 1 && n > 0 && d % 16 == 0 && d <= kRangeLds &&
      (segs & (segs - 1)) == 0 && reinterpret_cast<uintptr_t>(pts) % 16 == 0) {
    const int rows = 256 / segs;
    hipLaunchKernelGGL(k_prep_i8, dim3(grid_for(n, 4 * rows, kPrepMaxBlocks)), dim3(256), 0, s,
                       static_cast<const int8_t*>(pts), n, d, minmax, norms);
    *norms_done = true;
  } else if (d <= kRangeLds) {
    const int g = grid_for(n * d, 256 * 16, 1024);
    if (elem_bytes == 1)
      hipLaunchKernelGGL(k_coord_range<int8_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, minmax);
    else
      hipLaunchKernelGGL(k_coord_range<int16_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const int16_t*>(pts), n, d, minmax);
  } else {
    dim3 grid(grid_for(n, 256, 64), d < 256 ? d : 256);
    if (elem_bytes == 1)
      hipLaunchKernelGGL(k_coord_range_wide<int8_t>, grid, dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, minmax);
    else
      hipLaunchKernelGGL(k_coord_range_wide<int16_t>, grid, dim3(256), 0, s,
                         static_cast<const int16_t*>(pts), n, d, minmax);
  }
  return hipGetLastError();
}

int64_t key_count_len(int64_t n, bool mfma) {
  const int64_t nb = (n + kTile - 1) / kTile;
  return 64 * seg_base(nb, mfma ? kSegTiles : 1);
}

// CUs of the current device, read once per device.
int device_cus_cached() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        c <= 0)
      c = 256;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

// Workgroups of 256 threads that one CU holds at once for `kernel` (its
// register and LDS use decide), read once per kernel through `slot`.
int per_cu_blocks(const void* kernel, std::atomic<int>& slot) {
  int b = slot.load(std::memory_order_relaxed);
  if (b <= 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, 256, 0) != hipSuccess || b <= 0)
      b = 1;
    slot.store(b, std::memory_order_relaxed);
  }
  return b;
}

// The grid is what the device holds at once (every workgroup loops over
// tiles, and no second wave of workgroups runs on a partly empty device),
// capped at `cap_per_cu` workgroups per CU and at `visited` tiles.
template <int MODE>
void keys_launch(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib, bool use_mfma,
                 int64_t ntiles, int64_t visited, int cap_per_cu, const KeyPass& kp,
                 hipStream_t s) {
  static std::atomic<int> occ[5];
  const int64_t cus = device_cus_cached();
  auto grid_of = [&](const void* kernel, int which) {
    int64_t g = std::min<int64_t>(per_cu_blocks(kernel, occ[which]), cap_per_cu) * cus;
    if (g > visited) g = visited;
    return dim3((unsigned)(g < 1 ? 1 : g));
  };
  if (use_mfma && elem_bytes == 1) {
    if (MODE != kKeysHist) {  // the MFMA passes hand out count segments
      const int64_t nb = (n + kTile - 1) / kTile;
      visited = seg_base(nb, kSegTiles);
    }
    const bool vec16 = (d % 16) == 0 && (reinterpret_cast<uintptr_t>(pts) % 16) == 0;
    if (!kp.norms_ready)
      hipLaunchKernelGGL(k_norms_i8, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, kp.norms);
    if (d <= 64 && vec16)
      hipLaunchKernelGGL((k_keys_mfma<MODE, 64, true>),
                         grid_of((const void*)k_keys_mfma<MODE, 64, true>, 0), dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, ib, ntiles,
                         (const int32_t*)kp.norms, vec16, kp);
    else if (d <= 64)
      hipLaunchKernelGGL((k_keys_mfma<MODE, 64, false>),
                         grid_of((const void*)k_keys_mfma<MODE, 64, false>, 4), dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, ib, ntiles,
                         (const int32_t*)kp.norms, vec16, kp);
    else
      hipLaunchKernelGGL((k_keys_mfma<MODE, 256, false>),
                         grid_of((const void*)k_keys_mfma<MODE, 256, false>, 1), dim3(256), 0, s,
                         static_cast<const int8_t*>(pts), n, d, ib, ntiles,
                         (const int32_t*)kp.norms, vec16, kp);
  } else if (elem_bytes == 1)
    hipLaunchKernelGGL((k_keys_alu<int8_t, MODE>),
                       grid_of((const void*)k_keys_alu<int8_t, MODE>, 2), dim3(256), 0, s,
                       static_cast<const int8_t*>(pts), n, d, ib, ntiles, kp);
  else
    hipLaunchKernelGGL((k_keys_alu<int16_t, MODE>),
                       grid_of((const void*)k_keys_alu<int16_t, MODE>, 3), dim3(256), 0, s,
                       static_cast<const int16_t*>(pts), n, d, ib, ntiles, kp);
}

hipError_t launch_keys_pass(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib,
                            bool use_mfma, const KeyPass& kp, hipStream_t s) {
  const int64_t nb = (n + kTile - 1) / kTile;
  const int64_t ntiles = nb * (nb + 1) / 2;
  const int64_t sample = kp.mode == kKeysHist ? (kp.sample > 0 ? kp.sample : 1) : 1;
  const int64_t visited = (ntiles + sample - 1) / sample;
  // The sampled histogram pass uses at most two workgroups per CU: every
  // workgroup flushes its LDS histogram (up to kHistBins global atomics on
  // the same kHistBins addresses), so fewer, longer workgroups cost less.
  const int cap = kp.mode == kKeysHist ? 2 : 8;
  KeyPass k = kp;
  k.sample = sample;
  switch (kp.mode) {
    case kKeysFull: keys_launch<kKeysFull>(pts, elem_bytes, n, d, ib, use_mfma, ntiles, visited, cap, k, s); break;
    case kKeysHist: keys_launch<kKeysHist>(pts, elem_bytes, n, d, ib, use_mfma, ntiles, visited, cap, k, s); break;
    case kKeysCount: keys_launch<kKeysCount>(pts, elem_bytes, n, d, ib, use_mfma, ntiles, visited, cap, k, s); break;
    default: keys_launch<kKeysEmit>(pts, elem_bytes, n, d, ib, use_mfma, ntiles, visited, cap, k, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_keys(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib,
                       uint64_t* keys, bool use_mfma, int hist_shift, uint32_t* hist,
                       int32_t* norms, hipStream_t s, const int32_t* hist_shift_dev) {
  KeyPass kp;
  kp.mode = kKeysFull;
  kp.keys = keys;
  kp.hist = hist;
  kp.hist_shift = hist_shift;
  kp.hist_shift_dev = hist_shift_dev;
  kp.norms = norms;
  return launch_keys_pass(pts, elem_bytes, n, d, ib, use_mfma, kp, s);
}

hipError_t launch_dist_shift(const int32_t* minmax, int32_t d, int32_t* shift, hipStream_t s) {
  hipLaunchKernelGGL(k_dist_shift, dim3(1), dim3(256), 0, s, minmax, d, shift);
  return hipGetLastError();
}

}  // namespace ph0
