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
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kTile = 64;  // points per tile side; a tile covers 64 x 64 edges

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

template <typename T>
__global__ void k_coord_range(const T* __restrict__ x, int64_t n, int32_t d,
                              int32_t* __restrict__ minmax) {
  // One block per dimension chunk; grid-stride over points.
  for (int k = blockIdx.y; k < d; k += gridDim.y) {
    int lo = 1 << 30, hi = -(1 << 30);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      int v = x[i * d + k];
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
    }
    // One atomic pair per wavefront: per-thread atomics on the same 2d
    // addresses serialize.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const int l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&minmax[2 * k], lo);
      atomicMax(&minmax[2 * k + 1], hi);
    }
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

template <typename T>
__global__ __launch_bounds__(256) void k_keys_alu(const T* __restrict__ x, int64_t n, int32_t d,
                                                  int ib, uint64_t* __restrict__ keys,
                                                  int64_t ntiles, int hist_shift,
                                                  uint32_t* __restrict__ hist) {
  __shared__ int32_t xs[2][kTile][kChunk + 1];
  __shared__ uint32_t lh[kHistBins];
  hist_zero(lh);

  const int il = threadIdx.x & 63;   // i inside the tile (one per lane)
  const int jl0 = threadIdx.x >> 6;  // first j of this wave; j = jl0 + 4q
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
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
      const int64_t j = j0 + jl0 + 4 * q;
      if (j < n && i < j) {
        const uint64_t delta = (uint64_t)acc[q];
        keys[j * (j - 1) / 2 + i] =
            (delta << (2 * ib)) | ((uint64_t)j << ib) | (uint64_t)i;
        atomicAdd(&lh[delta >> hist_shift], 1u);
      }
    }
  }
  hist_flush(lh, hist);
}

// ---- int8 MFMA Gram path ----
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

constexpr int kMaxDpad = 256;  // int8 dims staged per LDS round (multiple of 32)

__global__ __launch_bounds__(256) void k_keys_mfma(const int8_t* __restrict__ x, int64_t n,
                                                   int32_t d, int ib,
                                                   uint64_t* __restrict__ keys,
                                                   int64_t ntiles, int hist_shift,
                                                   uint32_t* __restrict__ hist) {
  // Rows padded by 16 bytes so that the 32 row reads of a half-wave spread
  // over the LDS banks.
  constexpr int kRow = kMaxDpad + 16;
  __shared__ __attribute__((aligned(16))) int8_t xs[2][kTile][kRow];
  __shared__ int32_t nrm[2][kTile];
  __shared__ uint32_t lh[kHistBins];
  hist_zero(lh);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int jsub = wave >> 1, isub = wave & 1;  // 32 x 32 sub-tile of this wave
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int64_t jb, ibk;
    tile_coords(t, &jb, &ibk);
    const int64_t i0 = ibk * kTile, j0 = jb * kTile;
    v16i c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = 0;
    __syncthreads();  // the previous tile's readers of nrm are done
    if (threadIdx.x < 2 * kTile) nrm[threadIdx.x >> 6][threadIdx.x & 63] = 0;
    for (int k0 = 0; k0 < d; k0 += kMaxDpad) {
      const int kc = d - k0 < kMaxDpad ? d - k0 : kMaxDpad;
      const int kpad = (kc + 31) & ~31;
      __syncthreads();
      for (int e = threadIdx.x; e < kTile * kpad; e += blockDim.x) {
        const int pt = e / kpad, kk = e - pt * kpad;
        const int64_t gi = i0 + pt, gj = j0 + pt;
        xs[0][pt][kk] = (gi < n && kk < kc) ? x[gi * d + k0 + kk] : (int8_t)0;
        xs[1][pt][kk] = (gj < n && kk < kc) ? x[gj * d + k0 + kk] : (int8_t)0;
      }
      __syncthreads();
      if (threadIdx.x < 2 * kTile) {
        const int side = threadIdx.x >> 6, pt = threadIdx.x & 63;
        int32_t s = 0;
        for (int kk = 0; kk < kc; ++kk) {
          const int32_t v = xs[side][pt][kk];
          s += v * v;
        }
        nrm[side][pt] += s;
      }
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
    __syncthreads();
    // D layout of a 32x32 MFMA: lane holds column n = lane % 32 and rows
    // m = 8 * (r / 4) + 4 * (lane / 32) + r % 4 for r = 0..15.
    const int il = isub * 32 + (lane & 31);
    const int64_t i = i0 + il;
    const int32_t ni = nrm[0][il];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int jl = jsub * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int64_t j = j0 + jl;
      if (j < n && i < j) {
        const uint64_t delta = (uint64_t)(int64_t)(nrm[1][jl] + ni - 2 * c[r]);
        keys[j * (j - 1) / 2 + i] =
            (delta << (2 * ib)) | ((uint64_t)j << ib) | (uint64_t)i;
        atomicAdd(&lh[delta >> hist_shift], 1u);
      }
    }
  }
  hist_flush(lh, hist);
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

hipError_t launch_coord_range(const void* pts, int elem_bytes, int64_t n, int32_t d,
                              int32_t* minmax, hipStream_t s) {
  dim3 grid(grid_for(n, 256, 64), d < 256 ? d : 256);
  if (elem_bytes == 1)
    hipLaunchKernelGGL(k_coord_range<int8_t>, grid, dim3(256), 0, s,
                       static_cast<const int8_t*>(pts), n, d, minmax);
  else
    hipLaunchKernelGGL(k_coord_range<int16_t>, grid, dim3(256), 0, s,
                       static_cast<const int16_t*>(pts), n, d, minmax);
  return hipGetLastError();
}

hipError_t launch_keys(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib,
                       uint64_t* keys, bool use_mfma, int hist_shift, uint32_t* hist,
                       hipStream_t s) {
  const int64_t nb = (n + kTile - 1) / kTile;
  const int64_t ntiles = nb * (nb + 1) / 2;
  // Resident-sized grid: each workgroup loops over tiles, so its histogram
  // is flushed once.
  int cus = 256;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  const int64_t cap = 8 * (int64_t)cus;
  const int grid = (int)(ntiles < cap ? ntiles : cap);
  if (use_mfma && elem_bytes == 1) {
    hipLaunchKernelGGL(k_keys_mfma, dim3(grid), dim3(256), 0, s,
                       static_cast<const int8_t*>(pts), n, d, ib, keys, ntiles, hist_shift, hist);
  } else if (elem_bytes == 1) {
    hipLaunchKernelGGL(k_keys_alu<int8_t>, dim3(grid), dim3(256), 0, s,
                       static_cast<const int8_t*>(pts), n, d, ib, keys, ntiles, hist_shift, hist);
  } else {
    hipLaunchKernelGGL(k_keys_alu<int16_t>, dim3(grid), dim3(256), 0, s,
                       static_cast<const int16_t*>(pts), n, d, ib, keys, ntiles, hist_shift, hist);
  }
  return hipGetLastError();
}

}  // namespace ph0
