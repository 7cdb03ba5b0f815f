// rank_emit.hip -- step 3 (dense grades: the 1-based index of an edge's
// distance in the duplicate-free list D, Section 2) over the sorted prefix
// that the reduction used, and step 5 (Section 4: "get the barcode
// interval"): each pivot row r gets the grade of the column stored for it;
// the canonical barcode lists the deaths ascending with the infinite bar last.
//
// The grade of sorted position p is 1 + the number of positions q in 1..p
// where the distance changes; only positions below E_eff are ever needed,
// because no pivot lies beyond the last one.  Grades never decrease with p,
// so listing the pivot positions in order lists the deaths in ascending
// order: the barcode needs a scan, not a sort.
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr int kGroup = 256;  // positions per group (one workgroup pass)
constexpr int64_t kShortScan = 65536;  // group counts scanned by one workgroup per array

// Marks the pivot columns: bit p of the bitmap, and the pivot row of p.
__global__ void k_pivot_marks(const int64_t* __restrict__ killer, int64_t n,
                              uint32_t* __restrict__ bitmap, int32_t* __restrict__ prow,
                              uint32_t* __restrict__ dbv) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = killer[r];
    if (p >= 0) {
      atomicOr(&bitmap[p >> 5], 1u << (p & 31));
      prow[p] = (int32_t)r;
    } else {
      dbv[r] = kInf;  // the essential class
    }
  }
}

// Distance change at sorted position q (q >= 1) and pivot flag.
__device__ inline void position_flags(const uint64_t* __restrict__ k, int64_t q, int64_t count,
                                      int shift, const uint32_t* __restrict__ bitmap,
                                      bool* change, bool* pivot) {
  *change = false;
  *pivot = false;
  if (q < count) {
    *change = q > 0 && (k[q] >> shift) != (k[q - 1] >> shift);
    *pivot = (bitmap[q >> 5] >> (q & 31)) & 1u;
  }
}

__device__ inline uint32_t wave_excl_count(bool f, uint64_t* m_out) {
  const uint64_t m = __ballot(f);
  *m_out = m;
  return (uint32_t)__popcll(m & ((1ull << (threadIdx.x & 63)) - 1ull));
}

// Per group of kGroup positions: the number of distance changes and pivots.
__global__ __launch_bounds__(kGroup) void k_grade_count(const uint64_t* __restrict__ k,
                                                        int64_t count, int shift,
                                                        const uint32_t* __restrict__ bitmap,
                                                        uint32_t* __restrict__ cc,
                                                        uint32_t* __restrict__ cp) {
  __shared__ uint32_t wc[2][kGroup / 64];
  const int64_t ng = (count + kGroup - 1) / kGroup;
  const int wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) cc[ng] = cp[ng] = 0;  // the scans' totals land here
  for (int64_t g = blockIdx.x; g < ng; g += gridDim.x) {
    bool ch, pv;
    position_flags(k, g * kGroup + threadIdx.x, count, shift, bitmap, &ch, &pv);
    const uint64_t mc = __ballot(ch), mp = __ballot(pv);
    if ((threadIdx.x & 63) == 0) {
      wc[0][wave] = (uint32_t)__popcll(mc);
      wc[1][wave] = (uint32_t)__popcll(mp);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      cc[g] = wc[0][0] + wc[0][1] + wc[0][2] + wc[0][3];
      cp[g] = wc[1][0] + wc[1][1] + wc[1][2] + wc[1][3];
    }
    __syncthreads();
  }
}

// With cc / cp scanned (exclusive): the grade of every pivot position, its
// bar (in position order = death order) and its vertex's death.
__global__ __launch_bounds__(kGroup) void k_grade_emit(const uint64_t* __restrict__ k,
                                                       int64_t count, int shift,
                                                       const uint32_t* __restrict__ bitmap,
                                                       const int32_t* __restrict__ prow,
                                                       const uint32_t* __restrict__ cc,
                                                       const uint32_t* __restrict__ cp,
                                                       uint32_t* __restrict__ dbv,
                                                       uint32_t* __restrict__ bars, int64_t n) {
  __shared__ uint32_t wc[2][kGroup / 64];
  const int64_t ng = (count + kGroup - 1) / kGroup;
  const int wave = threadIdx.x >> 6;
  if (bars && blockIdx.x == 0 && threadIdx.x == 0) {  // the essential bar, last
    bars[2 * (n - 1)] = 0u;
    bars[2 * (n - 1) + 1] = kInf;
  }
  for (int64_t g = blockIdx.x; g < ng; g += gridDim.x) {
    const int64_t q = g * kGroup + threadIdx.x;
    bool ch, pv;
    position_flags(k, q, count, shift, bitmap, &ch, &pv);
    uint64_t mc, mp;
    const uint32_t ec = wave_excl_count(ch, &mc), ep = wave_excl_count(pv, &mp);
    if ((threadIdx.x & 63) == 0) {
      wc[0][wave] = (uint32_t)__popcll(mc);
      wc[1][wave] = (uint32_t)__popcll(mp);
    }
    __syncthreads();
    uint32_t bc = 0, bp = 0;
    for (int w = 0; w < wave; ++w) {
      bc += wc[0][w];
      bp += wc[1][w];
    }
    if (pv) {
      const uint32_t grade = 1u + cc[g] + bc + ec + (ch ? 1u : 0u);
      dbv[prow[q]] = grade;
      if (bars) {
        const uint32_t at = cp[g] + bp + ep;
        bars[2 * at] = 0u;
        bars[2 * at + 1] = grade;
      }
    }
    __syncthreads();
  }
}

__global__ void k_pairs_detail(const int64_t* __restrict__ killer,
                               const uint64_t* __restrict__ skeys, int ib,
                               const int32_t* __restrict__ part, int64_t n,
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
      other = part[r];  // the stored column's other row
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

size_t grades_work_bytes(int64_t E_eff) {
  const int64_t ng = (E_eff + kGroup - 1) / kGroup + 1;
  const int64_t words = (E_eff + 31) / 32;
  return 4 * (size_t)E_eff + 4 * (size_t)words + 2 * 4 * (size_t)ng +
         2 * 4 * (size_t)scan_totals_len(ng) + 64;
}

hipError_t launch_grades_and_bars(const uint64_t* skeys, int64_t E_eff, int shift,
                                  const int64_t* killer, int64_t n, void* work, uint32_t* dbv,
                                  uint32_t* bars, hipStream_t s, const uint32_t** distinct,
                                  const uint32_t** pivots) {
  const int64_t ng = (E_eff + kGroup - 1) / kGroup;
  const int64_t words = (E_eff + 31) / 32;
  int32_t* prow = static_cast<int32_t*>(work);
  uint32_t* bitmap = reinterpret_cast<uint32_t*>(prow + E_eff);
  uint32_t* cc = bitmap + words;
  uint32_t* cp = cc + ng + 1;
  uint32_t* tot_c = cp + ng + 1;
  uint32_t* tot_p = tot_c + scan_totals_len(ng + 1);
  hipError_t e = launch_fill_u32(bitmap, 0u, words, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pivot_marks, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, killer, n,
                     bitmap, prow, dbv);
  const int g = grid_for(E_eff, kGroup, 4096);
  hipLaunchKernelGGL(k_grade_count, dim3(g), dim3(kGroup), 0, s, skeys, E_eff, shift, bitmap, cc,
                     cp);
  // The two count arrays are adjacent (cp = cc + ng + 1): short ones are
  // scanned together, one workgroup each; long ones block-wise.
  if (ng + 1 <= kShortScan) {
    if ((e = launch_scan_columns(cc, ng + 1, 2, tot_c, s)) != hipSuccess) return e;
  } else {
    if ((e = launch_scan_u32(cc, ng + 1, tot_c, s)) != hipSuccess) return e;
    if ((e = launch_scan_u32(cp, ng + 1, tot_p, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_grade_emit, dim3(g), dim3(kGroup), 0, s, skeys, E_eff, shift, bitmap,
                     prow, cc, cp, dbv, bars, n);
  *distinct = cc + ng;
  *pivots = cp + ng;
  return hipGetLastError();
}

hipError_t launch_pairs_detail(const int64_t* killer, const uint64_t* skeys, int ib,
                               const int32_t* part, int64_t n,
                               int64_t* killer_pos, uint64_t* killer_edge,
                               int64_t* killer_sqdist, int32_t* partner, hipStream_t s) {
  hipLaunchKernelGGL(k_pairs_detail, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, killer,
                     skeys, ib, part, n, killer_pos, killer_edge, killer_sqdist, partner);
  return hipGetLastError();
}

}  // namespace ph0
