// reduce.hip -- steps 4-5 of the GPU pipeline (Section 4: "for each diagonal
// entry of the matrix: reduction step"): column reduction over F2 of the
// vertex-by-edge boundary matrix, left to right, with pivots (Section 2).
//
// Data layout.  The pivot table holds, for each row r, the reduced column
// stored with low r.  Every column of the vertex-by-edge boundary matrix
// stays 2-sparse under F2 column additions: a reduced column has nonzero rows
// {a, r}, a < r, and adding the stored column {x, r} of row r cancels row r
// and leaves {a, x} (nothing when x = a).  A stored column is therefore fully
// described by its other row x, and the table is part[r] = x, or -1 while
// row r is free: N 4-byte entries (64 KB at N = 16384, resident in the
// caches) instead of N dense N-bit rows.  Every addition is still exactly
// the one the sequential dense reduction makes -- the same pivots, the same
// stored columns, the same count -- only its representation is sparse; the
// oracle reduces dense bitset columns and the results agree bit for bit.
//
// The walk gives each column one lane: a chain of dependent table loads
// (x = part[r]), 64 independent chains per wavefront.  For n <= 32768 each
// walk workgroup first copies a 16-bit mirror of the table (part16, kept in
// step with part by the commit step; 32 KB at n = 16384) into its LDS, so
// every step of a chain is an LDS load rather than an L2 round trip, and the
// walk runs 1024-lane workgroups, two per compute unit (full occupancy).

// Rounds.  A window of consecutive sorted columns [F, Wend) is reduced side
// by side against the table as committed so far (every slot there belongs to
// an earlier column, so each step is one the sequential reduction also
// takes).  A column that stops on an empty slot r is a survivor with low r.
// The sequential order is then restored exactly:
//   * survivors before the first survivor whose low repeats an earlier
//     survivor's low commit (none of them would have met another's slot);
//   * a later survivor also commits if no earlier survivor touches the
//     component of its low r -- no earlier survivor has low r, and none has
//     r as the root of its other row: then no earlier column can take slot r
//     first, and its walk is final;
//   * every other survivor stays and continues next round against the
//     grown table.
// The result -- every stored column, every pivot, the number of additions
// -- equals the sequential left-to-right reduction.  Once N-1 pivots exist
// the remaining columns must reduce to zero (the complete graph is
// connected), so the reduction stops there.
//
// A round is two launches -- walk, commit -- and its control uses no atomic
// on a shared address (on MI355X same-address atomics from hundreds of
// workgroups serialize, and a grid-wide barrier costs several times a
// launch):
//   * the first wave of every walk workgroup reduces the previous commit's
//     slots into the state entering this round (the same in each;
//     workgroup 0 stores it, into the other of two state copies, for the
//     commit and the next round), with the offsets of the kept segments in
//     its LDS;
//   * the walk also finds the first survivor whose low repeats an earlier
//     one: within a workgroup from its LDS hash of row minima, across
//     workgroups from the values the row-minimum atomics return; each
//     workgroup leaves its candidate in a slot of its own;
//   * the commit workgroup of a walk workgroup's survivors commits or keeps
//     them, writes the kept ones (with their state) to a segment of its own
//     and its totals to a slot of its own.
// Where the host looks at the state (the end of a burst of rounds), one
// wave advances it on its own and leaves a copy in host memory.
#include <algorithm>

#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr uint64_t kNoValue = ~0ull;
constexpr uint16_t kFree16 = 0xFFFF;  // a free row in the 16-bit table mirror
constexpr int kWalkThreads = 1024;
constexpr int kWalkWaves = kWalkThreads / 64;
constexpr int kCommitThreads = 256;
static_assert(kCommitThreads <= kWalkThreads, "a commit pass fits one walk segment");
constexpr int kHashBits = 11;  // log2 of the LDS hash slots (2 x kWalkThreads)

// Row minima carry the round in their top bits, so that a value left by an
// earlier round is larger than any of this round's and never matches.
constexpr int kPosBits = 40;
__device__ inline uint64_t enc(int64_t round, int64_t p) {
  return ((uint64_t)(0xFFFFFF - (round & 0xFFFFFF)) << kPosBits) | (uint64_t)p;
}
__device__ inline bool same_round(uint64_t v, int64_t round) {
  return (v >> kPosBits) == (uint64_t)(0xFFFFFF - (round & 0xFFFFFF));
}
__device__ inline int64_t enc_pos(uint64_t v) {
  return (int64_t)(v & ((1ull << kPosBits) - 1ull));
}

__device__ inline uint64_t shfl64_down(uint64_t v, int delta) {
  const uint32_t lo = __shfl_down((uint32_t)v, delta, 64);
  const uint32_t hi = __shfl_down((uint32_t)(v >> 32), delta, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl64_up(uint64_t v, int delta) {
  const uint32_t lo = __shfl_up((uint32_t)v, delta, 64);
  const uint32_t hi = __shfl_up((uint32_t)(v >> 32), delta, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl64_idx(uint64_t v, int src) {
  const uint32_t lo = __shfl((uint32_t)v, src, 64);
  const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = shfl64_down(v, o);
    v = w < v ? w : v;
  }
  return v;
}

__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = shfl64_down(v, o);
    v = w > v ? w : v;
  }
  return v;
}

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = __shfl_down(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t w = __shfl_down(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (int64_t)shfl64_down((uint64_t)v, o);
  return v;
}

// Block-wide reductions and scans; `tmp` holds one entry per wave.  Every
// thread of the block must call them (they synchronize).
template <int kWaves>
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t* tmp) {
  v = wave_min_u64(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = tmp[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) r = tmp[w] < r ? tmp[w] : r;
  __syncthreads();
  return r;
}

template <int kWaves>
__device__ inline uint64_t block_max_u64(uint64_t v, uint64_t* tmp) {
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = tmp[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) r = tmp[w] > r ? tmp[w] : r;
  __syncthreads();
  return r;
}

template <int kWaves>
__device__ inline int64_t block_sum_i64(int64_t v, int64_t* tmp) {
  v = wave_sum_i64(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t r = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) r += tmp[w];
  __syncthreads();
  return r;
}

// Exclusive prefix of v over the block, and the block total.
template <int kWaves>
__device__ inline int64_t block_excl_i64(int64_t v, int64_t* tmp, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = (int64_t)shfl64_up((uint64_t)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  int64_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    base += w < wave ? tmp[w] : 0;
    all += tmp[w];
  }
  *total = all;
  __syncthreads();
  return base + x - v;
}

// The fields of a round state the walk uses.
struct RoundView {
  int64_t nA, round, fresh_lo, fresh_hi, F;
  int32_t done, need_more;
};

// The view held in scalar registers (the values are the same in every lane).
__device__ inline int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline RoundView uniform_view(RoundView v) {
  v.nA = uniform64(v.nA);
  v.round = uniform64(v.round);
  v.fresh_lo = uniform64(v.fresh_lo);
  v.fresh_hi = uniform64(v.fresh_hi);
  v.F = uniform64(v.F);
  v.done = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v.done);
  v.need_more = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v.need_more);
  return v;
}

// The state entering the next round, formed by one wave (lane l reduces
// the commit slots 8l .. 8l + 7 of the round just committed: pivots,
// columns kept, end of the last pivot, first kept column) from the state
// `c` entering that round; stored to `out` and `publish` when given.
// pre[0..nblocks] (LDS) receives the kept columns before each commit
// segment and their total.  With `compute` false, `c` is the state already
// (only pre is formed).  A state that is done or waits for more columns
// carries over unchanged.  The window start moves to the first column that
// is not final; the window end never moves back; the width doubles (up to
// the ring's capacity) while almost every column of a round becomes final
// and halves (down to the base width) when many stay.  Every lane gets the
// same view back.
__device__ RoundView advance_wave(const RedArgs& A, const RedCtl* c, bool compute, RedCtl* out,
                                  RedCtl* publish, int64_t* pre) {
  constexpr int kWords = (int)(sizeof(RedCtl) / 8);
  static_assert(sizeof(RedCtl) % 8 == 0 && kWords <= 64, "the state is one 8-byte word per lane");
  constexpr int kPer = kMaxWalkBlocks / 64;
  const int lane = threadIdx.x & 63;
  const int nb = A.nblocks;
  // Everything read is requested at once (one memory round trip): lane w
  // holds word w of the state, each lane the commit slots it reduces, and
  // the walk error word.  Loads and reductions run whatever the state says
  // (selects, no branches), so that no load is moved behind a wait.
  const uint64_t word = reinterpret_cast<const uint64_t*>(c)[lane < kWords ? lane : 0];
  const int32_t werr = __hip_atomic_load(A.werr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint4* slots = reinterpret_cast<const uint4*>(A.cslot);
  uint4 sl[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int b = lane * kPer + q;
    sl[q] = slots[b < nb ? b : 0];
  }
  uint32_t kept[kPer];
  int64_t piv = 0, lane_kept = 0;
  uint32_t end_off = 0, stay_off = ~0u;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const bool ok = lane * kPer + q < nb;
    kept[q] = ok ? sl[q].y : 0u;
    lane_kept += kept[q];
    piv += ok ? sl[q].x : 0u;
    const uint32_t eq = ok ? sl[q].z : 0u;
    const uint32_t sq = ok ? sl[q].w : ~0u;
    end_off = eq > end_off ? eq : end_off;
    stay_off = sq < stay_off ? sq : stay_off;
  }
  // Fields of the state, the same in every lane: an 8-byte one, and a
  // 4-byte one (either half of a word).
  auto word_at = [&](size_t off) -> uint64_t {
    const int w = (int)(off / 8);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)word, w);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(word >> 32), w);
    return ((uint64_t)hi << 32) | lo;
  };
  auto field = [&](size_t off) -> int64_t { return (int64_t)word_at(off); };
  auto field32 = [&](size_t off) -> int32_t {
    return (int32_t)(uint32_t)(word_at(off) >> (8 * (off % 8)));
  };
  static_assert(offsetof(RedCtl, done) % 8 == 0 && offsetof(RedCtl, err) == offsetof(RedCtl, done) + 4 &&
                    offsetof(RedCtl, need_more) % 8 == 0,
                "done and err share a word, need_more starts one");
  int64_t incl = lane_kept;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = (int64_t)shfl64_up((uint64_t)incl, o);
    if (lane >= o) incl += y;
  }
  piv = uniform64(wave_sum_i64(piv));
  end_off = __builtin_amdgcn_readfirstlane(wave_max_u32(end_off));
  stay_off = __builtin_amdgcn_readfirstlane(wave_min_u32(stay_off));
  RoundView cv;
  cv.nA = field(offsetof(RedCtl, nA));
  cv.round = field(offsetof(RedCtl, round));
  cv.fresh_lo = field(offsetof(RedCtl, fresh_lo));
  cv.fresh_hi = field(offsetof(RedCtl, fresh_hi));
  cv.F = field(offsetof(RedCtl, F));
  cv.done = field32(offsetof(RedCtl, done));
  cv.need_more = field32(offsetof(RedCtl, need_more));
  if (cv.done || cv.need_more) {
    if (compute && lane < kWords) {
      if (out) reinterpret_cast<uint64_t*>(out)[lane] = word;
      if (publish) reinterpret_cast<uint64_t*>(publish)[lane] = word;
    }
    return cv;
  }
  if (!compute && cv.nA == 0) return cv;  // no kept columns to place
  int64_t run = incl - lane_kept;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int b = lane * kPer + q;
    if (b < nb) pre[b] = run;
    run += kept[q];
  }
  const int64_t all_kept = uniform64((int64_t)shfl64_idx((uint64_t)incl, 63));
  if (lane == 0) pre[nb] = all_kept;
  if (!compute) return cv;
  const int64_t n = A.n, E = A.E, Wcap = A.Wcap;
  const int64_t c_Wend = field(offsetof(RedCtl, Wend));
  const int64_t c_E_eff = field(offsetof(RedCtl, E_eff));
  const int64_t pivots = field(offsetof(RedCtl, pivots)) + piv;
  const int64_t end = end_off ? cv.F + (int64_t)end_off : 0;
  const int64_t E_eff = end > c_E_eff ? end : c_E_eff;
  const int64_t F = stay_off == ~0u ? c_Wend : cv.F + (int64_t)stay_off;
  int64_t Wend = c_Wend, width = field(offsetof(RedCtl, width));
  int32_t done = 0, need_more = 0;
  int32_t err = field32(offsetof(RedCtl, err)) | werr;
  if (pivots >= n - 1) {
    // Every later column reduces to zero; only columns before the last
    // pivot still need finishing (for the exact addition count).
    if (F >= E_eff) done = 1;
  } else {
    const int64_t lim = field(offsetof(RedCtl, E_lim));
    const int64_t width_min = field(offsetof(RedCtl, width_min));
    if (all_kept < width / 256)
      width = 2 * width < Wcap ? 2 * width : Wcap;
    else if (all_kept > width / 16)
      width = width / 2 > width_min ? width / 2 : width_min;
    const int64_t want = F + width < lim ? F + width : lim;
    Wend = want > Wend ? want : Wend;
    if (F >= lim) {
      if (lim < E) {
        need_more = 1;  // the host sorts the next distance range
      } else {
        done = 1;
        err |= 2;
      }
    }
  }
  RoundView v;
  v.nA = all_kept;
  v.round = cv.round + 1;
  v.fresh_lo = c_Wend;
  v.fresh_hi = Wend;
  v.F = F;
  v.done = done;
  v.need_more = need_more;
  if (out || publish) {
    // The new state, word w from lane w: the fields the advance sets
    // replace the old ones, the rest carry over.
    const int64_t c_maxWend = field(offsetof(RedCtl, maxWend));
    const int64_t maxWend = Wend > c_maxWend ? Wend : c_maxWend;
    auto at = [&](size_t off) { return lane == (int)(off / 8); };
    uint64_t o = word;
    if (at(offsetof(RedCtl, F))) o = (uint64_t)F;
    if (at(offsetof(RedCtl, Wend))) o = (uint64_t)Wend;
    if (at(offsetof(RedCtl, width))) o = (uint64_t)width;
    if (at(offsetof(RedCtl, maxWend))) o = (uint64_t)maxWend;
    if (at(offsetof(RedCtl, fresh_lo))) o = (uint64_t)v.fresh_lo;
    if (at(offsetof(RedCtl, fresh_hi))) o = (uint64_t)v.fresh_hi;
    if (at(offsetof(RedCtl, nA))) o = (uint64_t)v.nA;
    if (at(offsetof(RedCtl, pivots))) o = (uint64_t)pivots;
    if (at(offsetof(RedCtl, E_eff))) o = (uint64_t)E_eff;
    if (at(offsetof(RedCtl, round))) o = (uint64_t)v.round;
    if (at(offsetof(RedCtl, done))) o = ((uint64_t)(uint32_t)err << 32) | (uint32_t)done;
    if (at(offsetof(RedCtl, need_more)))
      o = (o & 0xFFFFFFFF00000000ull) | (uint32_t)need_more;
    if (lane < kWords) {
      if (out) reinterpret_cast<uint64_t*>(out)[lane] = o;
      if (publish) reinterpret_cast<uint64_t*>(publish)[lane] = o;
    }
  }
  return v;
}

// Per-workgroup aggregation of the survivors' row minima.  Survivors of one
// row are many (up to 2e5 on the root of a large component when clusters
// merge) and same-address global atomics serialize, while spreading them
// over random rows makes each one a separate memory transaction.  So the
// lanes of a walk workgroup first meet in an LDS hash table keyed by row
// (open addressing, kHashSlots >= 2 x the lanes of one pass, so an insert
// always finds a slot); the value is the smallest position offset p - F.
// Only the lane holding the row's minimum then lowers the global entry:
// one global atomic per (workgroup, pass, row).
constexpr int kHashSlots = 2 * kWalkThreads;
constexpr uint32_t kHashEmpty = 0, kRelNone = 0xFFFFFFFFu;
static_assert(kHashSlots == 1 << kHashBits, "hash slots must be 2^kHashBits");

__device__ inline int hash_insert(uint32_t* keys, uint32_t* vals, int row, uint32_t rel) {
  const uint32_t key = (uint32_t)row + 1u;
  uint32_t h = (key * 0x9E3779B1u) >> (32 - kHashBits);
  while (true) {
    const uint32_t prev = atomicCAS(&keys[h], kHashEmpty, key);
    if (prev == kHashEmpty || prev == key) {
      atomicMin(&vals[h], rel);
      return (int)h;
    }
    h = (h + 1) & (kHashSlots - 1);
  }
}

// One round's walk.  Every item -- a column kept by the previous commit
// (listed in the commit workgroups' segments, in workgroup order) or a
// fresh column of the window -- is reduced against the table as committed
// so far, one lane per column.  A column stops on a free row (a survivor) or
// becomes zero.  For a survivor {a, r} the root of a in the pivot forest
// (follow part[] down to a free row) is found, and the round-tagged minima
// for row r (lowc) and that root (touch) are lowered.  Every walked column
// leaves its addition count in the ring (for the overshoot sum).  Each
// workgroup lists its survivors, with their rows, root and addition count,
// in its own segment of `surv` (the commit passes the kept ones on to the
// next walk the same way), and leaves in fdslot[block] the smallest
// survivor it saw whose low repeats an earlier survivor's low.
// kLds: the table is read from the workgroup's LDS copy of part16 (0xFFFF =
// free), else from part in global memory.
template <bool kLds>
__global__ __launch_bounds__(kWalkThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_walk(RedArgs A, int64_t n16, int64_t k, int advanced) {
  extern __shared__ uint4 s_tab4[];  // kLds: n16 / 8 entries of 8 table rows
  __shared__ uint32_t s_wave[kWalkWaves];
  __shared__ int64_t s_view[6];
  __shared__ uint64_t s_red[kWalkWaves][4];
  __shared__ int64_t s_pre[kMaxWalkBlocks + 1];  // kept columns before each commit segment
  // Row-minimum hash tables: [0] by low r (lowc), [1] by root rlo (touch).
  __shared__ uint32_t s_hkey[2][kHashSlots];
  __shared__ uint32_t s_hval[2][kHashSlots];
  const int nb = (int)gridDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // The state entering this round: advanced here past round k - 1 by the
  // first wave (every workgroup forms the same; workgroup 0 stores it for
  // the commit and the next round), or already advanced.  A state that is
  // done or waits for more columns carries over unchanged, and the round
  // does nothing.  The first wave also places the previous commit's kept
  // columns (s_pre).
  if (wave == 0) {
    const RoundView v =
        advance_wave(A, A.ctl + ((advanced ? k : k - 1) & 1), !advanced,
                     !advanced && blockIdx.x == 0 ? A.ctl + (k & 1) : nullptr, nullptr, s_pre);
    if (lane == 0) {
      s_view[0] = v.nA;
      s_view[1] = v.round;
      s_view[2] = v.fresh_lo;
      s_view[3] = v.fresh_hi;
      s_view[4] = v.F;
      s_view[5] = (int64_t)(v.done | (v.need_more << 1));
    }
  } else {
    // Meanwhile the other waves empty the hash tables and copy the table
    // (the previous commit's, read-only in this round) into LDS.
    const int t2 = tid - 64;
    constexpr int kOthers = kWalkThreads - 64;
    for (int h = t2; h < kHashSlots; h += kOthers) {
      s_hkey[0][h] = s_hkey[1][h] = kHashEmpty;
      s_hval[0][h] = s_hval[1][h] = kRelNone;
    }
    if (kLds) {
      // Four 16-byte pieces in flight per thread.
      const uint4* src = reinterpret_cast<const uint4*>(A.part16);
      const int64_t pieces = n16 / 8;
      for (int64_t h0 = t2; h0 < pieces; h0 += 4 * kOthers) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t h = h0 + u * kOthers;
          v[u] = src[h < pieces ? h : 0];
        }
        // A piece past the end rewrites piece 0 with its own value (the
        // store is unconditional so that the loads are not moved after a
        // branch, one wait each).
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t h = h0 + u * kOthers;
          s_tab4[h < pieces ? h : 0] = v[u];
        }
      }
    }
  }
  __syncthreads();
  RoundView c;
  c.nA = s_view[0];
  c.round = s_view[1];
  c.fresh_lo = s_view[2];
  c.fresh_hi = s_view[3];
  c.F = s_view[4];
  c.done = (int32_t)(s_view[5] & 1);
  c.need_more = (int32_t)(s_view[5] >> 1);
  c = uniform_view(c);
  if (c.done || c.need_more) return;  // the commit returns too
  const int64_t nA = c.nA, round = c.round, fresh_lo = c.fresh_lo, F = c.F;
  const int64_t items = nA + (c.fresh_hi - fresh_lo);
  int64_t* my_surv = A.surv + blockIdx.x * A.seg;
  uint64_t* my_ra = A.surv_ra + blockIdx.x * A.seg;
  uint64_t* my_x = A.surv_x + blockIdx.x * A.seg;
  if ((int64_t)blockIdx.x * kWalkThreads >= items) {  // nothing for this block
    if (tid == 0) {
      A.scount[blockIdx.x] = 0;
      A.fdslot[blockIdx.x] = kNoValue;
    }
    return;
  }
  const uint16_t* s_tab = reinterpret_cast<const uint16_t*>(s_tab4);
  const int32_t* __restrict__ part = A.part;
  auto lookup = [&](int row) -> int {
    if (kLds) {
      const uint16_t v = s_tab[row];
      return v == kFree16 ? -1 : (int)v;
    }
    return part[row];
  };
  // The previous commit's segments: kept columns and their states.
  const int64_t* kept_cols = A.act[(round - 1) & 1];
  const uint64_t* kept_ra = A.act_ra[(round - 1) & 1];
  const uint64_t* kept_x = A.act_x[(round - 1) & 1];
  const uint64_t* __restrict__ skeys = A.skeys;
  const int ib = A.ib;
  const Ring ring = A.ring;
  const int64_t Wcap = A.Wcap, seg = A.seg;
  const int64_t stride = (int64_t)gridDim.x * kWalkThreads;
  const uint64_t imask = (1ull << ib) - 1ull;
  uint32_t nsurv = 0;  // this block's survivors so far (same in every thread)
  uint32_t adds = 0, finds = 0, words = 0;  // this lane's counts (a few columns' chains)
  uint64_t fd = kNoValue;  // smallest repeated-low survivor seen by this lane
  int32_t bad = 0;
  for (int64_t t0 = blockIdx.x * (int64_t)kWalkThreads; t0 < items; t0 += stride) {
    const int64_t t = t0 + tid;
    bool survivor = false;
    int64_t p = 0;
    int32_t a = 0, r = 0, rlo = 0, steps = 0;
    int hs_low = 0, hs_root = 0;  // this survivor's hash slots
    if (t < items) {
      int32_t prev_steps;
      if (t < nA) {
        // The segment holding kept column t: the last sg with s_pre[sg] <= t.
        int lo = 0, hi = nb;  // s_pre[lo] <= t < s_pre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] <= t)
            lo = mid;
          else
            hi = mid;
        }
        const int64_t at = lo * seg + (t - s_pre[lo]);
        p = kept_cols[at];
        const uint64_t ra = kept_ra[at], x = kept_x[at];
        r = (int32_t)(ra >> 32);
        a = (int32_t)(uint32_t)ra;
        rlo = (int32_t)(x >> 32);
        prev_steps = (int32_t)(uint32_t)x;
      } else {
        p = fresh_lo + (t - nA);
        const uint64_t key = skeys[p];
        a = (int32_t)(key & imask);
        r = (int32_t)((key >> ib) & imask);
        rlo = a;
        prev_steps = 0;
      }
      int moved = 0;
      bool zero = false;
      while (true) {
        const int x = lookup(r);
        ++words;
        if (x < 0) break;  // row r is free
        ++moved;
        if (x == a) {  // {a, r} + {a, r} = 0
          zero = true;
          break;
        }
        if (x >= r) {  // a stored row lies below its low; a corrupt table ends the walk
          bad = 1;
          zero = true;
          break;
        }
        // {a, r} + {x, r} = {a, x}
        const int lo2 = x < a ? x : a;
        r = x < a ? a : x;
        a = lo2;
      }
      adds += moved;
      steps = prev_steps + moved;
      const int64_t kk = p & (Wcap - 1);
      if (zero) {
        ring.st[kk] = kZero | (steps << 2);
      } else {
        // Root of row a in the current forest: follow stored columns down.
        int v = moved ? a : rlo;
        while (true) {
          const int c = lookup(v);
          ++words;
          if (c < 0) break;  // free row: v is a root
          ++finds;
          if (c >= v) {
            bad = 1;
            break;
          }
          v = c;
        }
        rlo = v;
        const uint32_t rel = (uint32_t)(p - F);
        hs_low = hash_insert(s_hkey[0], s_hval[0], r, rel);
        hs_root = hash_insert(s_hkey[1], s_hval[1], rlo, rel);
        survivor = true;
        ring.st[kk] = kActive | (steps << 2);
      }
    }
    // Append this pass's survivors to the block's segment; the lane holding
    // a row's smallest position lowers that row's global minimum.
    const uint64_t m = __ballot(survivor);
    if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    if (survivor) {
      const uint32_t rel = (uint32_t)(p - F);
      const uint64_t e = enc(round, p);
      if (s_hval[0][hs_low] == rel) {
        // Across workgroups: of two survivors on one row, the later one is a
        // repeat; the value the atomic returns names every such pair with
        // the row's second-smallest survivor among them.
        const uint64_t old = atomicMin((unsigned long long*)&A.lowc[r], e);
        if (same_round(old, round)) {
          const uint64_t later = old > e ? old : e;
          fd = (uint64_t)enc_pos(later) < fd ? (uint64_t)enc_pos(later) : fd;
        }
      } else {
        fd = (uint64_t)p < fd ? (uint64_t)p : fd;  // an earlier survivor here has low r
      }
      if (s_hval[1][hs_root] == rel) atomicMin((unsigned long long*)&A.touch[rlo], e);
    }
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWalkWaves; ++w) {
      before += w < wave ? s_wave[w] : 0u;
      total += s_wave[w];
    }
    if (survivor) {
      const uint32_t at = nsurv + before + __popcll(m & ((1ull << lane) - 1ull));
      my_surv[at] = p;
      my_ra[at] = ((uint64_t)(uint32_t)r << 32) | (uint32_t)a;
      my_x[at] = ((uint64_t)(uint32_t)rlo << 32) | (uint32_t)steps;
    }
    nsurv += total;
    __syncthreads();
    if (survivor) {  // empty the slots for the next pass (every used slot has a survivor)
      s_hkey[0][hs_low] = kHashEmpty;
      s_hval[0][hs_low] = kRelNone;
      s_hkey[1][hs_root] = kHashEmpty;
      s_hval[1][hs_root] = kRelNone;
    }
    __syncthreads();
  }
  // One block reduction, one barrier: the smallest repeat, a corrupt-table
  // flag and (when counting) the counters, per wave into LDS, then summed
  // by the first thread into the block's own slots (the grid is the same
  // every round; the counter slots are summed once at the finish).
  fd = wave_min_u64(fd);
  const uint64_t wbad = __ballot(bad != 0);
  uint64_t wadds = 0, wfinds = 0, wwords = 0;
  if (A.count) {
    wadds = (uint64_t)wave_sum_i64(adds);
    wfinds = (uint64_t)wave_sum_i64(finds);
    wwords = (uint64_t)wave_sum_i64(words);
  }
  if (lane == 0) {
    s_red[wave][0] = fd;
    s_red[wave][1] = wadds;
    s_red[wave][2] = wfinds;
    s_red[wave][3] = wwords | (wbad ? 1ull << 63 : 0ull);
  }
  __syncthreads();
  if (wave == 0) {  // lane w takes wave w's entry
    const bool has = lane < kWalkWaves;
    const uint64_t m = wave_min_u64(has ? s_red[lane][0] : kNoValue);
    const uint64_t w3 = has ? s_red[lane][3] : 0ull;
    const bool anybad = __ballot(w3 >> 63) != 0;
    uint64_t c0 = 0, c1 = 0, c2 = 0;
    if (A.count) {
      c0 = (uint64_t)wave_sum_i64(has ? (int64_t)s_red[lane][1] : 0);
      c1 = (uint64_t)wave_sum_i64(has ? (int64_t)s_red[lane][2] : 0);
      c2 = (uint64_t)wave_sum_i64((int64_t)(w3 & ~(1ull << 63)));
    }
    if (lane == 0) {
      A.scount[blockIdx.x] = nsurv;
      A.fdslot[blockIdx.x] = m;
      if (A.count) {
        uint64_t* mine = A.wstat + 3 * (int64_t)blockIdx.x;
        atomicAdd((unsigned long long*)&mine[0], c0);  // no value returned: no wait
        atomicAdd((unsigned long long*)&mine[1], c1);
        atomicAdd((unsigned long long*)&mine[2], c2);
      }
      if (anybad) atomicOr(A.werr, 1);
    }
  }
}

// Commit, one workgroup per walk workgroup, over that workgroup's survivors:
// a survivor commits if it precedes the round's first repeated low (the
// smallest of the walk's slots) or is the first survivor on its row and no
// earlier survivor has that row as its root; the others are kept, in this
// workgroup's own segment of the next list.  The slot gets the pivots
// committed, the end of the last one, the first column kept and the number
// kept.
__global__ __launch_bounds__(kCommitThreads) void k_commit(RedArgs A, int64_t k) {
  constexpr int kWaves = kCommitThreads / 64;
  __shared__ uint64_t s_fd[kWaves];
  __shared__ uint64_t s_tot[kWaves][3];
  __shared__ int64_t itmp[kWaves];
  const int tid = threadIdx.x;
  const int nb = (int)gridDim.x;
  // Slot: pivots, columns kept, and as offsets from F the end of the last
  // pivot (0: none) and the first kept column (~0u: none).
  uint4* slot = reinterpret_cast<uint4*>(A.cslot) + blockIdx.x;
  const RedCtl* ctl = A.ctl + (k & 1);  // the state the walk of this round used
  const int64_t my0 = blockIdx.x * A.seg;
  const int64_t* my = A.surv + my0;
  const uint64_t* my_ra = A.surv_ra + my0;
  const uint64_t* my_x = A.surv_x + my0;
  // A survivor's inputs: its position, rows and state (from the walk), then
  // its rows' minima.  The first pass's list entries (a segment holds at
  // least kCommitThreads) and the walk slots are requested with the state,
  // before the survivor count is known.
  struct Item {
    int64_t p;
    uint64_t ra, x, lc, tc;
  };
  Item it;
  it.p = my[tid];
  it.ra = my_ra[tid];
  it.x = my_x[tid];
  static_assert(kMaxWalkBlocks <= 2 * kCommitThreads, "two walk slots per thread");
  const uint64_t fd0 = A.fdslot[tid < nb ? tid : 0];
  const uint64_t fd1 = A.fdslot[tid + kCommitThreads < nb ? tid + kCommitThreads : 0];
  const int32_t done = ctl->done, need_more = ctl->need_more;
  const int64_t round = ctl->round, F = ctl->F;
  const uint32_t cnt = A.scount[blockIdx.x];
  // All of the above arrive together: a branch on the first would
  // otherwise hold back the loads of the others.
  asm volatile("" ::"s"(done), "s"(need_more), "s"(round), "s"(F), "s"(cnt));
  uint64_t fd = tid < nb ? fd0 : kNoValue;
  fd = tid + kCommitThreads < nb && fd1 < fd ? fd1 : fd;
  if (done | need_more) return;
  if (cnt == 0) {
    if (tid == 0) *slot = make_uint4(0u, 0u, 0u, ~0u);
    return;
  }
  int64_t* kept_out = A.act[round & 1] + my0;
  uint64_t* kept_ra = A.act_ra[round & 1] + my0;
  uint64_t* kept_x = A.act_x[round & 1] + my0;
  auto minima = [&](uint32_t i, Item& t) {
    t.lc = kNoValue;
    t.tc = kNoValue;
    if (i < cnt) {
      const int32_t r = (int32_t)(t.ra >> 32);
      t.lc = A.lowc[r];
      t.tc = A.touch[r];
    }
  };
  auto load = [&](uint32_t i) -> Item {
    Item t = {0, 0, 0, kNoValue, kNoValue};
    if (i < cnt) {
      t.p = my[i];
      t.ra = my_ra[i];
      t.x = my_x[i];
    }
    minima(i, t);
    return t;
  };
  minima(tid, it);  // in flight while the smallest repeat is found
  fd = wave_min_u64(fd);
  if ((tid & 63) == 0) s_fd[tid >> 6] = fd;
  __syncthreads();
  fd = s_fd[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) fd = s_fd[w] < fd ? s_fd[w] : fd;
  uint64_t stay_min = kNoValue;
  int64_t npiv = 0, last = -1, nkept = 0;
  for (uint32_t i0 = 0; i0 < cnt; i0 += kCommitThreads) {
    const uint32_t i = i0 + tid;
    bool keep = false;
    const int64_t p = it.p;
    const uint64_t ra = it.ra, x = it.x;
    if (i < cnt) {
      const uint64_t e = enc(round, p);
      if ((uint64_t)p < fd || (it.lc == e && it.tc > e)) {
        const int32_t r = (int32_t)(ra >> 32), a = (int32_t)(uint32_t)ra;
        A.part[r] = a;  // the stored column {a, r}
        if (A.part16) A.part16[r] = (uint16_t)a;
        A.killer[r] = p;
        ++npiv;
        last = p > last ? p : last;
      } else {
        keep = true;
        stay_min = (uint64_t)p < stay_min ? (uint64_t)p : stay_min;
      }
    }
    if (i0 + kCommitThreads < cnt) it = load(i + kCommitThreads);
    int64_t total;
    const int64_t at = block_excl_i64<kWaves>(keep ? 1 : 0, itmp, &total);
    if (keep) {
      kept_out[nkept + at] = p;
      kept_ra[nkept + at] = ra;
      kept_x[nkept + at] = x;
    }
    nkept += total;
  }
  // The three totals in one barrier.
  {
    const int64_t wn = wave_sum_i64(npiv);
    const uint64_t we = wave_max_u64((uint64_t)(last + 1));
    const uint64_t wst = wave_min_u64(stay_min);
    if ((tid & 63) == 0) {
      s_tot[tid >> 6][0] = (uint64_t)wn;
      s_tot[tid >> 6][1] = we;
      s_tot[tid >> 6][2] = wst;
    }
  }
  __syncthreads();
  uint64_t last_end = 0;
  if (tid == 0) {
    npiv = 0;
    stay_min = kNoValue;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      npiv += (int64_t)s_tot[w][0];
      last_end = s_tot[w][1] > last_end ? s_tot[w][1] : last_end;
      stay_min = s_tot[w][2] < stay_min ? s_tot[w][2] : stay_min;
    }
    // Offsets below the ring's capacity (< 2^31).
    *slot = make_uint4((uint32_t)npiv, (uint32_t)nkept,
                       npiv ? (uint32_t)((int64_t)last_end - F) : 0u,
                       stay_min == kNoValue ? ~0u : (uint32_t)((int64_t)stay_min - F));
  }
}

// The state entering round `rounds` on its own, one wave (the walk of that
// round would form the same), also left in pinned host memory when
// `publish` is given.
__global__ __launch_bounds__(64) void k_advance(RedArgs A, int64_t rounds, RedCtl* publish) {
  __shared__ int64_t pre[kMaxWalkBlocks + 1];
  (void)advance_wave(A, A.ctl + ((rounds - 1) & 1), true, A.ctl + (rounds & 1), publish, pre);
}

// Sum of the walk blocks' counter slots into the control block.
__global__ __launch_bounds__(256) void k_walk_stats(const uint64_t* wstat, int64_t blocks,
                                                    RedCtl* ctl) {
  __shared__ int64_t tmp[4];
  int64_t c[3] = {0, 0, 0};
  for (int64_t b = threadIdx.x; b < blocks; b += blockDim.x)
    for (int q = 0; q < 3; ++q) c[q] += (int64_t)wstat[3 * b + q];
  for (int q = 0; q < 3; ++q) c[q] = block_sum_i64<4>(c[q], tmp);
  if (threadIdx.x == 0) {
    ctl->additions_all = c[0];
    ctl->find_steps = c[1];
    ctl->words_read = c[2];
  }
}

// More sorted columns are available (the last round stopped with need_more,
// every column before the old limit final, none kept): the window continues
// behind its old end at its current width.
__global__ void k_reduce_extend(RedCtl* ctl, int64_t E_lim) {
  const RedCtl c = *ctl;
  const int64_t Wend = c.F + c.width < E_lim ? c.F + c.width : E_lim;
  ctl->E_lim = E_lim;
  ctl->need_more = 0;
  ctl->fresh_lo = c.Wend;
  ctl->fresh_hi = Wend;
  ctl->Wend = Wend;
  if (Wend > c.maxWend) ctl->maxWend = Wend;
}

// The reduction's starting state in one launch: an empty pivot table (part,
// its 16-bit mirror and killer all free), no row minima or touches, zeroed
// per-block counters, and the control block of the first window.
__global__ __launch_bounds__(256) void k_reduce_init(RedArgs A, int64_t E_lim, int64_t n16,
                                                     int64_t nwstat) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = g; i < A.n; i += stride) {
    A.part[i] = -1;
    A.killer[i] = -1;
    A.lowc[i] = kNoValue;
    A.touch[i] = kNoValue;
  }
  for (int64_t i = g; i < n16; i += stride) A.part16[i] = kFree16;
  for (int64_t i = g; i < nwstat; i += stride) A.wstat[i] = 0;
  if (g == 0) {
    RedCtl c = {};
    c.F = 0;
    c.E_lim = E_lim;
    c.width = A.width;
    c.width_min = A.width;
    c.Wend = A.width < E_lim ? A.width : E_lim;
    c.maxWend = c.Wend;
    c.fresh_lo = 0;
    c.fresh_hi = c.Wend;
    c.done = (A.n <= 1 || E_lim == 0) ? 1 : 0;
    A.ctl[0] = c;
    *A.werr = 0;
  }
}

// Additions of columns at or after E_eff (walked before the last pivot was
// known) are not part of the sequential count; sum them for subtraction.
// Every column of [E_eff, maxWend) was walked and still owns its ring entry:
// the reduction ends with the window start F >= E_eff, the window [F, maxWend)
// is at most Wcap wide and holds every column walked since F, so no later
// column has reused an entry of that range.
__global__ __launch_bounds__(256) void k_overshoot(Ring ring, int64_t Wcap, RedCtl* ctl) {
  __shared__ int64_t tmp[4];
  const int64_t lo = ctl->E_eff, hi = ctl->maxWend;
  int64_t s = 0;
  for (int64_t p = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < hi;
       p += (int64_t)gridDim.x * blockDim.x)
    s += ring.st[p & (Wcap - 1)] >> 2;
  s = block_sum_i64<4>(s, tmp);  // one atomic per block
  if (threadIdx.x == 0 && s)
    atomicAdd((unsigned long long*)&ctl->additions_overshoot, (unsigned long long)s);
}

// Grid of the end-of-reduction sweep: up to four 256-thread blocks per CU.
int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
      cus = 256;
    else
      cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  }
  return cus;
}

int scan_blocks(int64_t Wcap) {
  int64_t b = (Wcap + 255) / 256;
  const int64_t cap = 4 * (int64_t)device_cus();
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

// One lane per column, up to kMaxWalkBlocks workgroups of 1024 lanes (two
// per compute unit of MI355X: 32 waves per CU); beyond that each lane takes
// several columns in turn.  The commit runs one workgroup per walk
// workgroup.  Fixed, not queried, so that workspace sizes do not depend on
// the device.
int walk_blocks(int64_t Wcap) {
  int64_t b = (Wcap + kWalkThreads - 1) / kWalkThreads;
  if (b > kMaxWalkBlocks) b = kMaxWalkBlocks;
  return (int)(b < 1 ? 1 : b);
}

// Survivor (and kept-column) entries per walk workgroup: the most items one
// workgroup can see in a round (a round has at most Wcap items).
int64_t walk_segment(int64_t Wcap) {
  const int64_t threads = kWalkThreads * (int64_t)walk_blocks(Wcap);
  return kWalkThreads * ((Wcap + threads - 1) / threads);
}

// Entries of the 16-bit table mirror (a multiple of 8, so that the walk
// copies it in 16-byte pieces), or 0 when n is too large for 16 bits.
int64_t part16_len(int64_t n) { return n <= kPart16MaxN ? (n + 7) / 8 * 8 : 0; }

hipError_t launch_reduce_extend(const RedArgs& a, int64_t E_lim, int64_t rounds, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_extend, dim3(1), dim3(1), 0, s, reduce_state(a, rounds), E_lim);
  return hipGetLastError();
}

hipError_t launch_reduce_init(const RedArgs& a, int64_t E_lim, hipStream_t s) {
  const int64_t n16 = a.part16 ? part16_len(a.n) : 0;
  const int64_t nwstat = 3 * (int64_t)walk_blocks(a.Wcap);
  const int64_t most = std::max(std::max(a.n, n16), nwstat);
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((most + 255) / 256, 1),
                                           4 * (int64_t)device_cus());
  hipLaunchKernelGGL(k_reduce_init, dim3((unsigned)blocks), dim3(256), 0, s, a, E_lim, n16,
                     nwstat);
  return hipGetLastError();
}

hipError_t launch_reduce_round(const RedArgs& a, hipStream_t s, hipEvent_t* ev_walk, int64_t k,
                               bool advanced) {
  // The LDS table copy of the largest n (64 KB) is beyond the default
  // dynamic LDS limit of a workgroup.
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)k_walk<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(2 * kPart16MaxN));
  if (attr != hipSuccess) return attr;
  if (k == 0 && !advanced) return hipErrorInvalidValue;  // round 0 starts from the init state
  const int wb = walk_blocks(a.Wcap);
  if (ev_walk) (void)hipEventRecord(ev_walk[0], s);
  const int64_t n16 = a.part16 ? part16_len(a.n) : 0;
  const int adv = advanced ? 1 : 0;
  if (a.part16)
    hipLaunchKernelGGL(k_walk<true>, dim3((unsigned)wb), dim3(kWalkThreads), 2 * n16, s, a, n16,
                       k, adv);
  else
    hipLaunchKernelGGL(k_walk<false>, dim3((unsigned)wb), dim3(kWalkThreads), 0, s, a, n16, k,
                       adv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_walk) (void)hipEventRecord(ev_walk[1], s);
  hipLaunchKernelGGL(k_commit, dim3((unsigned)wb), dim3(kCommitThreads), 0, s, a, k);
  return hipGetLastError();
}

hipError_t launch_reduce_advance(const RedArgs& a, int64_t rounds, RedCtl* publish,
                                 hipStream_t s) {
  if (rounds < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, a, rounds, publish);
  return hipGetLastError();
}

hipError_t launch_reduce_finish(const RedArgs& a, int64_t rounds, hipStream_t s) {
  if (!a.count) return hipSuccess;
  RedCtl* ctl = reduce_state(a, rounds);
  hipLaunchKernelGGL(k_walk_stats, dim3(1), dim3(256), 0, s, a.wstat,
                     (int64_t)walk_blocks(a.Wcap), ctl);
  hipLaunchKernelGGL(k_overshoot, dim3(scan_blocks(a.Wcap)), dim3(256), 0, s, a.ring, a.Wcap,
                     ctl);
  return hipGetLastError();
}

}  // namespace ph0
