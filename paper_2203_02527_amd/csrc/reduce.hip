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
#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr uint64_t kNoValue = ~0ull;
constexpr uint16_t kFree16 = 0xFFFF;  // a free row in the 16-bit table mirror
constexpr int kWalkThreads = 1024;
constexpr int kWalkWaves = kWalkThreads / 64;
constexpr int kHashBits = 11;  // log2 of the LDS hash slots (2 x kWalkThreads)

__device__ inline uint64_t enc(int64_t round, int64_t p) {
  return ((uint64_t)(0xFFFFFF - (round & 0xFFFFFF)) << 40) | (uint64_t)p;
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

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = shfl64_down(v, o);
    v = w < v ? w : v;
  }
  return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (int64_t)shfl64_down((uint64_t)v, o);
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

__device__ inline int64_t item_column(const RedCtl* ctl, const int64_t* act, int64_t t) {
  return t < ctl->nA ? act[t] : ctl->fresh_lo + (t - ctl->nA);
}

// One round's walk: every item (carried active column or fresh column of the
// window) is reduced against the table as committed so far, one lane per
// column.  A column stops on a free row (a survivor) or becomes zero.  For a
// survivor {a, r} the root of a in the pivot forest (follow part[] down to a
// free row) is found, and the round-tagged minima for row r and that root
// are lowered.  A survivor's state goes back to the ring; a zero column only
// leaves its addition count there (for the overshoot sum).  Each block lists
// its survivors in its own segment of `surv` (seg entries per block, the
// count in scount[block]), so that the decide and commit steps visit
// survivors only, one block per walk block, with no shared counter.
// kLds: the table is read from the block's LDS copy of part16 (0xFFFF =
// free), else from part in global memory.
template <bool kLds>
__global__ __launch_bounds__(kWalkThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_walk(
    const uint64_t* __restrict__ skeys, int ib, const int32_t* __restrict__ part,
    const uint16_t* __restrict__ part16, int64_t n16, Ring ring, int64_t Wcap,
    const int64_t* act0, const int64_t* act1, uint64_t* lowc, uint64_t* touch, int64_t* surv,
    uint32_t* scount, int64_t seg, uint64_t* wstat, RedCtl* ctl) {
  extern __shared__ uint4 s_tab4[];  // kLds: n16 / 8 entries of 8 table rows
  __shared__ uint32_t s_wave[kWalkWaves];
  __shared__ unsigned long long s_cnt[3];
  __shared__ int s_bad;
  // Row-minimum hash tables: [0] by low r (lowc), [1] by root rlo (touch).
  __shared__ uint32_t s_hkey[2][kHashSlots];
  __shared__ uint32_t s_hval[2][kHashSlots];
  if (ctl->done) return;
  const int64_t nA = ctl->nA, round = ctl->round, fresh_lo = ctl->fresh_lo;
  const int64_t F = ctl->F;  // every item p has F <= p < F + Wcap
  const int64_t items = nA + (ctl->fresh_hi - fresh_lo);
  if ((int64_t)blockIdx.x * kWalkThreads >= items) {  // nothing for this block
    if (threadIdx.x == 0) scount[blockIdx.x] = 0;
    return;
  }
  for (int k = threadIdx.x; k < kHashSlots; k += kWalkThreads) {
    s_hkey[0][k] = s_hkey[1][k] = kHashEmpty;
    s_hval[0][k] = s_hval[1][k] = kRelNone;
  }
  if (kLds) {
    const uint4* src = reinterpret_cast<const uint4*>(part16);
    for (int64_t k = threadIdx.x; k < n16 / 8; k += kWalkThreads) s_tab4[k] = src[k];
  }
  __syncthreads();
  const uint16_t* s_tab = reinterpret_cast<const uint16_t*>(s_tab4);
  auto lookup = [&](int row) -> int {
    if (kLds) {
      const uint16_t v = s_tab[row];
      return v == kFree16 ? -1 : (int)v;
    }
    return part[row];
  };
  const int64_t* act = ctl->cur ? act1 : act0;
  const int64_t stride = (int64_t)gridDim.x * kWalkThreads;
  const uint64_t imask = (1ull << ib) - 1ull;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t* my_surv = surv + blockIdx.x * seg;
  uint32_t nsurv = 0;  // this block's survivors so far (same in every thread)
  int64_t adds = 0, finds = 0, words = 0;
  int32_t bad = 0;
  for (int64_t t0 = blockIdx.x * (int64_t)kWalkThreads; t0 < items; t0 += stride) {
    const int64_t t = t0 + threadIdx.x;
    bool survivor = false;
    int64_t p = 0;
    int32_t a, r, rlo;
    int hs_low = 0, hs_root = 0;  // this survivor's hash slots
    if (t < items) {
      int32_t prev_steps;
      if (t < nA) {
        p = act[t];
        const int64_t k = p & (Wcap - 1);
        a = ring.a[k];
        r = ring.r[k];
        rlo = ring.rlo[k];
        prev_steps = ring.st[k] >> 2;
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
        const int lo = x < a ? x : a;
        r = x < a ? a : x;
        a = lo;
      }
      adds += moved;
      const int64_t k = p & (Wcap - 1);
      if (zero) {
        ring.st[k] = kZero | ((prev_steps + moved) << 2);
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
        ring.a[k] = a;
        ring.r[k] = r;
        ring.rlo[k] = rlo;
        ring.st[k] = kActive | ((prev_steps + moved) << 2);
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
      if (s_hval[0][hs_low] == rel) atomicMin((unsigned long long*)&lowc[r], e);
      if (s_hval[1][hs_root] == rel) atomicMin((unsigned long long*)&touch[rlo], e);
    }
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWalkWaves; ++w) {
      before += w < wave ? s_wave[w] : 0u;
      total += s_wave[w];
    }
    if (survivor) my_surv[nsurv + before + __popcll(m & ((1ull << lane) - 1ull))] = p;
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
  if (threadIdx.x == 0) scount[blockIdx.x] = nsurv;
  // Counters: wave sums -> block totals in LDS -> the block's own slots.
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  adds = wave_sum_i64(adds);
  finds = wave_sum_i64(finds);
  words = wave_sum_i64(words);
  if (__ballot(bad != 0)) bad = 1;
  if ((threadIdx.x & 63) == 0) {
    if (adds) atomicAdd(&s_cnt[0], (unsigned long long)adds);
    if (finds) atomicAdd(&s_cnt[1], (unsigned long long)finds);
    if (words) atomicAdd(&s_cnt[2], (unsigned long long)words);
    if (bad) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // The block's own slots (the grid is the same every round), summed once
    // at the finish: an atomic per block and round on the three shared
    // counters serializes at one address and showed in the walk's time.
    uint64_t* mine = wstat + 3 * (int64_t)blockIdx.x;
    mine[0] += s_cnt[0];
    mine[1] += s_cnt[1];
    mine[2] += s_cnt[2];
    if (s_bad) atomicOr(&ctl->err, 1);
  }
}


// Block-wide reductions for the 256-thread decide/commit kernels.
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t* tmp /* 4 */) {
  v = wave_min_u64(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = tmp[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) r = tmp[w] < r ? tmp[w] : r;
  __syncthreads();
  return r;
}

__device__ inline int64_t block_sum_i64(int64_t v, int64_t* tmp /* 4 */) {
  v = wave_sum_i64(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  const int64_t r = tmp[0] + tmp[1] + tmp[2] + tmp[3];
  __syncthreads();
  return r;
}

// Sum of the walk blocks' counter slots into the control block.
__global__ __launch_bounds__(256) void k_walk_stats(const uint64_t* wstat, int64_t blocks,
                                                    RedCtl* ctl) {
  int64_t c[3] = {0, 0, 0};
  for (int64_t b = threadIdx.x; b < blocks; b += blockDim.x)
    for (int k = 0; k < 3; ++k) c[k] += (int64_t)wstat[3 * b + k];
  __shared__ int64_t tmp[4];
  for (int k = 0; k < 3; ++k) c[k] = block_sum_i64(c[k], tmp);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctl->additions_all, (unsigned long long)c[0]);
    atomicAdd((unsigned long long*)&ctl->find_steps, (unsigned long long)c[1]);
    atomicAdd((unsigned long long*)&ctl->words_read, (unsigned long long)c[2]);
  }
}

// Exclusive prefix of v over the block (and the block total).
__device__ inline int64_t block_excl_i64(int64_t v, int64_t* tmp /* 4 */, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = (int64_t)shfl64_up((uint64_t)x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  int64_t base = 0;
  for (int w = 0; w < wave; ++w) base += tmp[w];
  *total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
  __syncthreads();
  return base + x - v;
}

// First survivor whose low repeats an earlier survivor's low: the lowest
// survivor p with lowc[r] != its own tag.  One block per walk block, over
// that block's survivors.
__global__ __launch_bounds__(256) void k_decide(Ring ring, int64_t Wcap, const int64_t* surv,
                                                const uint32_t* scount, int64_t seg,
                                                const uint64_t* lowc, RedCtl* ctl) {
  __shared__ uint64_t tmp[4];
  if (ctl->done) return;
  const uint32_t cnt = scount[blockIdx.x];
  if (cnt == 0) return;
  const int64_t round = ctl->round;
  const int64_t* my = surv + blockIdx.x * seg;
  uint64_t best = kNoValue;
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t p = my[i];
    const int64_t k = p & (Wcap - 1);
    if (lowc[ring.r[k]] != enc(round, p) && (uint64_t)p < best) best = (uint64_t)p;
  }
  best = block_min_u64(best, tmp);
  if (threadIdx.x == 0 && best != kNoValue)
    atomicMin((unsigned long long*)&ctl->firstdup[round & 1], (unsigned long long)best);
}

// End of a round: the pivots and E_eff with this round's commits, the next
// window start F (first column left active, nf; none: the window end), the
// next window, and the hand-over of the active list (one thread of its own
// launch; electing the last commit workgroup with a ticket instead costs
// more, its same-address atomics serialize across the grid).
__device__ void advance_round(RedCtl* ctl, int64_t n, int64_t E, int64_t Wcap, uint64_t nf,
                              int64_t new_pivots, int64_t end) {
  // The control block is read once, up front, and written at the end: one
  // thread that read a field back after writing it could get the old value
  // from the scalar cache.
  const RedCtl c = *ctl;
  const int64_t pivots = c.pivots + new_pivots;
  const int64_t E_eff = end > c.E_eff ? end : c.E_eff;
  const int64_t F = nf == kNoValue ? c.Wend : (int64_t)nf;
  int64_t Wend = c.Wend, width = c.width;
  int32_t done = c.done, need_more = c.need_more, err = c.err;
  if (pivots >= n - 1) {
    // Every later column reduces to zero; only columns before the last
    // pivot still need finishing (for the exact addition count).
    if (F >= E_eff) done = 1;
  } else {
    const int64_t lim = c.E_lim;
    // Window width: doubles (up to the ring's capacity) while almost every
    // column of a round becomes final, halves (down to the base width) when
    // many stay.  The end never moves back: columns already in the window
    // stay there.
    const int64_t stay = c.nA_next;
    if (stay < width / 256)
      width = 2 * width < Wcap ? 2 * width : Wcap;
    else if (stay > width / 16)
      width = width / 2 > c.width_min ? width / 2 : c.width_min;
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
  ctl->pivots = pivots;
  ctl->E_eff = E_eff;
  ctl->width = width;
  ctl->done = done;
  ctl->need_more = need_more;
  ctl->err = err;
  ctl->fresh_lo = c.Wend;
  ctl->fresh_hi = Wend;
  ctl->nA = c.nA_next;
  ctl->nA_next = 0;
  ctl->cur = c.cur ^ 1;
  ctl->F = F;
  ctl->Wend = Wend;
  ctl->maxWend = Wend > c.maxWend ? Wend : c.maxWend;
  ctl->round = c.round + 1;
}

// Commit the survivors the rule allows; append the rest to the next active
// list.  One block per walk block, over that block's survivors, in two phases
// so that the list needs one atomic per block: commit and count, then (after
// one block-wide scan) write the stayers.
__global__ __launch_bounds__(256) void k_commit(Ring ring, int64_t Wcap, const int64_t* surv,
                                                const uint32_t* scount, int64_t seg,
                                                int64_t* act0, int64_t* act1,
                                                const uint64_t* lowc, const uint64_t* touch,
                                                int32_t* part, uint16_t* part16,
                                                int64_t* killer, uint64_t* cslot,
                                                RedCtl* ctl) {
  __shared__ int64_t itmp[4];
  __shared__ uint64_t utmp[4];
  __shared__ int64_t s_base;
  if (ctl->done) return;
  const int64_t round = ctl->round;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->firstdup[(round + 1) & 1] = kNoValue;
  // This block's slot: pivots committed, end of the last one, first stayer.
  uint64_t* slot = cslot + 3 * (int64_t)blockIdx.x;
  const uint32_t cnt = scount[blockIdx.x];
  if (cnt == 0) {
    if (threadIdx.x == 0) {
      slot[0] = 0;
      slot[1] = 0;
      slot[2] = kNoValue;
    }
    return;
  }
  int64_t* next = ctl->cur ? act0 : act1;
  const uint64_t fd = ctl->firstdup[round & 1];
  const int64_t* my = surv + blockIdx.x * seg;
  uint64_t stay_min = kNoValue;
  int64_t npiv = 0, last = -1, nstay = 0;
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t p = my[i];
    const int64_t k = p & (Wcap - 1);
    const int32_t r = ring.r[k];
    const uint64_t e = enc(round, p);
    if ((uint64_t)p < fd || (lowc[r] == e && touch[r] > e)) {
      const int32_t a = ring.a[k];
      part[r] = a;  // the stored column {a, r}
      if (part16) part16[r] = (uint16_t)a;
      killer[r] = p;
      ring.st[k] = (ring.st[k] & ~3) | kCommitted;
      ++npiv;
      last = p > last ? p : last;
    } else {
      ++nstay;
      if ((uint64_t)p < stay_min) stay_min = (uint64_t)p;
    }
  }
  int64_t total;
  const int64_t mine = block_excl_i64(nstay, itmp, &total);
  if (threadIdx.x == 0 && total)
    s_base = (int64_t)atomicAdd((unsigned long long*)&ctl->nA_next, (unsigned long long)total);
  __syncthreads();
  if (nstay) {
    int64_t at = s_base + mine;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
      const int64_t p = my[i];
      if ((ring.st[p & (Wcap - 1)] & 3) == kActive) next[at++] = p;
    }
  }
  npiv = block_sum_i64(npiv, itmp);
  const uint64_t last_c = block_min_u64(~(uint64_t)(last + 1), utmp);
  stay_min = block_min_u64(stay_min, utmp);
  if (threadIdx.x == 0) {
    slot[0] = (uint64_t)npiv;
    slot[1] = ~last_c;  // last committed position + 1, or 0
    slot[2] = stay_min;
  }
}

// The commit blocks' slots (pivot counts, pivot ends, first stayers) are
// reduced here, by one block, instead of three atomics per commit block on
// the shared control block; then the round advances.
__global__ __launch_bounds__(256) void k_advance(RedCtl* ctl, const uint64_t* cslot,
                                                 int64_t blocks, int64_t n, int64_t E,
                                                 int64_t Wcap) {
  __shared__ int64_t itmp[4];
  __shared__ uint64_t utmp[4];
  if (ctl->done) return;
  int64_t piv = 0;
  uint64_t end_c = kNoValue, stay = kNoValue;  // end_c: complement, so a min finds the max
  for (int64_t b = threadIdx.x; b < blocks; b += blockDim.x) {
    piv += (int64_t)cslot[3 * b];
    const uint64_t e = ~cslot[3 * b + 1];
    end_c = e < end_c ? e : end_c;
    stay = cslot[3 * b + 2] < stay ? cslot[3 * b + 2] : stay;
  }
  piv = block_sum_i64(piv, itmp);
  end_c = block_min_u64(end_c, utmp);
  stay = block_min_u64(stay, utmp);
  if (threadIdx.x == 0) advance_round(ctl, n, E, Wcap, stay, piv, (int64_t)~end_c);
}

__global__ void k_reduce_extend(RedCtl* ctl, int64_t E_lim) {
  // All columns before the old limit are final here (F == old limit).
  ctl->E_lim = E_lim;
  ctl->need_more = 0;
  const int64_t F = ctl->F;
  const int64_t width = ctl->width;
  const int64_t Wend = F + width < E_lim ? F + width : E_lim;
  ctl->fresh_lo = ctl->Wend;
  ctl->fresh_hi = Wend;
  ctl->Wend = Wend;
  if (Wend > ctl->maxWend) ctl->maxWend = Wend;
}

__global__ void k_reduce_init(RedCtl* ctl, int64_t E_lim, int64_t width, int64_t n) {
  RedCtl c = {};
  c.F = 0;
  c.E_lim = E_lim;
  c.width = width;
  c.width_min = width;
  c.Wend = width < E_lim ? width : E_lim;
  c.maxWend = c.Wend;
  c.fresh_lo = 0;
  c.fresh_hi = c.Wend;
  c.firstdup[0] = c.firstdup[1] = kNoValue;
  c.done = (n <= 1 || E_lim == 0) ? 1 : 0;
  *ctl = c;
}

// Additions of columns at or after E_eff (walked before the last pivot was
// known) are not part of the sequential count; sum them for subtraction.
// Every column of [E_eff, maxWend) was walked and still owns its ring entry:
// the reduction ends with the window start F >= E_eff, the window [F, maxWend)
// is at most Wcap wide and holds every column walked since F, so no later
// column has reused an entry of that range.
__global__ __launch_bounds__(256) void k_overshoot(Ring ring, int64_t Wcap, RedCtl* ctl) {
  const int64_t lo = ctl->E_eff, hi = ctl->maxWend;
  int64_t s = 0;
  for (int64_t p = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < hi;
       p += (int64_t)gridDim.x * blockDim.x)
    s += ring.st[p & (Wcap - 1)] >> 2;
  __shared__ int64_t tmp[4];
  s = block_sum_i64(s, tmp);  // one atomic per block: same-address atomics serialize
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

// One lane per column, up to 512 workgroups of 1024 lanes (two per compute
// unit of MI355X: 32 waves per CU); beyond that each lane takes several
// columns in turn.  The decide and commit steps run one block per walk
// block.  Fixed, not queried, so that workspace sizes do not depend on the
// device.
int walk_blocks(int64_t Wcap) {
  int64_t b = (Wcap + kWalkThreads - 1) / kWalkThreads;
  const int64_t cap = 512;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

// Survivor entries per walk block: the most items one block can see in a
// round (a round has at most Wcap items).
int64_t walk_segment(int64_t Wcap) {
  const int64_t threads = kWalkThreads * (int64_t)walk_blocks(Wcap);
  return kWalkThreads * ((Wcap + threads - 1) / threads);
}

// Entries of the 16-bit table mirror (a multiple of 8, so that the walk
// copies it in 16-byte pieces), or 0 when n is too large for 16 bits.
int64_t part16_len(int64_t n) { return n <= kPart16MaxN ? (n + 7) / 8 * 8 : 0; }

hipError_t launch_reduce_extend(const RedArgs& a, int64_t E_lim, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_extend, dim3(1), dim3(1), 0, s, a.ctl, E_lim);
  return hipGetLastError();
}

hipError_t launch_reduce_init(const RedArgs& a, int64_t E_lim, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(a.part), 0xFFFFFFFFu, a.n, s)) !=
      hipSuccess)
    return e;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(a.killer), ~0ull, a.n, s)) != hipSuccess)
    return e;
  if ((e = launch_fill_u64(a.lowc, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(a.touch, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(a.wstat, 0ull, 3 * (int64_t)walk_blocks(a.Wcap), s)) != hipSuccess)
    return e;
  if (a.part16 && (e = launch_fill_u32(reinterpret_cast<uint32_t*>(a.part16), 0xFFFFFFFFu,
                                       part16_len(a.n) / 2, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_reduce_init, dim3(1), dim3(1), 0, s, a.ctl, E_lim, a.width, a.n);
  return hipGetLastError();
}

hipError_t launch_reduce_round(const RedArgs& a, hipStream_t s, hipEvent_t* ev_walk) {
  // The LDS table copy of the largest n (64 KB) is beyond the default
  // dynamic LDS limit of a workgroup; two such workgroups still fit a CU.
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)k_walk<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(2 * kPart16MaxN));
  if (attr != hipSuccess) return attr;
  const int wb = walk_blocks(a.Wcap);
  const int64_t seg = walk_segment(a.Wcap);
  if (ev_walk) (void)hipEventRecord(ev_walk[0], s);
  const int64_t n16 = a.part16 ? part16_len(a.n) : 0;
  if (a.part16)
    hipLaunchKernelGGL(k_walk<true>, dim3((unsigned)wb), dim3(kWalkThreads), 2 * n16, s,
                       a.skeys, a.ib, a.part, a.part16, n16, a.ring, a.Wcap, a.act[0], a.act[1],
                       a.lowc, a.touch, a.surv, a.scount, seg, a.wstat, a.ctl);
  else
    hipLaunchKernelGGL(k_walk<false>, dim3((unsigned)wb), dim3(kWalkThreads), 0, s, a.skeys,
                       a.ib, a.part, a.part16, n16, a.ring, a.Wcap, a.act[0], a.act[1], a.lowc,
                       a.touch, a.surv, a.scount, seg, a.wstat, a.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_walk) (void)hipEventRecord(ev_walk[1], s);
  hipLaunchKernelGGL(k_decide, dim3((unsigned)wb), dim3(256), 0, s, a.ring, a.Wcap, a.surv,
                     a.scount, seg, a.lowc, a.ctl);
  hipLaunchKernelGGL(k_commit, dim3((unsigned)wb), dim3(256), 0, s, a.ring, a.Wcap, a.surv,
                     a.scount, seg, a.act[0], a.act[1], a.lowc, a.touch, a.part, a.part16,
                     a.killer, a.cslot, a.ctl);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, s, a.ctl, a.cslot, (int64_t)wb, a.n,
                     a.E, a.Wcap);
  return hipGetLastError();
}

hipError_t launch_reduce_finish(const RedArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_walk_stats, dim3(1), dim3(256), 0, s, a.wstat,
                     (int64_t)walk_blocks(a.Wcap), a.ctl);
  hipLaunchKernelGGL(k_overshoot, dim3(scan_blocks(a.Wcap)), dim3(256), 0, s, a.ring, a.Wcap,
                     a.ctl);
  return hipGetLastError();
}

}  // namespace ph0
