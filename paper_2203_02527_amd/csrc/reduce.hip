// reduce.hip -- steps 4-5 of the GPU pipeline (Section 4: "for each diagonal
// entry of the matrix: reduction step"): column reduction over F2 of the
// vertex-by-edge boundary matrix, left to right, with pivots (Section 2).
//
// Data layout.  The pivot table is dense and bit-packed: row r (the stored
// column whose low is r) holds N bits in LW = ceil(N/64) 64-bit words at
// table[r * LW].  The pivot bit r itself is implicit (a stored column's low
// is its row index), so row r holds exactly the column's other bit, below r:
// a lookup reads words 0 .. r/64 only, and a row is taken iff it is nonzero
// (the table starts zeroed).
//
// Columns are 2-sparse.  A reduced column has nonzero rows {a, r}, a < r,
// and the stored column of row r is {x, r}; adding one to the other over F2
// cancels row r and leaves {a, x} (nothing when x = a).  So the walk carries
// the column as its two rows and performs each addition on that support,
// while each stored column is read from the dense table by a lane group
// (word w in lane w % G, slot w / G) and its bit x found with a per-lane
// highest-set-bit, a ballot over the group and a lane read.  An all-zero row
// means slot r is free.  Every addition is exactly the one the sequential
// dense reduction makes.

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
#include <climits>

#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr uint64_t kNoValue = ~0ull;

__device__ inline uint64_t enc(int64_t round, int64_t p) {
  return ((uint64_t)(0xFFFFFF - (round & 0xFFFFFF)) << 40) | (uint64_t)p;
}

// Column layout inside a group of G lanes: word w lives in lane w % G, slot
// w / G, so one load instruction covers G consecutive words of a row.

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
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

__device__ inline uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = __shfl((uint32_t)v, src, 64);
  const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Highest set bit of the group's column, looking only at slots <= qmax
// (words above are known to be zero), or -1 for the zero column.
template <int G, int WPL>
__device__ inline int group_top_bit(const uint64_t (&w)[WPL], int gbase, int qmax) {
#pragma unroll
  for (int q = WPL - 1; q >= 0; --q) {
    if (q > qmax) continue;
    uint64_t m = __ballot(w[q] != 0);
    if constexpr (G < 64) m = (m >> gbase) & ((1ull << G) - 1ull);
    if (m) {
      const int top = 63 - __clzll(m);
      uint64_t word;
      if constexpr (G == 64)
        word = readlane64(w[q], top);
      else
        word = shfl64(w[q], gbase + top);
      return (q * G + top) * 64 + 63 - __clzll(word);
    }
  }
  return -1;
}

// Words 0..(r >> 6) of stored row r into w (the rest are zero).  Every lane
// issues all WPL loads unconditionally (addresses past the top word are
// clamped to it and the value masked), so the loads of one step are in
// flight together and wait once.
template <int G, int WPL>
__device__ inline void load_row(uint64_t (&w)[WPL], const uint64_t* __restrict__ table,
                                int64_t LW, int r, int gl) {
  const int top = r >> 6;
  const uint64_t* rp = table + (int64_t)r * LW;
  uint64_t v[WPL];
#pragma unroll
  for (int q = 0; q < WPL; ++q) {
    const int widx = q * G + gl;
    v[q] = rp[widx <= top ? widx : top];
  }
#pragma unroll
  for (int q = 0; q < WPL; ++q) {
    const int widx = q * G + gl;
    w[q] = widx <= top ? v[q] : 0ull;
  }
}

// The bit stored in row r (the stored column's other row), or -1 if the row
// is empty (slot r free).
template <int G, int WPL>
__device__ inline int row_bit(const uint64_t* __restrict__ table, int64_t LW, int r, int gl,
                              int gbase) {
  uint64_t w[WPL];
  load_row<G, WPL>(w, table, LW, r, gl);
  return group_top_bit<G, WPL>(w, gbase, (r >> 6) / G);
}

// A value the whole group agrees on; for a full-wave group it is moved to a
// scalar register so that branches on it are scalar.
template <int G>
__device__ inline int group_uniform(int x) {
  if constexpr (G == 64)
    return __builtin_amdgcn_readfirstlane(x);
  else
    return x;
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

// atomicMin that first looks at the current value: rows that many survivors
// share would otherwise serialize on one address.  A stale read only costs
// an unneeded atomic.
__device__ inline void filtered_min(uint64_t* addr, uint64_t v) {
  if (*(volatile uint64_t*)addr > v)
    atomicMin((unsigned long long*)addr, (unsigned long long)v);
}

__device__ inline int64_t item_column(const RedCtl* ctl, const int64_t* act, int64_t t) {
  return t < ctl->nA ? act[t] : ctl->fresh_lo + (t - ctl->nA);
}

template <int G, int WPL>
__global__ __launch_bounds__(256) void k_walk(const uint64_t* __restrict__ skeys, int ib,
                                              int64_t LW, const uint64_t* __restrict__ table,
                                              Ring ring, int64_t Wcap, const int64_t* act0,
                                              const int64_t* act1, uint64_t* lowc,
                                              uint64_t* touch, RedCtl* ctl) {
  if (ctl->done) return;
  const int64_t nA = ctl->nA, round = ctl->round;
  const int64_t items = nA + (ctl->fresh_hi - ctl->fresh_lo);
  const int64_t* act = ctl->cur ? act1 : act0;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int64_t gpb = blockDim.x / G;
  const int64_t gid = blockIdx.x * gpb + threadIdx.x / G;
  const int64_t gtotal = (int64_t)gridDim.x * gpb;
  const uint64_t imask = (1ull << ib) - 1ull;

  int64_t adds = 0, finds = 0, words = 0;
  int32_t bad = 0;
  for (int64_t t = gid; t < items; t += gtotal) {
    int64_t p;
    int32_t a, r, rlo, prev_steps;
    if (t < nA) {
      p = act[t];
      const int64_t k = p & (Wcap - 1);
      a = ring.a[k];
      r = ring.r[k];
      rlo = ring.rlo[k];
      prev_steps = ring.st[k] >> 2;
    } else {
      p = ctl->fresh_lo + (t - nA);
      const uint64_t key = skeys[p];
      a = (int32_t)(key & imask);
      r = (int32_t)((key >> ib) & imask);
      rlo = a;
      prev_steps = 0;
    }
    int moved = 0;
    bool zero = false;
    r = group_uniform<G>(r);
    a = group_uniform<G>(a);
    while (true) {
      const int x = group_uniform<G>(row_bit<G, WPL>(table, LW, r, gl, gbase));
      words += (r >> 6) + 1;
      if (x < 0) break;  // row r is empty: slot r is free
      ++moved;
      if (x == a) {  // {a, r} + {a, r} = 0
        zero = true;
        break;
      }
      if (x >= r) {  // a stored bit must lie below its row; a corrupt table ends the walk
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
    int32_t status = kActive;
    if (zero) {
      status = kZero;
    } else {
      // Root of row a in the current forest: follow stored columns down.
      int v = group_uniform<G>(moved ? a : rlo);
      while (true) {
        const int c = group_uniform<G>(row_bit<G, WPL>(table, LW, v, gl, gbase));
        words += (v >> 6) + 1;
        if (c < 0) break;  // empty row: v is a root
        ++finds;
        if (c >= v) {  // a stored bit must lie below its row
          bad = 1;
          break;
        }
        v = c;
      }
      rlo = v;
      if (gl == 0) {
        const uint64_t e = enc(round, p);
        filtered_min(&lowc[r], e);
        filtered_min(&touch[rlo], e);
      }
    }
    if (gl == 0) {
      const int64_t k = p & (Wcap - 1);
      ring.a[k] = a;
      ring.r[k] = r;
      ring.rlo[k] = rlo;
      ring.st[k] = status | ((prev_steps + moved) << 2);
      ring.tag[k] = p;
    }
  }
  // Counters: group leaders -> block totals in LDS -> one atomic per block.
  __shared__ unsigned long long s_cnt[3];
  __shared__ int s_bad;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (gl == 0) {
    if (adds) atomicAdd(&s_cnt[0], (unsigned long long)adds);
    if (finds) atomicAdd(&s_cnt[1], (unsigned long long)finds);
    if (words) atomicAdd(&s_cnt[2], (unsigned long long)words);
    if (bad) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_cnt[0]) atomicAdd((unsigned long long*)&ctl->additions_all, s_cnt[0]);
    if (s_cnt[1]) atomicAdd((unsigned long long*)&ctl->find_steps, s_cnt[1]);
    if (s_cnt[2]) atomicAdd((unsigned long long*)&ctl->words_read, s_cnt[2]);
    if (s_bad) atomicOr(&ctl->err, 1);
  }
}

// ---- full-wave walk (N > 2048: a pivot row needs all 64 lanes) ----
//
// A reduced column is 2-sparse: its nonzero rows are {a, r}, a < r, and the
// stored column of row r is {x, r}, x < r.  Adding one to the other over F2
// cancels row r and leaves {a, x} (or nothing when x = a).  The full-wave
// walk therefore carries the column as its two rows (wave-uniform scalars)
// and performs each addition on that support, while the stored column is
// read from the dense bit-packed table: the 64 lanes load its words 0..r/64
// (word w in lane w % 64, slot w / 64), bit r is cleared, and x is the
// highest remaining set bit, found with one ballot per slot and a lane read.
// An empty row (no bit below r) means slot r is free.  Each addition is
// exactly the one the sequential dense reduction makes.
//
// The row's address and length (r / 64 + 1 words) go into a buffer resource,
// so the hardware range check returns zeros past the row's top word, and the
// loop runs in stages by the number S of 64-word slots the row prefix spans
// (S = r / 4096 + 1, which only falls as r falls), so each stage loads and
// searches exactly S slots with no per-slot tests.

__device__ inline __amdgpu_buffer_rsrc_t wide_rsrc(const char* tbase, uint32_t rowb, int r) {
  const uint32_t nrec = (((uint32_t)r | 63u) >> 3) + 1u;  // (r / 64 + 1) words
  return __builtin_amdgcn_make_buffer_rsrc((void*)(tbase + (uint32_t)r * rowb), 0, (int)nrec,
                                           0x00020000);
}

template <int S>
__device__ inline void wide_issue(uint64_t (&v)[S], __amdgpu_buffer_rsrc_t rs, int lane) {
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, q * 512, 0);
    v[q] = ((uint64_t)x[1] << 32) | x[0];
  }
}

// XOR S loaded slots into the column and return its new top bit (-1 if the
// column became zero).  Slots >= S of the column are zero already (its bits
// are <= r), so only S slots are searched: one ballot per slot, the highest
// non-empty slot picked with scalar selects, one lane read.
// Highest set bit among slots 0..S-1 of w (-1 if none): one ballot per slot,
// the highest non-empty slot picked with scalar selects, one lane read.
template <int S, int N>
__device__ inline int slots_top(const uint64_t (&w)[N]) {
  static_assert(S <= N, "slot count");
  uint64_t m = __ballot(w[0] != 0);
  int qs = 0;
#pragma unroll
  for (int q = 1; q < S; ++q) {
    const uint64_t mq = __ballot(w[q] != 0);
    qs = mq ? q : qs;
    m = mq ? mq : m;
  }
  if (m == 0) return -1;
  const int L = 63 - __clzll(m);
  uint64_t word = readlane64(w[0], L);
#pragma unroll
  for (int q = 1; q < S; ++q) {
    const uint64_t wq = readlane64(w[q], L);
    word = qs == q ? wq : word;
  }
  return (qs * 64 + L) * 64 + 63 - __clzll(word);
}

// The bit stored in row v (-1 if the row is empty): the row's prefix spans
// S = v / 4096 + 1 slots.
template <int S>
__device__ inline int row_top(const char* tbase, uint32_t rowb, int v, int lane) {
  uint64_t row[S];
  wide_issue<S>(row, wide_rsrc(tbase, rowb, v), lane);
  return slots_top<S>(row);
}

template <int WPL, int S = WPL>
__device__ inline int row_top_n(const char* tbase, uint32_t rowb, int v, int lane) {
  if constexpr (S > 1) {
    if (v < (S - 1) * 4096) return row_top_n<WPL, S - 1>(tbase, rowb, v, lane);
  }
  return row_top<S>(tbase, rowb, v, lane);
}

struct WalkState {
  int r;      // the column's low (wave-uniform)
  int a;      // its other row (wave-uniform)
  int moved;  // additions made
  int words;  // table words loaded
  bool stop, zero, bad;
};

// Steps on rows whose prefix spans S slots -- r >= (S - 1) * 4096; r < S *
// 4096 holds already since r only decreases -- then the stages below.
// Returns the last row read's other bit x when the walk stopped (x < 0: slot
// r is free; x == a: the column became zero), or INT_MIN if it did not stop.
template <int WPL, int S>
__device__ inline int wide_stages(const char* tbase, uint32_t rowb, int lane, int& r, int& a,
                                  int& moved, int& words) {
  while (r >= (S - 1) * 4096) {
    uint64_t w[S];
    wide_issue<S>(w, wide_rsrc(tbase, rowb, r), lane);
    words += r >> 6;
    // The stored bit x: highest non-empty slot, highest lane, highest bit.
    uint64_t m = __ballot(w[0] != 0);
    int qs = 0;
#pragma unroll
    for (int q = 1; q < S; ++q) {
      const uint64_t mq = __ballot(w[q] != 0);
      qs = mq ? q : qs;
      m = mq ? mq : m;
    }
    if (m == 0) return -1;  // row r is empty: slot r is free
    const int L = 63 - __builtin_clzll(m);
    uint64_t word = readlane64(w[0], L);
#pragma unroll
    for (int q = 1; q < S; ++q) {
      const uint64_t wq = readlane64(w[q], L);
      word = qs == q ? wq : word;
    }
    const int x = (qs * 64 + L) * 64 + 63 - __builtin_clzll(word);
    if (x == a) return x;  // {a, r} + {a, r} = 0
    ++moved;
    // {a, r} + {x, r} = {a, x}
    const int lo = x < a ? x : a;
    r = x < a ? a : x;
    a = lo;
  }
  if constexpr (S > 1) return wide_stages<WPL, S - 1>(tbase, rowb, lane, r, a, moved, words);
  return INT_MIN;  // unreachable: r >= 0 always stops in the last stage
}

// Walk a column to its stop: a free slot r (survivor) or zero.
template <int WPL>
__device__ inline void wide_walk(const char* tbase, uint32_t rowb, int lane, WalkState& w) {
  int r = w.r, a = w.a, moved = 0, words = 0;
  const int x = wide_stages<WPL, WPL>(tbase, rowb, lane, r, a, moved, words);
  const bool zero = x >= 0;  // x == a: the addition cancelled the column
  w.r = r;
  w.a = a;
  w.moved = moved + (zero ? 1 : 0);
  w.words = words + moved + 1;  // one row load per step: (r / 64 + 1) words
  w.zero = zero;
  w.stop = true;
}

// Per-launch context of the full-wave walk kernels.
struct WideCtx {
  const uint64_t* skeys;
  const int64_t* act;
  Ring ring;
  uint64_t* lowc;
  uint64_t* touch;
  const char* tbase;
  const uint64_t* table;
  int64_t LW, Wcap, nA, fresh_lo, round;
  uint64_t imask;
  uint32_t rowb;
  int ib, lane;
  // per-wave tallies
  int64_t adds, finds, words;
  int32_t bad;
};

// A column in flight: sorted position, other row a, root of a, earlier
// additions, and the walk state (current low, this launch's additions).
struct WideCol {
  int64_t p;
  int a, rlo, prev;
  WalkState w;
};

// The wave's next work item, fetched while the current one walks: stage 1
// (at the start of the walk) reads the active-list entry or the fresh key,
// stage 2 (after the walk) the ring entry of a resumed column, so neither
// dependent load sits on the path between two columns.
struct WideNext {
  int64_t t;
  uint64_t raw;  // the column p (resumed item) or the key (fresh item)
  int32_t a, r, rlo, st;
};

// One load from one of two places (a single destination keeps the compiler
// from merging two conditional stores into a dynamically indexed one).
__device__ inline void next_fetch1(const WideCtx& x, WideNext& nx, int64_t items) {
  if (nx.t < items) {
    const uint64_t* src = nx.t < x.nA ? reinterpret_cast<const uint64_t*>(x.act) + nx.t
                                      : x.skeys + x.fresh_lo + (nx.t - x.nA);
    nx.raw = *src;
  }
}

__device__ inline void next_fetch2(const WideCtx& x, WideNext& nx) {
  if (nx.t < x.nA) {
    const int64_t q = (int64_t)nx.raw & (x.Wcap - 1);
    nx.a = x.ring.a[q];
    nx.r = x.ring.r[q];
    nx.rlo = x.ring.rlo[q];
    nx.st = x.ring.st[q];
  }
}

// Start the prefetched item: an active column resumed from its ring entry,
// or a fresh column {i, j} from its key.
__device__ inline void wide_begin(const WideCtx& x, const WideNext& nx, WideCol& c) {
  int a, r, rlo;
  if (nx.t < x.nA) {
    c.p = (int64_t)nx.raw;
    a = nx.a;
    r = nx.r;
    rlo = nx.rlo;
    c.prev = nx.st >> 2;
  } else {
    c.p = x.fresh_lo + (nx.t - x.nA);
    a = (int)(nx.raw & x.imask);
    r = (int)((nx.raw >> x.ib) & x.imask);
    rlo = a;
    c.prev = 0;
  }
  c.a = __builtin_amdgcn_readfirstlane(a);
  c.rlo = __builtin_amdgcn_readfirstlane(rlo);
  c.w = WalkState{__builtin_amdgcn_readfirstlane(r), c.a, 0, 0, false, false, false};
}

// A column whose walk stopped: a zero column, or a survivor {a, r} on free
// slot r.  For a survivor the root of a in the current forest is found by
// following stored columns down, and the round-tagged minima for slot r and
// that root are lowered (both current values are read before either atomic,
// so the wave waits once).  The column's state goes back to the ring (a zero
// column needs only its status and owner).
template <int WPL>
__device__ inline void wide_finish(WideCtx& x, WideCol& c) {
  const int lane = x.lane;
  const int r = c.w.r, a = c.w.a;
  int rlo = c.rlo;
  x.adds += c.w.moved;
  x.words += c.w.words;
  if (c.w.bad) x.bad = 1;
  const int64_t q = c.p & (x.Wcap - 1);
  if (c.w.zero) {
    if (lane == 0) {
      x.ring.st[q] = kZero | ((c.prev + c.w.moved) << 2);
      x.ring.tag[q] = c.p;
    }
    return;
  }
  // Root of row a in the current forest: follow stored columns down.
  int v = c.w.moved ? a : rlo;
  while (true) {
    x.words += (v >> 6) + 1;
    const int cb = __builtin_amdgcn_readfirstlane(row_top_n<WPL>(x.tbase, x.rowb, v, lane));
    if (cb < 0) break;  // empty row: v is a root
    ++x.finds;
    v = cb;
  }
  rlo = v;
  if (lane == 0) {
    const uint64_t e = enc(x.round, c.p);
    const uint64_t cur_l = *(volatile uint64_t*)&x.lowc[r];
    const uint64_t cur_t = *(volatile uint64_t*)&x.touch[rlo];
    if (cur_l > e) atomicMin((unsigned long long*)&x.lowc[r], (unsigned long long)e);
    if (cur_t > e) atomicMin((unsigned long long*)&x.touch[rlo], (unsigned long long)e);
    x.ring.a[q] = a;
    x.ring.r[q] = r;
    x.ring.rlo[q] = rlo;
    x.ring.st[q] = kActive | ((c.prev + c.w.moved) << 2);
    x.ring.tag[q] = c.p;
  }
}

__device__ inline bool wide_setup(WideCtx& x, const uint64_t* skeys, int ib, int64_t LW,
                                  const uint64_t* table, Ring ring, int64_t Wcap,
                                  const int64_t* act0, const int64_t* act1, uint64_t* lowc,
                                  uint64_t* touch, const RedCtl* ctl, int64_t* items) {
  if (ctl->done) return false;
  x.nA = ctl->nA;
  x.round = ctl->round;
  x.fresh_lo = ctl->fresh_lo;
  *items = x.nA + (ctl->fresh_hi - x.fresh_lo);
  x.act = ctl->cur ? act1 : act0;
  x.skeys = skeys;
  x.ring = ring;
  x.lowc = lowc;
  x.touch = touch;
  x.table = table;
  x.tbase = reinterpret_cast<const char*>(table);
  x.LW = LW;
  x.Wcap = Wcap;
  x.imask = (1ull << ib) - 1ull;
  x.rowb = (uint32_t)LW * 8u;
  x.ib = ib;
  x.lane = threadIdx.x & 63;
  x.adds = x.finds = x.words = 0;
  x.bad = 0;
  return true;
}

// Block-level flush of the per-wave tallies: one global atomic per counter
// and block.
__device__ inline void wide_flush(const WideCtx& x, RedCtl* ctl) {
  __shared__ unsigned long long s_cnt[3];
  __shared__ int s_bad;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (x.lane == 0) {
    if (x.adds) atomicAdd(&s_cnt[0], (unsigned long long)x.adds);
    if (x.finds) atomicAdd(&s_cnt[1], (unsigned long long)x.finds);
    if (x.words) atomicAdd(&s_cnt[2], (unsigned long long)x.words);
    if (x.bad) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_cnt[0]) atomicAdd((unsigned long long*)&ctl->additions_all, s_cnt[0]);
    if (s_cnt[1]) atomicAdd((unsigned long long*)&ctl->find_steps, s_cnt[1]);
    if (s_cnt[2]) atomicAdd((unsigned long long*)&ctl->words_read, s_cnt[2]);
    if (s_bad) atomicOr(&ctl->err, 1);
  }
}

template <int WPL>
__global__ __launch_bounds__(256) void k_walk_wide(const uint64_t* __restrict__ skeys, int ib,
                                                   int64_t LW, const uint64_t* __restrict__ table,
                                                   Ring ring, int64_t Wcap, const int64_t* act0,
                                                   const int64_t* act1, uint64_t* lowc,
                                                   uint64_t* touch, RedCtl* ctl) {
  WideCtx x;
  int64_t items;
  if (!wide_setup(x, skeys, ib, LW, table, ring, Wcap, act0, act1, lowc, touch, ctl, &items))
    return;
  const int64_t wid = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  const int64_t wtotal = (int64_t)gridDim.x * (blockDim.x / 64);
  WideNext nx;
  nx.t = wid;
  next_fetch1(x, nx, items);
  next_fetch2(x, nx);
  while (nx.t < items) {
    WideCol c;
    wide_begin(x, nx, c);
    nx.t += wtotal;
    next_fetch1(x, nx, items);
    wide_walk<WPL>(x.tbase, x.rowb, x.lane, c.w);
    next_fetch2(x, nx);
    wide_finish<WPL>(x, c);
  }
  wide_flush(x, ctl);
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

__global__ __launch_bounds__(256) void k_decide(Ring ring, int64_t Wcap, const int64_t* act0,
                                                const int64_t* act1, const uint64_t* lowc,
                                                RedCtl* ctl) {
  __shared__ uint64_t tmp[4];
  if (ctl->done) return;
  const int64_t round = ctl->round;
  const int64_t items = ctl->nA + (ctl->fresh_hi - ctl->fresh_lo);
  const int64_t* act = ctl->cur ? act1 : act0;
  uint64_t best = kNoValue;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < items;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = item_column(ctl, act, t);
    const int64_t k = p & (Wcap - 1);
    if ((ring.st[k] & 3) != kActive) continue;
    if (lowc[ring.r[k]] != enc(round, p) && (uint64_t)p < best) best = (uint64_t)p;
  }
  best = block_min_u64(best, tmp);
  if (threadIdx.x == 0 && best != kNoValue)
    atomicMin((unsigned long long*)&ctl->firstdup[round & 1], (unsigned long long)best);
}

// End of a round: the next window start F (first column left active), the
// next window, and the hand-over of the active list (one thread; a separate
// launch costs less than electing the last commit workgroup with a ticket,
// whose same-address atomics serialize across the grid).
__device__ void advance_round(RedCtl* ctl_, int64_t n, int64_t E, int64_t Wcap) {
  volatile RedCtl* ctl = ctl_;
  const int64_t round = ctl->round;
  const uint64_t nf = ctl->newF[round & 1];
  const int64_t F = nf == kNoValue ? ctl->Wend : (int64_t)nf;
  int64_t Wend = ctl->Wend;
  if (ctl->pivots >= n - 1) {
    // Every later column reduces to zero; only columns before the last
    // pivot still need finishing (for the exact addition count).
    if (F >= ctl->E_eff) ctl->done = 1;
  } else {
    const int64_t lim = ctl->E_lim;
    Wend = F + Wcap < lim ? F + Wcap : lim;
    if (F >= lim) {
      if (lim < E) {
        ctl->need_more = 1;  // the host sorts the next distance range
      } else {
        ctl->done = 1;
        ctl->err |= 2;
      }
    }
  }
  ctl->fresh_lo = ctl->Wend;
  ctl->fresh_hi = Wend;
  ctl->nA = ctl->nA_next;
  ctl->nA_next = 0;
  ctl->cur ^= 1;
  ctl->F = F;
  ctl->Wend = Wend;
  if (Wend > ctl->maxWend) ctl->maxWend = Wend;
  ctl->round = round + 1;
}

// Commit the survivors the rule allows; append the rest to the next active
// list.  Two phases per block so that the list needs one atomic per block:
// commit and count, then (after one block-wide scan) write the stayers.
__global__ __launch_bounds__(256) void k_commit(Ring ring, int64_t Wcap, int64_t* act0,
                                                int64_t* act1, const uint64_t* lowc,
                                                const uint64_t* touch,
                                                uint64_t* table, int64_t LW, int64_t* killer,
                                                RedCtl* ctl) {
  __shared__ int64_t itmp[4];
  __shared__ uint64_t utmp[4];
  __shared__ int64_t s_base;
  if (ctl->done) return;
  const int64_t round = ctl->round;
  const int64_t items = ctl->nA + (ctl->fresh_hi - ctl->fresh_lo);
  const int64_t* act = ctl->cur ? act1 : act0;
  int64_t* next = ctl->cur ? act0 : act1;
  const uint64_t fd = ctl->firstdup[round & 1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint64_t stay_min = kNoValue;
  int64_t npiv = 0, last = -1, nstay = 0;
  for (int64_t t = t0; t < items; t += stride) {
    const int64_t p = item_column(ctl, act, t);
    const int64_t k = p & (Wcap - 1);
    const int32_t st = ring.st[k];
    if ((st & 3) != kActive) continue;
    const int32_t r = ring.r[k];
    const uint64_t e = enc(round, p);
    if ((uint64_t)p < fd || (lowc[r] == e && touch[r] > e)) {
      const int32_t a = ring.a[k];
      table[(int64_t)r * LW + (a >> 6)] = 1ull << (a & 63);  // pivot bit r is implicit
      killer[r] = p;
      ring.st[k] = (st & ~3) | kCommitted;
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
    for (int64_t t = t0; t < items; t += stride) {
      const int64_t p = item_column(ctl, act, t);
      if ((ring.st[p & (Wcap - 1)] & 3) == kActive) next[at++] = p;
    }
  }
  npiv = block_sum_i64(npiv, itmp);
  const uint64_t last_c = block_min_u64(~(uint64_t)(last + 1), utmp);
  stay_min = block_min_u64(stay_min, utmp);
  if (threadIdx.x == 0) {
    if (npiv) {
      atomicAdd((unsigned long long*)&ctl->pivots, (unsigned long long)npiv);
      atomicMax((long long*)&ctl->E_eff, (long long)~last_c);
    }
    if (stay_min != kNoValue)
      atomicMin((unsigned long long*)&ctl->newF[round & 1], (unsigned long long)stay_min);
    if (blockIdx.x == 0) {
      ctl->firstdup[(round + 1) & 1] = kNoValue;
      ctl->newF[(round + 1) & 1] = kNoValue;
    }
  }
}

__global__ void k_advance(RedCtl* ctl, int64_t n, int64_t E, int64_t Wcap) {
  if (ctl->done) return;
  advance_round(ctl, n, E, Wcap);
}

__global__ void k_reduce_extend(RedCtl* ctl, int64_t E_lim, int64_t Wcap) {
  // All columns before the old limit are final here (F == old limit).
  ctl->E_lim = E_lim;
  ctl->need_more = 0;
  const int64_t F = ctl->F;
  const int64_t Wend = F + Wcap < E_lim ? F + Wcap : E_lim;
  ctl->fresh_lo = ctl->Wend;
  ctl->fresh_hi = Wend;
  ctl->Wend = Wend;
  if (Wend > ctl->maxWend) ctl->maxWend = Wend;
}

__global__ void k_reduce_init(RedCtl* ctl, int64_t E_lim, int64_t Wcap, int64_t n) {
  RedCtl c = {};
  c.F = 0;
  c.E_lim = E_lim;
  c.Wend = Wcap < E_lim ? Wcap : E_lim;
  c.maxWend = c.Wend;
  c.fresh_lo = 0;
  c.fresh_hi = c.Wend;
  c.firstdup[0] = c.firstdup[1] = kNoValue;
  c.newF[0] = c.newF[1] = kNoValue;
  c.done = (n <= 1 || E_lim == 0) ? 1 : 0;
  *ctl = c;
}

// Additions of columns at or after E_eff (walked before the last pivot was
// known) are not part of the sequential count; sum them for subtraction.
__global__ __launch_bounds__(256) void k_overshoot(Ring ring, int64_t Wcap, RedCtl* ctl) {
  const int64_t lo = ctl->E_eff, hi = ctl->maxWend;
  int64_t s = 0;
  for (int64_t p = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < hi;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = p & (Wcap - 1);
    if (ring.tag[k] == p) s += ring.st[k] >> 2;
  }
  __shared__ int64_t tmp[4];
  s = block_sum_i64(s, tmp);  // one atomic per block: same-address atomics serialize
  if (threadIdx.x == 0 && s)
    atomicAdd((unsigned long long*)&ctl->additions_overshoot, (unsigned long long)s);
}

// Resident-sized grids: the walk keeps about 32 waves per CU busy and loops.
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

template <int G, int WPL>
void walk_launch(const RedArgs& a, hipStream_t s) {
  const int64_t gpb = 256 / G;
  int64_t blocks = (a.Wcap + gpb - 1) / gpb;
  const int64_t cap = 8 * (int64_t)device_cus();
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  if constexpr (G == 64) {
    hipLaunchKernelGGL((k_walk_wide<WPL>), dim3((unsigned)blocks), dim3(256), 0, s, a.skeys, a.ib,
                       a.LW, a.table, a.ring, a.Wcap, a.act[0], a.act[1], a.lowc, a.touch,
                       a.ctl);
    return;
  }
  hipLaunchKernelGGL((k_walk<G, WPL>), dim3((unsigned)blocks), dim3(256), 0, s, a.skeys, a.ib,
                     a.LW, a.table, a.ring, a.Wcap, a.act[0], a.act[1], a.lowc, a.touch, a.ctl);
}

int scan_blocks(int64_t Wcap) {
  int64_t b = (Wcap + 255) / 256;
  const int64_t cap = 4 * (int64_t)device_cus();
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

// Lanes per column: enough words per lane to cover a row, and at most
// 64 lanes; `want` (a power of two) asks for fewer lanes and more words each.
bool launch_walk_shape(const RedArgs& a, hipStream_t s) {
  const int64_t LW = a.LW;
  int G = 1;
  while (G < 64 && G < LW) G <<= 1;
  if (a.lanes > 0 && a.lanes < G) G = a.lanes;
  const int64_t wpl = (LW + G - 1) / G;
#define PH0_WALK(g, w)                      \
  if (G == g && wpl <= w) {                 \
    walk_launch<g, w>(a, s);                \
    return true;                            \
  }
  PH0_WALK(1, 1) PH0_WALK(2, 1) PH0_WALK(4, 1) PH0_WALK(8, 1) PH0_WALK(16, 1)
  PH0_WALK(32, 1) PH0_WALK(64, 1) PH0_WALK(64, 2) PH0_WALK(64, 4) PH0_WALK(64, 8)
  PH0_WALK(64, 16) PH0_WALK(32, 2) PH0_WALK(32, 4) PH0_WALK(32, 8) PH0_WALK(32, 16)
  PH0_WALK(16, 2) PH0_WALK(16, 4) PH0_WALK(16, 8) PH0_WALK(16, 16)
#undef PH0_WALK
  if (a.lanes > 0) {  // requested shape not built: use the default one
    RedArgs d = a;
    d.lanes = 0;
    return launch_walk_shape(d, s);
  }
  return false;
}

}  // namespace

hipError_t launch_reduce_extend(const RedArgs& a, int64_t E_lim, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_extend, dim3(1), dim3(1), 0, s, a.ctl, E_lim, a.Wcap);
  return hipGetLastError();
}

hipError_t launch_reduce_init(const RedArgs& a, int64_t E_lim, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u64(a.table, 0ull, a.n * a.LW, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(a.killer), ~0ull, a.n, s)) != hipSuccess)
    return e;
  if ((e = launch_fill_u64(a.lowc, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(a.touch, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(a.ring.tag), ~0ull, a.Wcap, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_reduce_init, dim3(1), dim3(1), 0, s, a.ctl, E_lim, a.Wcap, a.n);
  return hipGetLastError();
}

hipError_t launch_reduce_round(const RedArgs& a, hipStream_t s, hipEvent_t* ev_walk) {
  if (ev_walk) (void)hipEventRecord(ev_walk[0], s);
  if (!launch_walk_shape(a, s)) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_walk) (void)hipEventRecord(ev_walk[1], s);
  const int sb = scan_blocks(a.Wcap);
  hipLaunchKernelGGL(k_decide, dim3(sb), dim3(256), 0, s, a.ring, a.Wcap, a.act[0], a.act[1],
                     a.lowc, a.ctl);
  hipLaunchKernelGGL(k_commit, dim3(sb), dim3(256), 0, s, a.ring, a.Wcap, a.act[0], a.act[1],
                     a.lowc, a.touch, a.table, a.LW, a.killer, a.ctl);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, a.ctl, a.n, a.E, a.Wcap);
  return hipGetLastError();
}

hipError_t launch_reduce_finish(const RedArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_overshoot, dim3(scan_blocks(a.Wcap)), dim3(256), 0, s, a.ring, a.Wcap,
                     a.ctl);
  return hipGetLastError();
}

}  // namespace ph0
