// h1.hip -- 1st persistent homology (H1) of the same filtration: reduction of
// the edge-by-triangle boundary matrix over F2, the higher-dimension case
// that Section 3 says repeats the H0 work with more computation, on the GPU
// steps of Section 4 (boundary matrix, then one reduction step per column).
//
// Filtration (readings; the paper gives no H1 details): edges in the H0
// order (delta, j, i) with their grades; a triangle enters with its latest
// edge q (the last of its three edges in that order) and has q's grade;
// triangles are ordered by (position of q, third vertex k), so triangle
// t lists the triangles of each edge q consecutively, k ascending.  Rows of
// the boundary matrix are edge positions, columns triangles; the low of a
// column is its largest edge position.  A reduced column with low e pairs e
// with the triangle: the interval [grade(e), grade(triangle)); zero-length
// intervals are not bars.
//
// Layout.  Stored columns are dense over the E edges: row e of the table
// holds the reduced column whose low is e in words 0 .. e/64 of a row of
// LWE = ceil(E/64) words (a column has no bit above its low); owner[e] is the
// triangle stored there, -1 while the row is free, so rows are never read
// before they are written and the table needs no clearing.  A column being
// reduced lives in the registers of one wavefront: word w in lane w % 64,
// slot w / 64.
//
// Emergent pairs.  The latest edge q of a triangle closes a cycle (the
// triangle's other two edges already join q's endpoints), so it never kills
// an H0 class; and no earlier triangle can have low q (all its edges precede
// q).  Hence the first triangle of each edge q reduces to nothing: its
// column stops at once on the free row q and is stored there unchanged.
// Every such pair is written into the table before any reduction, which the
// sequential order would also have done before any later column reads it.
// The remaining columns are then reduced side by side in rounds, as for H0:
// each walks against the table as committed so far; a column that reaches
// zero is final; a survivor stops on a free row L; survivors before the first
// survivor whose low repeats another's commit (no earlier column can take
// their rows first: a walk only passes rows that were taken when the round
// began), the rest walk again next round.  A committing survivor repeats its
// walk (the rows it passes cannot change meanwhile) and writes its column.
#include <algorithm>

#include "ph0_internal.h"

namespace ph0 {

namespace {

constexpr uint64_t kNoLow = ~0ull;

__device__ inline int64_t colex(int64_t i, int64_t j) {  // i < j
  return j * (j - 1) / 2 + i;
}

__device__ inline int edge_pos(const int32_t* inv, int a, int b) {
  return a < b ? inv[colex(a, b)] : inv[colex(b, a)];
}

__device__ inline uint64_t rl64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Position -> (colex inverse, distance-change flag).
__global__ void k_h1_index(const uint64_t* __restrict__ keys, int64_t E, int ib,
                           int32_t* __restrict__ inv, uint32_t* __restrict__ flag) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= E) return;
  const uint64_t m = (1ull << ib) - 1ull;
  const uint64_t k = keys[q];
  const int64_t i = (int64_t)(k & m), j = (int64_t)((k >> ib) & m);
  inv[colex(i, j)] = (int32_t)q;
  flag[q] = (q == 0 || (k >> (2 * ib)) != (keys[q - 1] >> (2 * ib))) ? 1u : 0u;
}

// grade[q] = number of distance changes in 0..q (flags scanned exclusively).
__global__ void k_h1_grade(const uint64_t* __restrict__ keys, int64_t E, int ib,
                           uint32_t* __restrict__ grade) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= E) return;
  const uint32_t f = (q == 0 || (keys[q] >> (2 * ib)) != (keys[q - 1] >> (2 * ib))) ? 1u : 0u;
  grade[q] += f;
}

// Triangles whose latest edge is q: vertices k with both other edges earlier.
// mode 0 counts them into cnt[q]; mode 1 writes (q << 32 | k) at start[q] + r.
template <int MODE>
__global__ void k_h1_tris(const uint64_t* __restrict__ keys, int64_t E, int ib, int n,
                          const int32_t* __restrict__ inv, uint32_t* __restrict__ cnt,
                          uint64_t* __restrict__ tri) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= E) return;
  const uint64_t m = (1ull << ib) - 1ull;
  const int i = (int)(keys[q] & m), j = (int)((keys[q] >> ib) & m);
  uint32_t c = 0;
  const uint32_t base = MODE == 1 ? cnt[q] : 0u;
  for (int k = 0; k < n; ++k) {
    if (k == i || k == j) continue;
    if (edge_pos(inv, i, k) < q && edge_pos(inv, j, k) < q) {
      if (MODE == 1) tri[base + c] = ((uint64_t)q << 32) | (uint32_t)k;
      ++c;
    }
  }
  if (MODE == 0) cnt[q] = c;
}

// The three edge positions of triangle t (e2 = its latest edge).
__device__ inline void tri_edges(const uint64_t* tri, const uint64_t* keys, int ib,
                                 const int32_t* inv, int64_t t, int* e0, int* e1, int* e2) {
  const uint64_t v = tri[t];
  const int q = (int)(v >> 32), k = (int)(uint32_t)v;
  const uint64_t m = (1ull << ib) - 1ull;
  const int i = (int)(keys[q] & m), j = (int)((keys[q] >> ib) & m);
  *e0 = edge_pos(inv, i, k);
  *e1 = edge_pos(inv, j, k);
  *e2 = q;
}

// Emergent pairs: row q <- the boundary of the first triangle of q (one wave
// per edge q, lanes over the row's words), owner[q] <- that triangle.
__global__ __launch_bounds__(256) void k_h1_emergent(const uint64_t* __restrict__ tri,
                                                     const uint64_t* __restrict__ keys, int ib,
                                                     const int32_t* __restrict__ inv,
                                                     const uint32_t* __restrict__ cnt,
                                                     const uint32_t* __restrict__ start, int64_t E,
                                                     int64_t LWE, uint64_t* __restrict__ table,
                                                     int32_t* __restrict__ owner) {
  const int64_t q = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (q >= E) return;
  if (cnt[q] == 0) {
    if (lane == 0) owner[q] = -1;
    return;
  }
  const int64_t t = start[q];
  int e0, e1, e2;
  tri_edges(tri, keys, ib, inv, t, &e0, &e1, &e2);
  uint64_t* row = table + q * LWE;
  const int64_t nw = q / 64 + 1;
  for (int64_t w = lane; w < nw; w += 64) {
    uint64_t v = 0;
    if (w == e0 / 64) v ^= 1ull << (e0 & 63);
    if (w == e1 / 64) v ^= 1ull << (e1 & 63);
    if (w == e2 / 64) v ^= 1ull << (e2 & 63);
    row[w] = v;
  }
  if (lane == 0) owner[q] = (int32_t)t;
}

// Dense column of one wavefront.
template <int WPL>
struct WCol {
  uint64_t c[WPL];
};

template <int WPL>
__device__ inline void wcol_set(WCol<WPL>& x, int b, int lane) {
  const int w = b >> 6;
#pragma unroll
  for (int s = 0; s < WPL; ++s)
    if (w == s * 64 + lane) x.c[s] ^= 1ull << (b & 63);
}

// Highest set bit of the column among words < nw (-1 if none).
template <int WPL>
__device__ inline int wcol_low(const WCol<WPL>& x, int nw) {
  int low = -1;
#pragma unroll
  for (int s = WPL - 1; s >= 0; --s) {
    if (low < 0 && s * 64 < nw) {
      const uint64_t m = __ballot(x.c[s] != 0);
      if (m) {
        const int L = 63 - __builtin_clzll(m);
        const uint64_t word = rl64(x.c[s], L);
        low = (s * 64 + L) * 64 + 63 - __builtin_clzll(word);
      }
    }
  }
  return low;
}

// Continue reducing the column `x`, whose low is `low`, against the table:
// returns its final low (-1 for zero) and adds the additions to *adds.  Each
// addition cancels the current low, so the low falls at every step; a row
// whose top bit is not its index (a corrupt table) ends the walk with -2.
template <int WPL>
__device__ inline int h1_reduce(const uint64_t* table, const int32_t* owner, int64_t LWE,
                                int low, int lane, WCol<WPL>& x, int64_t* adds) {
  int64_t a = 0;
  while (true) {
    const int o = __builtin_amdgcn_readfirstlane(owner[low]);
    if (o < 0) break;  // row `low` is free: a survivor
    const uint64_t* row = table + (int64_t)low * LWE;
    const int nw = low / 64 + 1;
#pragma unroll
    for (int s = 0; s < WPL; ++s) {
      const int w = s * 64 + lane;
      if (w < nw) x.c[s] ^= row[w];
    }
    ++a;
    const int next = __builtin_amdgcn_readfirstlane(wcol_low<WPL>(x, nw));
    if (next >= low) {
      low = -2;
      break;
    }
    low = next;
    if (low < 0) break;  // zero column
  }
  *adds += a;
  return low;
}

// Words 0 .. low/64 of a column to or from the column store.
template <int WPL>
__device__ inline void wcol_put(const WCol<WPL>& x, uint64_t* dst, int low, int lane) {
  const int nw = low / 64 + 1;
#pragma unroll
  for (int s = 0; s < WPL; ++s) {
    const int w = s * 64 + lane;
    if (w < nw) dst[w] = x.c[s];
  }
}

template <int WPL>
__device__ inline void wcol_get(WCol<WPL>& x, const uint64_t* src, int low, int lane) {
  const int nw = low / 64 + 1;
#pragma unroll
  for (int s = 0; s < WPL; ++s) {
    const int w = s * 64 + lane;
    x.c[s] = w < nw ? src[w] : 0ull;
  }
}

// Walk triangle t's column against the table from its boundary; returns its
// final low (-1 for zero, -2 for a corrupt table) and the additions.
template <int WPL>
__device__ inline int h1_walk(const uint64_t* tri, const uint64_t* keys, int ib,
                              const int32_t* inv, const uint64_t* table, const int32_t* owner,
                              int64_t LWE, int64_t t, int lane, WCol<WPL>& x, int64_t* adds) {
  int e0, e1, e2;
  tri_edges(tri, keys, ib, inv, t, &e0, &e1, &e2);
  e0 = __builtin_amdgcn_readfirstlane(e0);
  e1 = __builtin_amdgcn_readfirstlane(e1);
  e2 = __builtin_amdgcn_readfirstlane(e2);
#pragma unroll
  for (int s = 0; s < WPL; ++s) x.c[s] = 0;
  wcol_set(x, e0, lane);
  wcol_set(x, e1, lane);
  wcol_set(x, e2, lane);
  return h1_reduce<WPL>(table, owner, LWE, e2, lane, x, adds);
}

// Per-wave addition and walk counts -> one atomic each per block.
__device__ inline void h1_flush(int64_t adds, int64_t walks, H1Ctl* ctl) {
  __shared__ unsigned long long s_cnt[2];
  if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    if (adds) atomicAdd(&s_cnt[0], (unsigned long long)adds);
    if (walks) atomicAdd(&s_cnt[1], (unsigned long long)walks);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_cnt[0]) atomicAdd((unsigned long long*)&ctl->additions, s_cnt[0]);
    if (s_cnt[1]) atomicAdd((unsigned long long*)&ctl->walks, s_cnt[1]);
  }
}

// Survivors live in one array S of (t << 32) | low entries for the whole
// reduction; an entry whose column has become final (zero, or stored) is
// marked kDead.  minc[L] is the smallest triangle among the live survivors
// on row L.  Rows only fill, and a walk passes only rows taken before it
// stopped, so a live survivor's walk stays valid until its own row L is
// taken; then it walks again.  A round is: the first survivor that is not
// the smallest on its row (the first duplicate); survivors before it commit
// (each is the smallest on its row, and no earlier column can take its row
// first); the survivors on rows just taken walk again.  The smallest live
// survivor always commits, so every round makes progress.
constexpr uint32_t kDead = 0xFFFFFFFFu;

// Round 0: walk every triangle that is not the first of its edge.  Zero
// columns are final; survivors are appended to S and lower minc[low].
template <int WPL>
__global__ __launch_bounds__(256) void k_h1_walk0(const uint64_t* __restrict__ tri,
                                                  const uint64_t* __restrict__ keys, int ib,
                                                  const int32_t* __restrict__ inv,
                                                  const uint32_t* __restrict__ start,
                                                  const uint64_t* __restrict__ table,
                                                  const int32_t* __restrict__ owner, int64_t LWE,
                                                  uint64_t* __restrict__ S,
                                                  uint64_t* __restrict__ minc,
                                                  uint64_t* __restrict__ store,
                                                  uint32_t* __restrict__ sadds, int64_t cap,
                                                  H1Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t items = ctl->T;
  const int64_t wid = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  const int64_t wtot = (int64_t)gridDim.x * (blockDim.x / 64);
  int64_t adds = 0, walks = 0;
  for (int64_t t = wid; t < items; t += wtot) {
    const int q = (int)(tri[t] >> 32);
    if ((int64_t)start[q] == t) continue;  // an emergent pair, already stored
    WCol<WPL> x;
    int64_t a = 0;
    const int low = h1_walk<WPL>(tri, keys, ib, inv, table, owner, LWE, t, lane, x, &a);
    ++walks;
    if (low == -2) {
      if (lane == 0) atomicOr(&ctl->err, 2);
      continue;
    }
    if (low < 0) {
      adds += a;  // final: a zero column
      continue;
    }
    uint32_t k = 0;
    if (lane == 0) {
      k = (uint32_t)atomicAdd((unsigned long long*)&ctl->nsurv, 1ull);
      S[k] = ((uint64_t)t << 32) | (uint32_t)low;
      atomicMin((unsigned long long*)&minc[low], (unsigned long long)t);
    }
    k = __builtin_amdgcn_readfirstlane(k);
    if (k < cap) {  // keep the column and its additions so far
      wcol_put<WPL>(x, store + (int64_t)k * LWE, low, lane);
      if (lane == 0) sadds[k] = (uint32_t)a;
    }
  }
  h1_flush(adds, walks, ctl);
}

// First live survivor that is not the smallest on its row (thread per entry).
__global__ __launch_bounds__(256) void k_h1_decide(const uint64_t* __restrict__ S,
                                                   const uint64_t* __restrict__ minc,
                                                   H1Ctl* ctl) {
  __shared__ unsigned long long s_min;
  if (threadIdx.x == 0) s_min = kNoLow;
  __syncthreads();
  const int64_t ns = ctl->nsurv;
  uint64_t best = kNoLow;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ns;
       k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = S[k];
    const uint32_t low = (uint32_t)v;
    if (low == kDead) continue;
    const uint64_t t = v >> 32;
    if (minc[low] != t && t < best) best = t;
  }
  if (best != kNoLow) atomicMin(&s_min, (unsigned long long)best);
  __syncthreads();
  if (threadIdx.x == 0 && s_min != kNoLow)
    atomicMin((unsigned long long*)&ctl->firstdup, s_min);
}

// Survivors before the first duplicate leave S for the commit list.
__global__ __launch_bounds__(256) void k_h1_pick(uint64_t* __restrict__ S,
                                                 uint64_t* __restrict__ clist, H1Ctl* ctl) {
  const int64_t ns = ctl->nsurv;
  const uint64_t fd = ctl->firstdup;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ns;
       k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = S[k];
    if ((uint32_t)v == kDead || (v >> 32) >= fd) continue;
    const unsigned long long c = atomicAdd((unsigned long long*)&ctl->ncommit, 1ull);
    clist[c] = ((uint64_t)k << 32) | (uint32_t)v;
    S[k] = v | kDead;
  }
}

// Each picked survivor stores its column in row `low`: the kept column, or,
// for a survivor beyond the store, its walk repeated from the boundary (the
// rows it passes are unchanged).  One wave per survivor.
template <int WPL>
__global__ __launch_bounds__(256) void k_h1_commit(const uint64_t* __restrict__ tri,
                                                   const uint64_t* __restrict__ keys, int ib,
                                                   const int32_t* __restrict__ inv,
                                                   uint64_t* __restrict__ table,
                                                   int32_t* __restrict__ owner, int64_t LWE,
                                                   const uint64_t* __restrict__ clist,
                                                   const uint64_t* __restrict__ S,
                                                   const uint64_t* __restrict__ store,
                                                   const uint32_t* __restrict__ sadds,
                                                   int64_t cap, H1Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t nc = ctl->ncommit;
  const int64_t wid = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  const int64_t wtot = (int64_t)gridDim.x * (blockDim.x / 64);
  int64_t adds = 0, walks = 0;
  for (int64_t c = wid; c < nc; c += wtot) {
    const uint32_t k = (uint32_t)(clist[c] >> 32);
    const int low = (int)(uint32_t)clist[c];
    const int64_t t = (int64_t)(S[k] >> 32);
    WCol<WPL> x;
    int64_t a = 0;
    if (k < cap) {
      wcol_get<WPL>(x, store + (int64_t)k * LWE, low, lane);
      a = sadds[k];
    } else {
      const int l2 = h1_walk<WPL>(tri, keys, ib, inv, table, owner, LWE, t, lane, x, &a);
      ++walks;
      if (l2 != low) {  // a repeated walk must end where the first did
        if (lane == 0) atomicOr(&ctl->err, 1);
        continue;
      }
    }
    adds += a;
    uint64_t* row = table + (int64_t)low * LWE;
    const int nw = low / 64 + 1;
#pragma unroll
    for (int q = 0; q < WPL; ++q) {
      const int w = q * 64 + lane;
      if (w < nw) row[w] = x.c[q];
    }
    __threadfence();
    if (lane == 0) owner[low] = (int32_t)t;
  }
  h1_flush(adds, walks, ctl);
}

// Live survivors whose row was just taken go to the walk list (one global
// atomic per block: a block-wide count, then a scan inside the block).
__global__ __launch_bounds__(256) void k_h1_mark(const uint64_t* __restrict__ S,
                                                 const int32_t* __restrict__ owner,
                                                 uint32_t* __restrict__ wlist, H1Ctl* ctl) {
  __shared__ uint32_t s_wave[4];
  __shared__ unsigned long long s_base;
  const int64_t ns = ctl->nsurv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t k0 = blockIdx.x * (int64_t)blockDim.x; k0 < ns;
       k0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    bool take = false;
    if (k < ns) {
      const uint64_t v = S[k];
      take = (uint32_t)v != kDead && owner[(uint32_t)v] >= 0;
    }
    const uint64_t m = __ballot(take);
    if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
      s_base = tot ? atomicAdd((unsigned long long*)&ctl->nwalk, (unsigned long long)tot) : 0;
    }
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    if (take)
      wlist[s_base + before + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)k;
    __syncthreads();
  }
}

// Survivors on taken rows continue: a kept column resumes at its row (now
// taken, so the stored column there is added next), a survivor beyond the
// store walks again from its boundary.  Zero columns die, the others move
// to their new (free) row.  One wave per survivor.
template <int WPL>
__global__ __launch_bounds__(256) void k_h1_rewalk(const uint64_t* __restrict__ tri,
                                                   const uint64_t* __restrict__ keys, int ib,
                                                   const int32_t* __restrict__ inv,
                                                   const uint64_t* __restrict__ table,
                                                   const int32_t* __restrict__ owner,
                                                   int64_t LWE, uint64_t* __restrict__ S,
                                                   const uint32_t* __restrict__ wlist,
                                                   uint64_t* __restrict__ minc,
                                                   uint64_t* __restrict__ store,
                                                   uint32_t* __restrict__ sadds, int64_t cap,
                                                   H1Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ctl->nwalk;
  const int64_t wid = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  const int64_t wtot = (int64_t)gridDim.x * (blockDim.x / 64);
  int64_t adds = 0, walks = 0;
  for (int64_t i = wid; i < nw; i += wtot) {
    const uint32_t k = wlist[i];
    const uint64_t v = S[k];
    const uint64_t t = v >> 32;
    WCol<WPL> x;
    int64_t a = 0;
    int low;
    if (k < cap) {
      const int old = (int)(uint32_t)v;
      wcol_get<WPL>(x, store + (int64_t)k * LWE, old, lane);
      a = sadds[k];
      low = h1_reduce<WPL>(table, owner, LWE, old, lane, x, &a);
    } else {
      low = h1_walk<WPL>(tri, keys, ib, inv, table, owner, LWE, (int64_t)t, lane, x, &a);
    }
    ++walks;
    if (low == -2) {
      if (lane == 0) atomicOr(&ctl->err, 2);
      continue;
    }
    if (low < 0) {
      adds += a;
      if (lane == 0) S[k] = (t << 32) | kDead;
      continue;
    }
    if (k < cap) {
      wcol_put<WPL>(x, store + (int64_t)k * LWE, low, lane);
      if (lane == 0) sadds[k] = (uint32_t)a;
    }
    if (lane == 0) {
      S[k] = (t << 32) | (uint32_t)low;
      atomicMin((unsigned long long*)&minc[low], (unsigned long long)t);
    }
  }
  h1_flush(adds, walks, ctl);
}

// End of a round: counters for the next one (k_h1_live then recounts).
// Accessed through a volatile pointer: plain accesses let the compiler read
// the counters with scalar loads and issue the vector stores that clear them
// before those loads have returned.
__global__ void k_h1_round_end(H1Ctl* ctl_) {
  volatile H1Ctl* ctl = ctl_;
  const int64_t nc = ctl->ncommit;
  const int64_t r = ctl->round;
  ctl->pivots = ctl->pivots + nc;
  ctl->round = r + 1;
  ctl->live = 0;
  ctl->firstdup = kNoLow;
  ctl->ncommit = 0;
  ctl->nwalk = 0;
}

// Live count after a round's walks: entries not marked dead.
__global__ __launch_bounds__(256) void k_h1_live(const uint64_t* __restrict__ S, H1Ctl* ctl) {
  __shared__ unsigned long long s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const int64_t ns = ctl->nsurv;
  uint32_t c = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ns;
       k += (int64_t)gridDim.x * blockDim.x)
    c += (uint32_t)S[k] != kDead;
  if (c) atomicAdd(&s_n, (unsigned long long)c);
  __syncthreads();
  if (threadIdx.x == 0 && s_n) atomicAdd((unsigned long long*)&ctl->live, s_n);
}

// Bars: for every stored row q, (grade(q), grade(latest edge of its
// triangle)) if the two differ, packed as birth << 20 | death for the sort.
__global__ void k_h1_bars(const int32_t* __restrict__ owner, const uint64_t* __restrict__ tri,
                          const uint32_t* __restrict__ grade, int64_t E,
                          uint64_t* __restrict__ out, H1Ctl* ctl) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= E) return;
  const int32_t o = owner[q];
  if (o < 0) return;
  const uint32_t b = grade[q], d = grade[(int64_t)(tri[o] >> 32)];
  atomicAdd((unsigned long long*)&ctl->stored, 1ull);
  if (b == d) return;
  const unsigned long long k = atomicAdd((unsigned long long*)&ctl->nbars, 1ull);
  out[k] = ((uint64_t)b << 20) | d;
}

__global__ void k_h1_bars_out(const uint64_t* __restrict__ sorted, int64_t m,
                              uint32_t* __restrict__ bars) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  bars[2 * k] = (uint32_t)(sorted[k] >> 20);
  bars[2 * k + 1] = (uint32_t)(sorted[k] & 0xFFFFF);
}

__global__ void k_h1_owner_out(const int32_t* __restrict__ owner, int64_t E,
                               int64_t* __restrict__ out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < E) out[q] = owner[q];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <int WPL>
hipError_t first_round(const H1Args& a, hipStream_t s) {
  const int64_t cap = (int64_t)a.cus * 8;
  const int64_t wb = std::min<int64_t>(cap, std::max<int64_t>(1, (a.T + 3) / 4));
  hipLaunchKernelGGL(k_h1_walk0<WPL>, dim3((unsigned)wb), dim3(256), 0, s, a.tri, a.keys, a.ib,
                     a.inv, a.start, a.table, a.owner, a.LWE, a.surv, a.lowc, a.store, a.sadds,
                     a.cap, a.ctl);
  hipLaunchKernelGGL(k_h1_live, dim3((unsigned)a.cus), dim3(256), 0, s, a.surv, a.ctl);
  return hipGetLastError();
}

template <int WPL>
hipError_t next_round(const H1Args& a, hipStream_t s) {
  const int64_t cap = (int64_t)a.cus * 8;
  const unsigned scan =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (a.nsurv_host + 255) / 256));
  const unsigned pass = scan;
  hipLaunchKernelGGL(k_h1_decide, dim3(scan), dim3(256), 0, s, a.surv, a.lowc, a.ctl);
  hipLaunchKernelGGL(k_h1_pick, dim3(scan), dim3(256), 0, s, a.surv, a.clist, a.ctl);
  hipLaunchKernelGGL(k_h1_commit<WPL>, dim3((unsigned)cap), dim3(256), 0, s, a.tri, a.keys, a.ib,
                     a.inv, a.table, a.owner, a.LWE, a.clist, a.surv, a.store, a.sadds, a.cap,
                     a.ctl);
  hipLaunchKernelGGL(k_h1_mark, dim3(scan), dim3(256), 0, s, a.surv, a.owner, a.wlist, a.ctl);
  hipLaunchKernelGGL(k_h1_rewalk<WPL>, dim3((unsigned)cap), dim3(256), 0, s, a.tri, a.keys, a.ib,
                     a.inv, a.table, a.owner, a.LWE, a.surv, a.wlist, a.lowc, a.store, a.sadds,
                     a.cap, a.ctl);
  hipLaunchKernelGGL(k_h1_round_end, dim3(1), dim3(1), 0, s, a.ctl);
  hipLaunchKernelGGL(k_h1_live, dim3(pass), dim3(256), 0, s, a.surv, a.ctl);
  return hipGetLastError();
}

}  // namespace

int h1_words_per_lane(int64_t LWE) {
  const int64_t need = (LWE + 63) / 64;
  int w = 1;
  while (w < need) w <<= 1;
  return w;
}

hipError_t launch_h1_setup(const H1Args& a, hipStream_t s) {
  const int64_t E = a.E;
  hipLaunchKernelGGL(k_h1_index, dim3(blocks_for(E, 256)), dim3(256), 0, s, a.keys, E, a.ib,
                     a.inv, a.grade);
  hipError_t e = launch_scan_u32(a.grade, E, a.scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_h1_grade, dim3(blocks_for(E, 256)), dim3(256), 0, s, a.keys, E, a.ib,
                     a.grade);
  hipLaunchKernelGGL(k_h1_tris<0>, dim3(blocks_for(E, 256)), dim3(256), 0, s, a.keys, E, a.ib,
                     (int)a.n, a.inv, a.cnt, (uint64_t*)nullptr);
  // start = exclusive scan of the counts (one extra entry holds T)
  e = hipMemcpyAsync(a.start, a.cnt, 4 * (size_t)E, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(a.start + E, 0u, 1, s);
  if (e != hipSuccess) return e;
  e = launch_scan_u32(a.start, E + 1, a.scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_h1_tris<1>, dim3(blocks_for(E, 256)), dim3(256), 0, s, a.keys, E, a.ib,
                     (int)a.n, a.inv, a.start, a.tri);
  hipLaunchKernelGGL(k_h1_emergent, dim3(blocks_for(E, 4)), dim3(256), 0, s, a.tri, a.keys, a.ib,
                     a.inv, a.cnt, a.start, E, a.LWE, a.table, a.owner);
  e = launch_fill_u64(a.lowc, kNoLow, E, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_h1_round(const H1Args& a, bool first, hipStream_t s) {
  switch (h1_words_per_lane(a.LWE)) {
#define H1_CASE(W) \
  case W: return first ? first_round<W>(a, s) : next_round<W>(a, s);
    H1_CASE(1)
    H1_CASE(2)
    H1_CASE(4)
    H1_CASE(8)
    H1_CASE(16)
    H1_CASE(32)
#undef H1_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_h1_bars(const H1Args& a, uint64_t* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_h1_bars, dim3(blocks_for(a.E, 256)), dim3(256), 0, s, a.owner, a.tri,
                     a.grade, a.E, packed, a.ctl);
  return hipGetLastError();
}

hipError_t launch_h1_bars_out(const uint64_t* sorted, int64_t m, uint32_t* bars, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_h1_bars_out, dim3(blocks_for(m, 256)), dim3(256), 0, s, sorted, m, bars);
  return hipGetLastError();
}

hipError_t launch_h1_owner_out(const int32_t* owner, int64_t E, int64_t* out, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_h1_owner_out, dim3(blocks_for(E, 256)), dim3(256), 0, s, owner, E, out);
  return hipGetLastError();
}

}  // namespace ph0
