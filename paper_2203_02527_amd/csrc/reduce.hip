// reduce.hip -- steps 4-5 of the GPU pipeline (Section 4: "for each diagonal
// entry of the matrix: reduction step"): column reduction over F2 of the
// vertex-by-edge boundary matrix, left to right, with pivots (Section 2).
//
// Data layout.  The pivot table is dense and bit-packed: row r (the stored
// column whose low is r) holds N bits in LW = ceil(N/64) 64-bit words at
// table[r * LW].  A stored column has bits only at rows <= r, so a lookup
// reads words 0 .. r/64 only.  Bit r of row r doubles as the "slot r is
// taken" flag (the table starts zeroed).
//
// One column, one lane group.  A group of G lanes (G = 64 for N > 2048)
// holds the current column as a dense register bitset, WPL words per lane.
// Each step loads the stored column of the current low, XORs it in, and
// finds the new low: per-lane highest set bit, a ballot over the group, and
// a shuffle from the highest nonzero lane.  Over F2 every column met on the
// way has exactly two nonzero rows, which the kernel checks.
//
// Rounds.  A window of consecutive sorted columns [F, Wend) is reduced side
// by side against the table as committed so far (every slot there belongs to
// an earlier column, so each step is one the sequential reduction also
// takes).  A column that stops on an empty slot r is a survivor with low r.
// The sequential order is then restored exactly:
//   * survivors before the first survivor whose low repeats an earlier
//     survivor's low commit (none of them would have met another's slot);
//   * a later survivor also commits if no earlier survivor touches the
//     component of its low r, i.e. neither low nor the root of its other row
//     equals r: then no earlier column can take slot r first, and its walk
//     is final;
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

__device__ inline uint64_t enc(int64_t round, int64_t p) {
  return ((uint64_t)(0xFFFFFF - (round & 0xFFFFFF)) << 40) | (uint64_t)p;
}

__device__ inline uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = __shfl((uint32_t)v, src, 64);
  const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Largest value of `hb` (>= 0 means present) across the lanes of a group.
template <int G>
__device__ inline int group_max_index(int hb, int gbase) {
  uint64_t m = __ballot(hb >= 0);
  if constexpr (G < 64) m = (m >> gbase) & ((1ull << G) - 1ull);
  if (m == 0) return -1;
  const int top = 63 - __clzll(m);
  return __shfl(hb, gbase + top, 64);
}

template <int WPL>
__device__ inline int lane_highest(const uint64_t (&w)[WPL], int gl) {
  int hb = -1;
#pragma unroll
  for (int k = WPL - 1; k >= 0; --k)
    if (hb < 0 && w[k] != 0) hb = (gl * WPL + k) * 64 + 63 - __clzll(w[k]);
  return hb;
}

template <int G>
__device__ inline bool group_any(bool v, int gbase) {
  uint64_t m = __ballot(v);
  if constexpr (G < 64) m = (m >> gbase) & ((1ull << G) - 1ull);
  return m != 0;
}

// Load words 0..r/64 of stored column r into the group's registers; return
// whether slot r is taken (bit r set).
template <int G, int WPL>
__device__ inline bool load_row(const uint64_t* __restrict__ table, int64_t LW, int r, int gl,
                                int gbase, uint64_t (&row)[WPL]) {
  const int top = r >> 6;
  const uint64_t* rp = table + (int64_t)r * LW;
  uint64_t mine = 0;
#pragma unroll
  for (int k = 0; k < WPL; ++k) {
    const int widx = gl * WPL + k;
    row[k] = widx <= top ? rp[widx] : 0ull;
    if (widx == top) mine = row[k];
  }
  const uint64_t topword = shfl64(mine, gbase + top / WPL);
  return (topword >> (r & 63)) & 1ull;
}

template <int WPL>
__device__ inline void clear_bit(uint64_t (&w)[WPL], int gl, int bit) {
#pragma unroll
  for (int k = 0; k < WPL; ++k)
    if (gl * WPL + k == (bit >> 6)) w[k] &= ~(1ull << (bit & 63));
}

template <int G, int WPL>
__global__ __launch_bounds__(256) void k_walk(const uint64_t* __restrict__ skeys, int ib,
                                              int64_t LW, const uint64_t* __restrict__ table,
                                              Ring ring, int64_t Wcap, uint64_t* lowc,
                                              uint64_t* touch, RedCtl* ctl) {
  if (ctl->done) return;
  const int64_t F = ctl->F, Wend = ctl->Wend, round = ctl->round;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int64_t gpb = blockDim.x / G;
  const int64_t gid = blockIdx.x * gpb + threadIdx.x / G;
  const int64_t gtotal = (int64_t)gridDim.x * gpb;
  const uint64_t imask = (1ull << ib) - 1ull;

  int64_t adds = 0, finds = 0, words = 0;
  int32_t bad = 0;
  for (int64_t p = F + gid; p < Wend; p += gtotal) {
    const int64_t k = p % Wcap;
    int32_t a, r, rlo, st;
    if (ring.tag[k] != p) {
      const uint64_t key = skeys[p];
      a = (int32_t)(key & imask);
      r = (int32_t)((key >> ib) & imask);
      rlo = a;
      st = kActive;
    } else {
      st = ring.st[k];
      if ((st & 3) != kActive) continue;
      a = ring.a[k];
      r = ring.r[k];
      rlo = ring.rlo[k];
    }
    uint64_t col[WPL];
#pragma unroll
    for (int q = 0; q < WPL; ++q) {
      const int widx = gl * WPL + q;
      col[q] = (widx == (a >> 6) ? 1ull << (a & 63) : 0ull) ^
               (widx == (r >> 6) ? 1ull << (r & 63) : 0ull);
    }
    int moved = 0;
    bool zero = false;
    while (true) {
      uint64_t row[WPL];
      words += (r >> 6) + 1;
      if (!load_row<G, WPL>(table, LW, r, gl, gbase, row)) break;
#pragma unroll
      for (int q = 0; q < WPL; ++q) col[q] ^= row[q];
      ++moved;
      const int nr = group_max_index<G>(lane_highest<WPL>(col, gl), gbase);
      if (nr < 0) {
        zero = true;
        break;
      }
      if (nr >= r) {  // lows must strictly decrease; a corrupt table ends the walk
        bad = 1;
        zero = true;
        break;
      }
      r = nr;
    }
    adds += moved;
    int32_t status = kActive;
    if (zero) {
      status = kZero;
    } else {
      clear_bit<WPL>(col, gl, r);
      const int na = group_max_index<G>(lane_highest<WPL>(col, gl), gbase);
      if (na >= 0) clear_bit<WPL>(col, gl, na);
      bool rest = false;
#pragma unroll
      for (int q = 0; q < WPL; ++q) rest |= col[q] != 0;
      if (na < 0 || group_any<G>(rest, gbase)) bad = 1;
      a = na < 0 ? 0 : na;
      // Root of row a in the current forest: follow stored columns down.
      int v = moved ? a : rlo;
      while (true) {
        uint64_t row[WPL];
        words += (v >> 6) + 1;
        if (!load_row<G, WPL>(table, LW, v, gl, gbase, row)) break;
        clear_bit<WPL>(row, gl, v);
        const int c = group_max_index<G>(lane_highest<WPL>(row, gl), gbase);
        ++finds;
        if (c < 0 || c >= v) {  // a stored column needs a second, smaller row
          bad = 1;
          break;
        }
        v = c;
      }
      rlo = v;
      if (gl == 0) {
        const uint64_t e = enc(round, p);
        atomicMin((unsigned long long*)&lowc[r], (unsigned long long)e);
        atomicMin((unsigned long long*)&touch[r], (unsigned long long)e);
        atomicMin((unsigned long long*)&touch[rlo], (unsigned long long)e);
      }
    }
    if (gl == 0) {
      const int32_t steps = (ring.tag[k] == p ? (st >> 2) : 0) + moved;
      ring.a[k] = a;
      ring.r[k] = r;
      ring.rlo[k] = rlo;
      ring.st[k] = status | (steps << 2);
      ring.tag[k] = p;
    }
  }
  // One atomic per group leader with work.
  if (gl == 0 && (adds | finds | words)) {
    atomicAdd((unsigned long long*)&ctl->additions_all, (unsigned long long)adds);
    atomicAdd((unsigned long long*)&ctl->find_steps, (unsigned long long)finds);
    atomicAdd((unsigned long long*)&ctl->words_read, (unsigned long long)words);
  }
  if (gl == 0 && bad) atomicOr(&ctl->err, 1);
}

__global__ __launch_bounds__(256) void k_decide(Ring ring, int64_t Wcap, const uint64_t* lowc,
                                                RedCtl* ctl) {
  if (ctl->done) return;
  const int64_t F = ctl->F, Wend = ctl->Wend, round = ctl->round;
  uint64_t best = kNoValue;
  for (int64_t p = F + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < Wend;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = p % Wcap;
    if ((ring.st[k] & 3) != kActive) continue;
    if (lowc[ring.r[k]] != enc(round, p) && (uint64_t)p < best) best = (uint64_t)p;
  }
  if (best != kNoValue)
    atomicMin((unsigned long long*)&ctl->firstdup[round & 1], (unsigned long long)best);
}

__global__ __launch_bounds__(256) void k_commit(Ring ring, int64_t Wcap, const uint64_t* touch,
                                                uint64_t* table, int64_t LW, int64_t* killer,
                                                RedCtl* ctl) {
  if (ctl->done) return;
  const int64_t F = ctl->F, Wend = ctl->Wend, round = ctl->round;
  const uint64_t fd = ctl->firstdup[round & 1];
  uint64_t stay = kNoValue;
  int64_t npiv = 0, last = -1;
  for (int64_t p = F + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < Wend;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = p % Wcap;
    const int32_t st = ring.st[k];
    if ((st & 3) != kActive) continue;
    const int32_t r = ring.r[k];
    if ((uint64_t)p < fd || touch[r] == enc(round, p)) {
      const int32_t a = ring.a[k];
      uint64_t* row = table + (int64_t)r * LW;
      if ((a >> 6) == (r >> 6)) {
        row[r >> 6] = (1ull << (r & 63)) | (1ull << (a & 63));
      } else {
        row[a >> 6] = 1ull << (a & 63);
        row[r >> 6] = 1ull << (r & 63);
      }
      killer[r] = p;
      ring.st[k] = (st & ~3) | kCommitted;
      ++npiv;
      last = p > last ? p : last;
    } else if ((uint64_t)p < stay) {
      stay = (uint64_t)p;
    }
  }
  if (npiv) {
    atomicAdd((unsigned long long*)&ctl->pivots, (unsigned long long)npiv);
    atomicMax((long long*)&ctl->E_eff, (long long)(last + 1));
  }
  if (stay != kNoValue)
    atomicMin((unsigned long long*)&ctl->newF[round & 1], (unsigned long long)stay);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->firstdup[(round + 1) & 1] = kNoValue;
    ctl->newF[(round + 1) & 1] = kNoValue;
  }
}

__global__ void k_advance(RedCtl* ctl, int64_t n, int64_t E, int64_t Wcap) {
  if (ctl->done) return;
  const int64_t round = ctl->round;
  const uint64_t nf = ctl->newF[round & 1];
  int64_t F = nf == kNoValue ? ctl->Wend : (int64_t)nf;
  int64_t Wend;
  if (ctl->pivots >= n - 1) {
    Wend = ctl->Wend < ctl->E_eff ? ctl->Wend : ctl->E_eff;
    if (F >= ctl->E_eff) ctl->done = 1;
  } else {
    Wend = F + Wcap < E ? F + Wcap : E;
    if (F >= E) {
      ctl->done = 1;
      ctl->err |= 2;
    }
  }
  ctl->F = F;
  ctl->Wend = Wend;
  if (Wend > ctl->maxWend) ctl->maxWend = Wend;
  ctl->round = round + 1;
}

__global__ void k_reduce_init(RedCtl* ctl, int64_t E, int64_t Wcap, int64_t n) {
  RedCtl c = {};
  c.F = 0;
  c.Wend = Wcap < E ? Wcap : E;
  c.maxWend = c.Wend;
  c.firstdup[0] = c.firstdup[1] = kNoValue;
  c.newF[0] = c.newF[1] = kNoValue;
  c.done = (n <= 1 || E == 0) ? 1 : 0;
  *ctl = c;
}

// Additions of columns at or after E_eff (walked before the last pivot was
// known) are not part of the sequential count; sum them for subtraction.
__global__ __launch_bounds__(256) void k_overshoot(Ring ring, int64_t Wcap, RedCtl* ctl) {
  const int64_t lo = ctl->E_eff, hi = ctl->maxWend;
  int64_t s = 0;
  for (int64_t p = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < hi;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = p % Wcap;
    if (ring.tag[k] == p) s += ring.st[k] >> 2;
  }
  if (s) atomicAdd((unsigned long long*)&ctl->additions_overshoot, (unsigned long long)s);
}

template <int G, int WPL>
void walk_launch(const RedArgs& a, hipStream_t s) {
  const int64_t gpb = 256 / G;
  int64_t blocks = (a.Wcap + gpb - 1) / gpb;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_walk<G, WPL>), dim3((unsigned)blocks), dim3(256), 0, s, a.skeys, a.ib,
                     a.LW, a.table, a.ring, a.Wcap, a.lowc, a.touch, a.ctl);
}

int scan_blocks(int64_t Wcap) {
  int64_t b = (Wcap + 255) / 256;
  if (b > 2048) b = 2048;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_reduce_init(const RedArgs& a, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u64(a.table, 0ull, a.n * a.LW, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(a.killer), ~0ull, a.n, s)) != hipSuccess)
    return e;
  if ((e = launch_fill_u64(a.lowc, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(a.touch, kNoValue, a.n, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(a.ring.tag), ~0ull, a.Wcap, s)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_reduce_init, dim3(1), dim3(1), 0, s, a.ctl, a.E, a.Wcap, a.n);
  return hipGetLastError();
}

hipError_t launch_reduce_round(const RedArgs& a, hipStream_t s) {
  // Lane-group shape: G lanes per column, WPL words per lane, G * WPL >= LW.
  const int64_t LW = a.LW;
  if (LW <= 1) walk_launch<1, 1>(a, s);
  else if (LW <= 2) walk_launch<2, 1>(a, s);
  else if (LW <= 4) walk_launch<4, 1>(a, s);
  else if (LW <= 8) walk_launch<8, 1>(a, s);
  else if (LW <= 16) walk_launch<16, 1>(a, s);
  else if (LW <= 32) walk_launch<32, 1>(a, s);
  else if (LW <= 64) walk_launch<64, 1>(a, s);
  else if (LW <= 128) walk_launch<64, 2>(a, s);
  else if (LW <= 256) walk_launch<64, 4>(a, s);
  else if (LW <= 512) walk_launch<64, 8>(a, s);
  else if (LW <= 1024) walk_launch<64, 16>(a, s);
  else return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int sb = scan_blocks(a.Wcap);
  hipLaunchKernelGGL(k_decide, dim3(sb), dim3(256), 0, s, a.ring, a.Wcap, a.lowc, a.ctl);
  hipLaunchKernelGGL(k_commit, dim3(sb), dim3(256), 0, s, a.ring, a.Wcap, a.touch, a.table,
                     a.LW, a.killer, a.ctl);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, a.ctl, a.n, a.E, a.Wcap);
  return hipGetLastError();
}

hipError_t launch_reduce_finish(const RedArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_overshoot, dim3(scan_blocks(a.Wcap)), dim3(256), 0, s, a.ring, a.Wcap,
                     a.ctl);
  return hipGetLastError();
}

}  // namespace ph0
