// ph0_internal.h -- declarations shared by the HIP translation units of the
// library (kernels and their launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ph0 {

constexpr int kMaxPasses = 8;
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint64_t kU64Max = ~0ull;

// Which key bits each LSD radix pass sorts on.
struct SortPlan {
  int passes;
  int shift[kMaxPasses];  // first key bit of the pass's digit
  int bits[kMaxPasses];   // digit width (1..8)
};

// State of the round-based reduction entering a round, resident in device
// memory (two copies, by the parity of the rounds launched: round k reads
// the state entering round k - 1 and writes the one entering round k).  A
// round works on "items": first the nA columns kept by the previous round's
// commit (listed in the commit workgroups' segments, in workgroup order),
// then the fresh columns [fresh_lo, fresh_hi) entering the window this round.
struct RedCtl {
  int64_t F;         // first column that is not final
  int64_t Wend;      // end of the window [F, Wend); Wend - F <= Wcap
  int64_t width;     // current window width (width_min .. Wcap)
  int64_t width_min; // base width
  int64_t maxWend;   // largest Wend ever used
  int64_t fresh_lo;  // columns entering this round
  int64_t fresh_hi;
  int64_t nA;        // kept columns carried into this round
  int64_t pivots;    // committed pivots
  int64_t E_eff;     // largest committed column + 1
  int64_t round;     // rounds completed
  int64_t additions_all;        // set by the finish step
  int64_t find_steps;           // set by the finish step
  int64_t words_read;           // set by the finish step
  int64_t additions_overshoot;  // additions of walked columns >= E_eff (finish step)
  int64_t E_lim;     // sorted columns available so far (a prefix of the order)
  int32_t done;
  int32_t err;        // bit 0: a walk met a stored row below its low (corrupt table);
                      // bit 1: ran out of columns
  int32_t need_more;  // every available column is final and pivots are missing
  int32_t pad;
};

// Per-column record of the reduction window, a ring indexed by p % Wcap:
// the status of the last walk (low 2 bits) | additions so far << 2.  (The
// rows of a column still active travel with it in the survivor and kept
// lists.)
struct Ring {
  int32_t* st;
};

enum : int32_t { kActive = 0, kZero = 1 };

// ---- launchers (each enqueues on `s`, returns hipError_t) ----

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
// Up to four small device -> host (pinned) copies in one launch.
struct Gather {
  const uint32_t* src[4];
  uint32_t* dst[4];
  int32_t words[4];
  int count = 0;
  void add(const void* from, void* to, size_t bytes) {
    if (count == 4) {  // full: launch_gather rejects the list
      count = 5;
      return;
    }
    if (count > 4) return;
    src[count] = static_cast<const uint32_t*>(from);
    dst[count] = static_cast<uint32_t*>(to);
    words[count] = (int32_t)(bytes / 4);
    ++count;
  }
};
hipError_t launch_gather(const Gather& g, hipStream_t s);

// Real coordinates onto the int16 grid 0..32767: q[k] = rint((x[k] - lo) *
// scale) in fp64; *err (cleared first) becomes nonzero when a value falls off
// the grid (a coordinate outside [lo, hi] for scale = 32767 / (hi - lo), or
// not finite).
hipError_t launch_quantize_f32(const float* x, int64_t count, double lo, double scale, int16_t* q,
                               int32_t* err, hipStream_t s);

// Per-dimension coordinate range -> bound on the squared distance.  When
// `norms` and `norms_done` are given and the points allow it (int8, rows of
// 16 * 2^k <= 1024 bytes, 16-byte aligned), the same pass also leaves the
// squared norms |x_i|^2 in norms[0..n) and sets *norms_done.  The launch
// that initialises the ranges also clears zero[0..zero_len) when given.
hipError_t launch_coord_range(const void* pts, int elem_bytes, int64_t n, int32_t d,
                              int32_t* minmax /* 2*d: lo[0..d) then hi[0..d) */,
                              hipStream_t s, int32_t* norms = nullptr,
                              bool* norms_done = nullptr, uint32_t* zero = nullptr,
                              int64_t zero_len = 0);

// Step 1: keys of all edges at colex positions, and the histogram of
// delta >> hist_shift over kHistBins bins (added into `hist`).  `norms`
// (n words) is scratch for the int8 Gram path.
constexpr int kHistBins = 2048;
// `hist_shift_dev`, when non-null, holds the shift on the device (written by
// launch_dist_shift) and takes the place of `hist_shift`.
hipError_t launch_keys(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib,
                       uint64_t* keys, bool use_mfma, int hist_shift, uint32_t* hist,
                       int32_t* norms, hipStream_t s, const int32_t* hist_shift_dev = nullptr);
// The histogram shift from the coordinate ranges (lo[0..d) then hi[0..d)):
// max(b - 11, 0) for b the bit length of sum_k (hi_k - lo_k)^2 (64 when the
// sum overflows), written to shift[0] on the device.
hipError_t launch_dist_shift(const int32_t* minmax, int32_t d, int32_t* shift, hipStream_t s);

// One pass of the key kernels over all tiles of the distance matrix.
//  * kKeysFull:  every key at its colex position, and the histogram;
//  * kKeysHist:  the histogram only, over every `sample`-th tile;
//  * kKeysCount: for the keys with dlo <= delta < dhi, their number per
//                (64-row band J, row j in the band, segment of tiles
//                I <= J), bands, then rows, then segments (key_count_len);
//  * kKeysEmit:  those keys again, each written at (the exclusive scan of
//                the counts at its (J, row, segment)) + (the kept keys of
//                its row in the segment's earlier tiles) + (its rank among
//                the kept keys of its row in the tile), i.e. in colex order.
// The selected keys of a distance range are thus written without ever
// storing the others: distances are recomputed, which costs a few MFMA
// instructions per tile, instead of 8 bytes of HBM traffic per edge.
enum : int { kKeysFull = 0, kKeysHist = 1, kKeysCount = 2, kKeysEmit = 3 };
struct KeyPass {
  int mode = kKeysFull;
  uint64_t* keys = nullptr;
  uint32_t* hist = nullptr;
  int hist_shift = 0;
  const int32_t* hist_shift_dev = nullptr;  // when set, the shift is read here
  int64_t sample = 1;
  uint64_t dlo = 0, dhi = 0;
  uint32_t* cnt = nullptr;
  int32_t* norms = nullptr;  // n words of scratch (int8 Gram path)
  bool norms_ready = false;  // norms already hold this cloud's |x_i|^2
};
hipError_t launch_keys_pass(const void* pts, int elem_bytes, int64_t n, int32_t d, int ib,
                            bool use_mfma, const KeyPass& kp, hipStream_t s);
// Entries of the count array: per (band, row, segment of 4 tiles) on the
// int8 MFMA path, per (band, row, tile) on the vector ALU path.
int64_t key_count_len(int64_t n, bool mfma);
// Exclusive prefix sum of v[0..len) in place; `totals` holds
// scan_totals_len(len) words of scratch.
int64_t scan_totals_len(int64_t len);
hipError_t launch_scan_u32(uint32_t* v, int64_t len, uint32_t* totals, hipStream_t s);
// Exclusive scans, in place, of `cols` arrays of `len` counts laid end to end
// (v + c * len), one workgroup each, in one launch; totals[c] receives each
// array's total.  For short arrays (a few tens of thousands of counts).
hipError_t launch_scan_columns(uint32_t* v, int64_t len, int cols, uint32_t* totals,
                               hipStream_t s);

// Step 2: one stable LSD pass in -> out by digit (key >> shift) & ((1<<bits)-1).
// `counts` holds radix_count_entries(count) words of scratch.
int64_t radix_tiles(int64_t count);
int64_t radix_count_entries(int64_t count);
// Keys with (key >> fshift) outside [flo, fhi) are skipped (neither counted
// nor written); `expect` is how many keys are kept (the output length).
struct KeyFilter {
  int fshift = 0;
  uint64_t flo = 0, fhi = ~0ull;
};
hipError_t launch_radix_pass(const uint64_t* in, uint64_t* out, int64_t count, int shift,
                             int bits, uint32_t* counts, int32_t* err, hipStream_t s,
                             KeyFilter f = KeyFilter(), int64_t expect = -1);

// Steps 4-5: round-based reduction.
constexpr int kMaxWalkBlocks = 512;  // walk (and commit) workgroups per round, at most
struct RedArgs {
  const uint64_t* skeys;
  int ib;
  int32_t nblocks;     // walk_blocks(Wcap)
  int32_t count;       // nonzero: the walks keep their counters (additions, root-find
                       // steps, table words) and the finish sums them and the
                       // overshoot; zero: those statistics are not formed
  int64_t n, E, Wcap;  // Wcap: ring capacity, a power of two
  int64_t width;       // base window width (<= Wcap)
  int64_t seg;         // walk_segment(Wcap): entries per workgroup segment
  int32_t* part;  // n: other row of the column stored with low r, -1 = free
  uint16_t* part16;  // part16_len(n): the same as 16-bit rows (0xFFFF = free), or
                     // null when n > kPart16MaxN
  int64_t* killer;
  uint64_t* lowc;   // n: round-tagged smallest survivor with low r
  uint64_t* touch;  // n: round-tagged smallest survivor whose other row has root r
  int64_t* act[2];  // kept columns, one segment per commit workgroup (by round parity)
  uint64_t* act_ra[2];  // beside each: its low r (high half) and other row a (low half)
  uint64_t* act_x[2];   // beside each: root of a last seen (high half), additions so far
  Ring ring;
  int64_t* surv;    // nblocks x seg: each walk workgroup's survivors
  uint64_t* surv_ra;  // nblocks x seg: beside each survivor, its low r (high half)
                      // and other row a (low half)
  uint64_t* surv_x;   // nblocks x seg: beside each survivor, the root of a (high half)
                      // and its additions so far (low half)
  uint32_t* scount; // nblocks: survivors per walk workgroup
  uint64_t* fdslot; // nblocks: each walk workgroup's smallest survivor whose low repeats
                    // an earlier survivor's low
  uint64_t* wstat;  // 3 x nblocks: each walk workgroup's additions, root-find steps and
                    // table words, summed by the finish step
  uint32_t* cslot;  // 4 x nblocks: each commit workgroup's pivots, columns kept, and, as
                    // offsets from the round's window start F, the end of its last
                    // pivot (0: none) and its first kept column (~0u: none)
  RedCtl* ctl;       // [2]: the round states, by parity of the rounds launched
  int32_t* werr;     // a walk met a stored row below its low (folded into err)
};
// Grid of the walk (and of the commit) and the segment entries per workgroup.
int walk_blocks(int64_t Wcap);
int64_t walk_segment(int64_t Wcap);
// Largest n whose table has a 16-bit mirror (staged in LDS by the walk).
constexpr int64_t kPart16MaxN = 32768;
int64_t part16_len(int64_t n);
// The state entering round `rounds` (after that many rounds were launched),
// once the walk of that round or launch_reduce_advance has run.
inline RedCtl* reduce_state(const RedArgs& a, int64_t rounds) { return a.ctl + (rounds & 1); }
// The state entering round 0.
hipError_t launch_reduce_init(const RedArgs& a, int64_t E_lim, hipStream_t s);
// More sorted columns are available: [old E_lim, E_lim) (after `rounds`
// rounds and launch_reduce_advance).
hipError_t launch_reduce_extend(const RedArgs& a, int64_t E_lim, int64_t rounds, hipStream_t s);
// Round `k` (the k-th launched, from 0): the walk, which first advances the
// state past round k - 1 unless `advanced` (round 0, or launch_reduce_advance
// ran since), then the commit.  When `ev_walk` is non-null its two events
// are recorded around the walk kernel.
hipError_t launch_reduce_round(const RedArgs& a, hipStream_t s, hipEvent_t* ev_walk, int64_t k,
                               bool advanced);
// The state entering round `rounds` on its own (one wave), also left in
// `publish` (pinned host memory) when given.
hipError_t launch_reduce_advance(const RedArgs& a, int64_t rounds, RedCtl* publish,
                                 hipStream_t s);
// Totals into the state entering round `rounds` (after launch_reduce_advance).
hipError_t launch_reduce_finish(const RedArgs& a, int64_t rounds, hipStream_t s);

// Steps 3 and 5 together, over the first E_eff sorted keys: the grade of a
// sorted position p is 1 + the number of distance changes in 1..p (dense
// ranks of D); the pivot columns, in sorted order, are the deaths in
// ascending order (grades only grow with p), so one ordered pass over the
// positions writes both the canonical barcode and the per-vertex deaths,
// with no sort.  `work` holds grades_work_bytes(E_eff) bytes; dbv may be the
// caller's or scratch (n words); bars may be null.  *distinct receives the
// device address of the number of distinct distances in the prefix, *pivots
// that of the pivot count (both in `work`, valid once the stream has run).
size_t grades_work_bytes(int64_t E_eff);
hipError_t launch_grades_and_bars(const uint64_t* skeys, int64_t E_eff, int shift,
                                  const int64_t* killer, int64_t n, void* work, uint32_t* dbv,
                                  uint32_t* bars, hipStream_t s, const uint32_t** distinct,
                                  const uint32_t** pivots);
hipError_t launch_pairs_detail(const int64_t* killer, const uint64_t* skeys, int ib,
                               const int32_t* part, int64_t n,
                               int64_t* killer_pos, uint64_t* killer_edge,
                               int64_t* killer_sqdist, int32_t* partner, hipStream_t s);


// Many small clouds, one persistent launch (one workgroup per cloud).
constexpr int kBatchMaxN = 512;     // largest cloud the fused kernel takes
constexpr int kBatchMaxPts = 8192;  // largest n * d it stages in LDS
struct BatchArgs {
  const void* pts;          // concatenated rows, n_total x d
  int elem_bytes;
  int32_t d;
  const int64_t* offsets;   // nclouds + 1 row offsets (device)
  const int32_t* order;     // processing order, largest first (device)
  int64_t nclouds;
  uint32_t* bars;           // 2 x n_total: (birth, death) per row
  uint64_t* scratch;        // per workgroup: 2 x emax keys
  uint32_t* grades;         // per workgroup: emax grades
  int64_t emax;             // largest edge count of any cloud
  uint32_t* queue;          // work counter, zero at launch
  int32_t* errs;            // per cloud, zero at launch
  int32_t chunk_mult[4];    // first chunk holds about chunk_mult[b] * n edges, for
                            // size buckets b: n <= 64, <= 128, <= 256, <= 512
  int64_t single_n = 0;     // > 0: one cloud of single_n rows, one workgroup, no queue,
                            // offsets or order; its status always goes to errs[0]
  int32_t digit_bits = 8;   // digit width of the chunk's radix passes (1..8)
  int32_t threads = 512;    // workgroup size: 512 or 1024 (8 or 16 waves per cloud)
};
// LDS bytes of one batched workgroup of `threads` threads.
size_t batched_shared_bytes(int threads);
hipError_t launch_batched(const BatchArgs& a, int blocks, hipStream_t s);

// H1: reduction of the edge-by-triangle boundary matrix (h1.hip).
constexpr int64_t kH1MaxN = 512;  // dense stored columns: E x ceil(E/64) words
constexpr int64_t kH1StoreBytes = int64_t(16) << 30;  // kept survivor columns, at most
struct H1Ctl {
  int64_t round;        // rounds completed
  int64_t T;            // triangles, n(n-1)(n-2)/6
  int64_t nsurv;        // entries of the survivor array (set by the first round)
  int64_t live;         // survivors whose column is not final yet
  int64_t ncommit;      // survivors picked to commit this round
  int64_t nwalk;        // survivors that walk again this round
  int64_t pivots;       // columns committed by the rounds (emergent pairs excluded)
  int64_t additions;    // column additions of final walks
  int64_t walks;        // column walks, counting repeats
  int64_t stored;       // rows taken at the end (all pivots)
  int64_t nbars;        // pairs of positive length
  uint64_t firstdup;    // first live survivor that is not the smallest on its row
  int32_t err;          // bit 0: a repeated walk ended elsewhere; bit 1: corrupt table
  int32_t pad;
};
struct H1Args {
  const uint64_t* keys;  // E sorted H0 keys
  int ib;
  int64_t n, E, T, LWE;
  int32_t* inv;          // E: colex edge id -> sorted position
  uint32_t* grade;       // E: grade of each sorted position
  uint32_t* cnt;         // E: triangles whose latest edge is q
  uint32_t* start;       // E + 1: exclusive scan of cnt
  uint32_t* scan_tmp;    // scan_totals_len(E + 1) words
  uint64_t* tri;         // T: (latest edge q << 32) | third vertex, in triangle order
  int32_t* owner;        // E: triangle stored in row q, -1 = free
  uint64_t* lowc;        // E: smallest live survivor per row
  uint64_t* table;       // E x LWE words
  uint64_t* surv;        // T: survivor array, (t << 32) | low, low = ~0 once final
  uint64_t* clist;       // E: survivors committing this round
  uint32_t* wlist;       // T: survivors walking again this round (indices into surv)
  uint64_t* store;       // cap x LWE words: the columns of survivors 0 .. cap-1
  uint32_t* sadds;       // cap: additions made so far by those survivors
  int64_t cap;           // survivors whose column is kept (the rest walk again)
  int64_t nsurv_host;    // entries of surv (for the grid sizes)
  int cus;
  H1Ctl* ctl;
};
int h1_words_per_lane(int64_t LWE);
hipError_t launch_h1_setup(const H1Args& a, hipStream_t s);
// The first round walks every triangle; later rounds commit and walk again.
hipError_t launch_h1_round(const H1Args& a, bool first, hipStream_t s);
hipError_t launch_h1_bars(const H1Args& a, uint64_t* packed, hipStream_t s);
hipError_t launch_h1_bars_out(const uint64_t* sorted, int64_t m, uint32_t* bars, hipStream_t s);
hipError_t launch_h1_owner_out(const int32_t* owner, int64_t E, int64_t* out, hipStream_t s);

}  // namespace ph0
