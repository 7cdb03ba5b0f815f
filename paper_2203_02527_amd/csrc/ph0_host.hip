// ph0_host.hip -- the C ABI declared in include/ph0.h: argument checks, key
// layout and sort planning, workspace carving, and the stage sequence
//   coordinate ranges -> keys -> LSD radix passes -> round-based reduction
//   -> grades -> per-vertex deaths -> canonical barcode.
// Every step of the computation runs in the HIP kernels of this library;
// the host only plans, launches and steers the reduction rounds.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <cstring>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ph0.h"
#include "ph0_internal.h"

using namespace ph0;

namespace {

thread_local char g_err[512] = "";
std::atomic<int64_t> g_window{0};

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PH0_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

constexpr int64_t kMaxN = 65536;
// Built-in chunk multipliers of the batched kernel per cloud size bucket
// (n <= 64, <= 128, <= 256, <= 512), used when no tuning is passed: the
// values the autotuner (paper_2203_02527_amd/autotune.py) chose on MI355X
// for the batch workload's clouds.
constexpr int32_t kChunkMult[4] = {6, 6, 8, 48};
// Built-in workgroups per compute unit of the batched kernel (two fit the
// 160 KB of LDS of a CU).
constexpr int32_t kBlocksPerCu = 2;
constexpr int32_t kDigitBits = 8;      // batched radix digit width
constexpr int32_t kWavesPerCloud = 8;  // batched workgroup: 512 threads
// Edge count from which the single-cloud path recomputes keys per distance
// range instead of storing all of them (below it, the extra passes and host
// round trips cost more than the stored keys).
constexpr int64_t kRecomputeMinE = int64_t(1) << 22;
constexpr size_t kAlign = 256;
// Largest single cloud that ph0_barcodes_device computes in one workgroup
// (measured on MI355X: faster than the grid-wide passes up to n of about
// 300 at d = 3 and 16; 256 keeps a margin).
constexpr int64_t kFusedSingleMaxN = 256;
// Size of the fixed device array that ph0_barcodes_batched_device_noalloc
// uses as its workspace (per device, held until the process ends).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int index_bits(int64_t n) { return n <= 1 ? 0 : 64 - __builtin_clzll((uint64_t)(n - 1)); }

// Window positions are kept as 32-bit offsets from the window start, so the
// ring (at most kWindowGrowth base windows) stays below 2^31 columns.
constexpr int64_t kMaxWindow = int64_t(1) << 26;

// Base number of columns in flight per reduction round; a power of two.
// Measured on MI355X (mixture clouds, seeds 0, 3, 5): 65536 is the fastest
// base at N = 4096 (against 8192 .. 32768) and at N = 16384 (against 16384
// .. 262144; 4-6% ahead of 262144, which takes 8-11 fewer rounds but walks
// more columns per round).
int64_t window_for(int64_t n, int64_t E) {
  int64_t w = g_window.load();
  if (w <= 0) w = std::max<int64_t>(65536, 4 * n);
  w = std::min<int64_t>(w, std::max<int64_t>(E, 1));
  w = std::min<int64_t>(w, kMaxWindow);
  int64_t p = 1;
  while (p < w) p <<= 1;
  return p;
}

// The window grows up to this many times its base width while rounds leave
// almost nothing active: the sweep past the forest-building phase (columns
// that almost all reduce to zero) then takes fewer rounds (N=16384: 25 -> 20
// rounds for about 10% more column walks past the last pivot).
constexpr int64_t kWindowGrowth = 16;
static_assert(kWindowGrowth * kMaxWindow < (int64_t(1) << 31), "ring offsets fit 31 bits");

// Capacity of the per-column ring (indexed by column & (capacity - 1)): the
// largest window, a power of two.
int64_t ring_for(int64_t n, int64_t E) {
  const int64_t w = window_for(n, E);
  int64_t p = 1;
  while (p < std::max<int64_t>(E, 1)) p <<= 1;
  return std::min<int64_t>(kWindowGrowth * w, std::max<int64_t>(p, w));
}

struct Layout {
  int64_t n, E, Wcap, width, tiles;
  size_t keysA, keysB, counts, hist, err, part, surv, surv_ra, surv_x, scount, fdslot, wstat, cslot, osum, killer,
      lowc, touch, act0, act1, actra0, actra1, actx0, actx1, werr, part16, rst, ctl, dbv, minmax, hshift, kcnt,
      kcnt_tot, norms, total;
};

Layout make_layout(int64_t n, int32_t d) {
  Layout L;
  L.n = n;
  L.E = n * (n - 1) / 2;
  L.width = window_for(n, L.E);
  L.Wcap = ring_for(n, L.E);
  const int64_t keys = std::max<int64_t>(L.E, 2 * n + 64);  // room for the bar sort too
  L.tiles = radix_tiles(keys);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.keysA = take(8 * (size_t)keys);
  L.keysB = take(8 * (size_t)keys);
  L.counts = take(4 * (size_t)radix_count_entries(keys));
  // The error word follows the histogram, so one fill clears both.
  L.hist = take(4 * (size_t)(kHistBins + 1));
  L.err = L.hist + 4 * (size_t)kHistBins;
  L.part = take(4 * (size_t)n);
  const size_t wb = (size_t)walk_blocks(L.Wcap), segs = wb * (size_t)walk_segment(L.Wcap);
  L.surv = take(8 * segs);
  L.surv_ra = take(8 * segs);
  L.surv_x = take(8 * segs);
  L.scount = take(4 * wb);
  L.fdslot = take(8 * wb);
  L.wstat = take(8 * 3 * wb);
  L.cslot = take(4 * 4 * wb);
  L.werr = take(4);
  L.killer = take(8 * (size_t)n);
  L.lowc = take(8 * (size_t)n);
  L.touch = take(8 * (size_t)n);
  L.act0 = take(8 * segs);
  L.act1 = take(8 * segs);
  L.actra0 = take(8 * segs);
  L.actra1 = take(8 * segs);
  L.actx0 = take(8 * segs);
  L.actx1 = take(8 * segs);
  L.part16 = take(2 * (size_t)std::max<int64_t>(part16_len(n), 8));
  L.rst = take(4 * (size_t)L.Wcap);
  L.ctl = take(2 * sizeof(RedCtl));  // the two round states
  L.dbv = take(4 * (size_t)n);
  L.minmax = take(8 * (size_t)d);
  L.hshift = take(4);
  // Sized for the finer (per-tile) layout; + 1: the scan leaves the total there.
  const int64_t kc = key_count_len(n, false) + 1;
  L.kcnt = take(4 * (size_t)kc);
  L.kcnt_tot = take(4 * (size_t)scan_totals_len(kc));
  L.norms = take(4 * (size_t)n);
  L.total = o;
  (void)d;
  return L;
}

int check_args(const void* p, ph0_dtype dt, int64_t n, int32_t d) {
  if (!p) return fail(PH0_EINVAL, "points pointer is NULL");
  if (dt != PH0_I8 && dt != PH0_I16) return fail(PH0_EINVAL, "dtype must be PH0_I8 or PH0_I16");
  if (n < 1) return fail(PH0_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
  if (n > kMaxN) return fail(PH0_EINVAL, "n must be <= %lld (got %lld)", (long long)kMaxN, (long long)n);
  if (d < 1) return fail(PH0_EINVAL, "d must be >= 1 (got %d)", d);
  return PH0_OK;
}

SortPlan plan_sort(int ib, int dbits) {
  SortPlan sp = {};
  sp.passes = (dbits + 7) / 8;
  int shift = 2 * ib;
  for (int p = 0; p < sp.passes; ++p) {
    const int w = dbits / sp.passes + (p < dbits % sp.passes ? 1 : 0);
    sp.shift[p] = shift;
    sp.bits[p] = w;
    shift += w;
  }
  return sp;
}

// Timing events are taken from a per-thread pool that grows on demand, so a
// call with statistics creates no events once the pool covers it.  The
// events are never destroyed: a thread-exit destructor could run after the
// HIP runtime has shut down at process exit.
struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
};

EventPool& event_pool() {
  thread_local EventPool pool;
  return pool;
}

// Returns the pool's events to it when a call ends (calls on one thread do
// not overlap, and each call reads its times before it returns).
struct PoolScope {
  size_t mark;
  PoolScope() : mark(event_pool().used) {}
  ~PoolScope() { event_pool().used = mark; }
};

struct Timer {
  bool on;
  hipStream_t s;
  hipEvent_t ev[8] = {};
  int k = 0;
  explicit Timer(bool enabled, hipStream_t st) : on(enabled), s(st) {
    if (on)
      for (auto& e : ev) on = on && (e = event_pool().get()) != nullptr;
  }
  void mark() {
    if (on && k < 8) (void)hipEventRecord(ev[k++], s);
  }
  float ms(int a, int b) {
    float v = 0;
    if (on && b < k) (void)hipEventElapsedTime(&v, ev[a], ev[b]);
    return v;
  }
};

// Event pairs around individual kernel launches (stats only).
struct KernelClock {
  bool on;
  std::vector<hipEvent_t> ev;
  explicit KernelClock(bool enabled) : on(enabled) {}
  hipEvent_t* pair() {
    if (!on) return nullptr;
    const hipEvent_t a = event_pool().get(), b = event_pool().get();
    if (!a || !b) return nullptr;
    ev.push_back(a);
    ev.push_back(b);
    return &ev[ev.size() - 2];
  }
  float total_ms() const {
    float t = 0;
    for (size_t k = 0; k + 1 < ev.size(); k += 2) {
      float v = 0;
      if (hipEventElapsedTime(&v, ev[k], ev[k + 1]) == hipSuccess) t += v;
    }
    return t;
  }
  int launches() const { return (int)(ev.size() / 2); }
};

// Two pinned control-block copies and their events per host thread: the
// reduction loop inspects one burst's copy while the next burst runs.
struct CtlReadback {
  RedCtl* hc = nullptr;      // [2]
  uint32_t* words = nullptr;  // [4]: radix error flag, distinct grades, pivot columns,
                              // keys in a distance range
  void* buf = nullptr;        // coordinate ranges and histogram, grown on demand
  size_t buf_bytes = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ok = false;
};

// The calling thread's pinned read-back area of at least `bytes` bytes
// (nothing is in flight into it between calls: every call ends synchronized).
void* pinned_buf(CtlReadback* rb, size_t bytes) {
  if (rb->buf_bytes < bytes) {
    if (rb->buf) (void)hipHostFree(rb->buf);
    rb->buf = nullptr;
    rb->buf_bytes = 0;
    if (hipHostMalloc(&rb->buf, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    rb->buf_bytes = bytes;
  }
  return rb->buf;
}

CtlReadback& thread_readback() {
  thread_local CtlReadback rb;
  return rb;
}

CtlReadback* pinned_ctl() {
  CtlReadback& rb = thread_readback();
  if (!rb.ok) {
    // Pinned, so that copies into it are asynchronous (a copy into pageable
    // memory waits for the stream).
    if (hipHostMalloc((void**)&rb.hc, 2 * sizeof(RedCtl) + 16, hipHostMallocDefault) !=
        hipSuccess)
      return nullptr;
    rb.words = reinterpret_cast<uint32_t*>(rb.hc + 2);
    for (int k = 0; k < 2; ++k)
      if (hipEventCreateWithFlags(&rb.ev[k], hipEventDisableTiming) != hipSuccess) return nullptr;
    rb.ok = true;
  }
  return &rb;
}

// Waits for the stream when a call leaves before its own final wait (an
// error return after work was queued): kernels still queued could otherwise
// write into the caller's workspace and outputs after the call returned.
// Success paths end synchronized and disarm it.
struct StreamDrain {
  hipStream_t s;
  bool armed = true;
  explicit StreamDrain(hipStream_t st) : s(st) {}
  ~StreamDrain() {
    if (armed) (void)hipStreamSynchronize(s);
  }
};

// Frees the calling thread's pinned read-back area and timing events.  A
// server worker calls it before it exits (the HIP runtime is alive then);
// threads that live until process exit keep theirs (see EventPool).
void release_thread_resources() {
  CtlReadback& rb = thread_readback();
  if (rb.hc) (void)hipHostFree(rb.hc);
  if (rb.buf) (void)hipHostFree(rb.buf);
  for (auto& e : rb.ev)
    if (e) (void)hipEventDestroy(e);
  rb = CtlReadback();
  EventPool& pool = event_pool();
  for (hipEvent_t e : pool.ev) (void)hipEventDestroy(e);
  pool.ev.clear();
  pool.used = 0;
}

enum Stop { kStopKeys = 1, kStopSorted = 2, kStopAll = 3 };

struct Outputs {
  ph0_bar* bars = nullptr;
  uint32_t* dbv = nullptr;
  int64_t* killer_pos = nullptr;
  uint64_t* killer_edge = nullptr;
  int64_t* killer_sqdist = nullptr;
  int32_t* partner = nullptr;
  uint64_t* keys = nullptr;  // for the stage entry points
};

int run(const void* d_points, ph0_dtype dt, int64_t n, int32_t d, const Outputs& out,
        void* d_ws, size_t ws_bytes, hipStream_t s, ph0_stats* st, Stop stop) {
  int rc = check_args(d_points, dt, n, d);
  if (rc) return rc;
  if (!d_ws) return fail(PH0_EINVAL, "workspace pointer is NULL");
  const Layout L = make_layout(n, d);
  if (ws_bytes < L.total)
    return fail(PH0_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  char* ws = static_cast<char*>(d_ws);
  auto at = [&](size_t off) { return static_cast<void*>(ws + off); };
  const int eb = dt == PH0_I8 ? 1 : 2;
  const int ib = index_bits(n);
  ph0_stats S = {};
  S.n = n;
  S.E = L.E;
  S.index_bits = ib;
  S.window = L.width;
  StreamDrain drain(s);

  if (n == 1) {
    if (stop != kStopAll) return PH0_OK;
    if (out.bars) {
      const ph0_bar one = {0u, PH0_INF};
      HIPCHK(hipMemcpyAsync(out.bars, &one, sizeof(one), hipMemcpyHostToDevice, s));
    }
    if (out.dbv) HIPCHK(launch_fill_u32(out.dbv, kInf, 1, s));
    if (out.killer_pos) HIPCHK(launch_fill_u64((uint64_t*)out.killer_pos, ~0ull, 1, s));
    if (out.killer_edge) HIPCHK(launch_fill_u64(out.killer_edge, ~0ull, 1, s));
    if (out.killer_sqdist) HIPCHK(launch_fill_u64((uint64_t*)out.killer_sqdist, ~0ull, 1, s));
    if (out.partner) HIPCHK(launch_fill_u32((uint32_t*)out.partner, ~0u, 1, s));
    HIPCHK(hipStreamSynchronize(s));
    drain.armed = false;
    if (st) *st = S;
    return PH0_OK;
  }

  // Small clouds, when only the barcode is asked for (no statistics, no
  // per-vertex detail): the whole computation in one workgroup -- the fused
  // kernel of the batched path, on this one cloud -- instead of the
  // grid-wide passes, whose launches and host round trips dominate there.
  if (stop == kStopAll && !st && out.bars && !out.dbv && !out.killer_pos && !out.killer_edge &&
      !out.killer_sqdist && !out.partner && n <= kFusedSingleMaxN && n * d <= kBatchMaxPts &&
      d <= 64) {
    CtlReadback* rb = pinned_ctl();
    if (!rb) return fail(PH0_ENOMEM, "pinned host allocation failed");
    const size_t scratch = align_up(16 * (size_t)L.E), grades = align_up(4 * (size_t)L.E);
    if (scratch + grades + kAlign > L.total)
      return fail(PH0_EDEVICE, "fused scratch does not fit the workspace");
    BatchArgs A;
    A.pts = d_points;
    A.elem_bytes = eb;
    A.d = d;
    A.offsets = nullptr;
    A.order = nullptr;
    A.nclouds = 1;
    A.bars = reinterpret_cast<uint32_t*>(out.bars);
    A.scratch = reinterpret_cast<uint64_t*>(ws);
    A.grades = reinterpret_cast<uint32_t*>(ws + scratch);
    A.emax = L.E;
    A.queue = nullptr;
    A.errs = reinterpret_cast<int32_t*>(ws + scratch + grades);
    for (int b = 0; b < 4; ++b) A.chunk_mult[b] = kChunkMult[b];
    A.single_n = n;
    HIPCHK(launch_batched(A, 1, s));
    HIPCHK(hipMemcpyAsync(&rb->words[0], A.errs, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    drain.armed = false;
    const int32_t code = (int32_t)rb->words[0];
    if (code)
      return fail(code == 3 ? PH0_ERANGE : PH0_EDEVICE,
                  code == 3 ? "packed key needs more than 64 bits (reduce the coordinate range)"
                            : "the fused kernel reported an inconsistency (code %d)",
                  code);
    return PH0_OK;
  }

  PoolScope pool_scope;
  Timer tm(st != nullptr, s);
  tm.mark();  // 0
  // The per-dimension coordinate ranges (lo[0..d) then hi[0..d)) bound the
  // squared distance.  The histogram's shift follows from them on the
  // device, and the host reads the ranges back with the histogram, so the
  // bound costs no wait of its own; it is checked before any key is used.
  CtlReadback* rb = pinned_ctl();
  if (!rb) return fail(PH0_ENOMEM, "pinned host allocation failed");
  const size_t ranges_bytes = align_up(8 * (size_t)d);
  char* back = static_cast<char*>(pinned_buf(rb, ranges_bytes + 4 * (size_t)kHistBins));
  if (!back) return fail(PH0_ENOMEM, "pinned host allocation failed");
  const int32_t* ranges = reinterpret_cast<const int32_t*>(back);
  const uint32_t* h = reinterpret_cast<const uint32_t*>(back + ranges_bytes);
  int32_t* mm = static_cast<int32_t*>(at(L.minmax));
  int32_t* dshift = static_cast<int32_t*>(at(L.hshift));
  int32_t* norms = static_cast<int32_t*>(at(L.norms));
  uint32_t* hist = static_cast<uint32_t*>(at(L.hist));
  int32_t* serr = static_cast<int32_t*>(at(L.err));
  bool norms_done = false;  // the range pass also formed the squared norms
  // The launch that initialises the ranges also clears the histogram and
  // the error word that follows it.
  HIPCHK(launch_coord_range(d_points, eb, n, d, mm, s, norms, &norms_done, hist,
                            kHistBins + 1));
  HIPCHK(launch_dist_shift(mm, d, dshift, s));
  const bool mfma = (eb == 1) && d >= 8 && d <= 32768;
  S.keys_path = mfma ? 1 : 0;

  uint64_t* keysA = static_cast<uint64_t*>(at(L.keysA));
  uint64_t* keysB = static_cast<uint64_t*>(at(L.keysB));
  uint32_t* counts = static_cast<uint32_t*>(at(L.counts));

  // Large problems never store all keys: a sampled histogram picks the
  // distance ranges, and each range's keys are recomputed and written, in
  // colex order, only when the reduction needs them.
  const bool recompute = stop == kStopAll && L.E >= kRecomputeMinE;
  const int64_t nbk = (n + 63) / 64;
  const int64_t sample = std::max<int64_t>(1, nbk * (nbk + 1) / 2 / 2048);
  bool keys_full = false;  // keysA holds every key at its colex position
  tm.mark();  // 1
  if (recompute) {
    KeyPass kp;
    kp.mode = kKeysHist;
    kp.norms = norms;
    kp.norms_ready = norms_done;
    kp.hist = hist;
    kp.hist_shift_dev = dshift;
    kp.sample = sample;
    HIPCHK(launch_keys_pass(d_points, eb, n, d, ib, mfma, kp, s));
  } else {
    HIPCHK(launch_keys(d_points, eb, n, d, ib, keysA, mfma, 0, hist, norms, s, dshift));
    keys_full = true;
  }
  tm.mark();  // 2
  // One wait: the ranges, and the histogram when the reduction follows.
  {
    Gather g;
    g.add(mm, back, 8 * (size_t)d);
    if (stop == kStopAll) g.add(hist, back + ranges_bytes, 4 * (size_t)kHistBins);
    HIPCHK(launch_gather(g, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  unsigned __int128 bound = 0;
  for (int32_t k = 0; k < d; ++k) {
    const int64_t w = (int64_t)ranges[d + k] - ranges[k];
    bound += (unsigned __int128)(w * w);
  }
  int dbits = 0;
  while (dbits < 100 && (bound >> dbits) != 0) ++dbits;
  S.delta_bits = dbits;
  if (2 * ib + dbits > 64)
    return fail(PH0_ERANGE,
                "packed key needs %d distance bits + 2 x %d index bits > 64 (reduce the "
                "coordinate range)",
                dbits, ib);
  const SortPlan sp = plan_sort(ib, dbits);
  S.sort_passes = sp.passes;
  const int hist_shift = dbits > 11 ? dbits - 11 : 0;  // as the device computed it
  if (stop == kStopKeys) {
    HIPCHK(hipMemcpyAsync(out.keys, keysA, 8 * (size_t)L.E, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    drain.armed = false;
    return PH0_OK;
  }

  KernelClock radix_clock(st != nullptr), walk_clock(st != nullptr);
  // One LSD pass, timed when stats are requested.
  auto pass = [&](const uint64_t* in, uint64_t* outk, int64_t count, int p, KeyFilter f,
                  int64_t expect) -> hipError_t {
    hipEvent_t* ev = radix_clock.pair();
    if (ev) (void)hipEventRecord(ev[0], s);
    const hipError_t e =
        launch_radix_pass(in, outk, count, sp.shift[p], sp.bits[p], counts, serr, s, f, expect);
    if (ev) (void)hipEventRecord(ev[1], s);
    return e;
  };
  // Every key, in sorted order, ping-ponging between the two key buffers.
  uint64_t* skeys = keysA;  // sorted order (a prefix of it while chunked)
  uint64_t* spare = keysB;  // the other buffer
  auto full_sort = [&]() -> hipError_t {
    if (!keys_full) {
      const hipError_t e = launch_keys(d_points, eb, n, d, ib, keysA, mfma, hist_shift, hist, norms, s);
      if (e != hipSuccess) return e;
      keys_full = true;
    }
    uint64_t* src = keysA;
    uint64_t* dst = keysB;
    for (int p = 0; p < sp.passes; ++p) {
      const hipError_t e = pass(src, dst, L.E, p, KeyFilter(), -1);
      if (e != hipSuccess) return e;
      std::swap(src, dst);
    }
    skeys = src;
    spare = dst;
    return hipSuccess;
  };
  if (stop == kStopSorted) {
    HIPCHK(full_sort());
    tm.mark();  // 3
    int32_t herr = 0;
    HIPCHK(hipMemcpyAsync(out.keys, skeys, 8 * (size_t)L.E, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(&herr, serr, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    drain.armed = false;
    if (herr) return fail(PH0_EDEVICE, "radix sort digit counts were inconsistent");
    return PH0_OK;
  }

  // The reduction only ever needs the sorted order up to its last pivot, so
  // the sort proceeds in distance ranges (chunks of histogram bins, growing
  // geometrically): a chunk's keys are picked out of all keys by the first
  // LSD pass and sorted into the next positions of the sorted array, which
  // therefore always holds an exact prefix of the full order.
  int64_t E_lim = 0;
  int bin_next = 0, chunks = 0;
  bool whole = false;
  uint32_t* kcnt = static_cast<uint32_t*>(at(L.kcnt));
  const int64_t kcnt_len = key_count_len(n, mfma);
  // Exact number of keys in bins [blo, bhi), with their colex bases left in
  // kcnt for the emit pass.
  auto count_range = [&](int blo, int bhi, int64_t* cnt) -> hipError_t {
    KeyPass kp;
    kp.mode = kKeysCount;
    kp.norms = norms;
    kp.norms_ready = true;  // the histogram pass computed them
    kp.dlo = (uint64_t)blo << hist_shift;
    kp.dhi = bhi >= kHistBins ? ~0ull : (uint64_t)bhi << hist_shift;
    kp.cnt = kcnt;
    hipError_t e = launch_keys_pass(d_points, eb, n, d, ib, mfma, kp, s);
    if (e == hipSuccess) e = launch_fill_u32(kcnt + kcnt_len, 0u, 1, s);
    if (e == hipSuccess)
      e = launch_scan_u32(kcnt, kcnt_len + 1, static_cast<uint32_t*>(at(L.kcnt_tot)), s);
    if (e == hipSuccess) {  // the total, into pinned memory
      Gather g;
      g.add(kcnt + kcnt_len, &rb->words[3], 4);
      e = launch_gather(g, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *cnt = e == hipSuccess ? (int64_t)rb->words[3] : 0;
    return e;
  };
  auto next_chunk = [&]() -> hipError_t {
    // The second range is as large as the first (a last pivot just past the
    // first range is the common case), later ones double.
    const int64_t target = std::max<int64_t>(L.E / 16, 8 * n)
                           << std::min(std::max(chunks - 1, 0), 20);
    int b = bin_next;
    int64_t cnt = 0;
    while (b < kHistBins && (cnt == 0 || cnt < target))
      cnt += (int64_t)h[b++] * (keys_full ? 1 : sample);
    ++chunks;
    if (!keys_full && sp.passes > 0) {
      // Exact count; a sampled histogram can show keys where there are none.
      while (true) {
        const hipError_t e = count_range(bin_next, b, &cnt);
        if (e != hipSuccess) return e;
        if (cnt > 0 || b >= kHistBins) break;
        while (b < kHistBins && h[b] == 0) ++b;
        if (b < kHistBins) ++b;
      }
    }
    if (sp.passes == 0 || E_lim + 2 * cnt > L.E) {
      // The rest in one full sort; its prefix equals the chunks sorted so far.
      whole = true;
      E_lim = L.E;
      return full_sort();
    }
    KeyFilter f;
    int64_t first_in = L.E;
    if (keys_full) {  // the first pass picks the range out of all keys
      f.fshift = 2 * ib + hist_shift;
      f.flo = (uint64_t)bin_next;
      f.fhi = (uint64_t)b;
    } else {  // the range's keys, recomputed into keysA in colex order
      KeyPass kp;
      kp.mode = kKeysEmit;
      kp.norms = norms;
      kp.norms_ready = true;
      kp.dlo = (uint64_t)bin_next << hist_shift;
      kp.dhi = b >= kHistBins ? ~0ull : (uint64_t)b << hist_shift;
      kp.cnt = kcnt;
      kp.keys = keysA;
      const hipError_t e = launch_keys_pass(d_points, eb, n, d, ib, mfma, kp, s);
      if (e != hipSuccess) return e;
      first_in = cnt;
    }
    uint64_t* D = keysB + E_lim;        // the chunk's final place
    uint64_t* T = keysB + E_lim + cnt;  // scratch for the ping-pong
    const uint64_t* in = keysA;
    for (int p = 0; p < sp.passes; ++p) {
      uint64_t* o = ((sp.passes - 1 - p) % 2 == 0) ? D : T;
      const hipError_t e = pass(in, o, p == 0 ? first_in : cnt, p, p == 0 ? f : KeyFilter(), cnt);
      if (e != hipSuccess) return e;
      in = o;
    }
    skeys = keysB;
    spare = keysA;
    E_lim += cnt;
    bin_next = b;
    return hipSuccess;
  };
  HIPCHK(next_chunk());
  tm.mark();  // 3

  // Reduction rounds.
  RedArgs ra;
  ra.skeys = skeys;
  ra.ib = ib;
  ra.n = n;
  ra.E = L.E;
  ra.Wcap = L.Wcap;
  ra.width = L.width;
  ra.seg = walk_segment(L.Wcap);
  ra.nblocks = walk_blocks(L.Wcap);
  ra.count = st != nullptr;  // the addition counts are statistics: formed only when asked
  ra.werr = static_cast<int32_t*>(at(L.werr));
  ra.act[0] = static_cast<int64_t*>(at(L.act0));
  ra.act[1] = static_cast<int64_t*>(at(L.act1));
  ra.act_ra[0] = static_cast<uint64_t*>(at(L.actra0));
  ra.act_ra[1] = static_cast<uint64_t*>(at(L.actra1));
  ra.act_x[0] = static_cast<uint64_t*>(at(L.actx0));
  ra.act_x[1] = static_cast<uint64_t*>(at(L.actx1));
  ra.part = static_cast<int32_t*>(at(L.part));
  ra.surv = static_cast<int64_t*>(at(L.surv));
  ra.surv_ra = static_cast<uint64_t*>(at(L.surv_ra));
  ra.surv_x = static_cast<uint64_t*>(at(L.surv_x));
  ra.scount = static_cast<uint32_t*>(at(L.scount));
  ra.fdslot = static_cast<uint64_t*>(at(L.fdslot));
  ra.wstat = static_cast<uint64_t*>(at(L.wstat));
  ra.cslot = static_cast<uint32_t*>(at(L.cslot));
  ra.killer = static_cast<int64_t*>(at(L.killer));
  ra.lowc = static_cast<uint64_t*>(at(L.lowc));
  ra.touch = static_cast<uint64_t*>(at(L.touch));
  ra.part16 = part16_len(n) ? static_cast<uint16_t*>(at(L.part16)) : nullptr;
  ra.ring.st = static_cast<int32_t*>(at(L.rst));
  ra.ctl = static_cast<RedCtl*>(at(L.ctl));
  RedCtl* hc = rb->hc;
  HIPCHK(launch_reduce_init(ra, E_lim, s));
  // Rounds go out in bursts; each burst ends with the one-wave advance,
  // which also leaves the state in pinned host memory, and an event.  The
  // host inspects a burst's state while the next burst already runs, so the
  // GPU never waits for the host; rounds
  // issued after the end find `done` (or an empty range) and return at once.
  // Every round finalizes at least the first unfinished column (it either
  // reduces to zero or commits), so the window start must advance.
  // The first burst is short and inspected before anything else is queued,
  // so that small problems (a round or two) do not queue idle rounds.
  int burst = 2;  // grows to 8
  int64_t R = 0;  // rounds launched
  auto issue = [&](int slot) -> hipError_t {
    for (int t = 0; t < burst; ++t) {
      // A burst's first round starts from a state advanced already (the
      // initial one, or the previous burst's); the others advance it in
      // their walk.
      const hipError_t e = launch_reduce_round(ra, s, walk_clock.pair(), R, t == 0);
      if (e != hipSuccess) return e;
      ++R;
    }
    // The state after the burst, also into the slot's pinned copy.
    const hipError_t e = launch_reduce_advance(ra, R, &hc[slot], s);
    return e == hipSuccess ? hipEventRecord(rb->ev[slot], s) : e;
  };
  // Up to two bursts in flight (slots alternate; a slot is reused only after
  // it was inspected); the first burst is inspected alone.
  int64_t prevF = -1;
  int next_slot = 0, q_head = 0, q_len = 0;
  int queue[2];
  int qburst[2] = {0, 0};  // rounds in each queued burst, by slot
  int64_t prev_piv = 0, prev_round = 0;
  auto issue_next = [&]() -> hipError_t {
    const hipError_t e = issue(next_slot);
    queue[(q_head + q_len) & 1] = next_slot;
    qburst[next_slot] = burst;
    ++q_len;
    next_slot ^= 1;
    return e;
  };
  bool pipelined = false;
  // Once every pivot exists exactly one more round remains: its walks all end
  // in zero (the only free row, vertex 0, can never be a column's low), so
  // nothing is queued behind the round that follows that state.
  bool last_round_queued = false;
  HIPCHK(issue_next());
  while (true) {
    if (pipelined && q_len < 2 && !last_round_queued) HIPCHK(issue_next());
    const int k = queue[q_head];
    q_head ^= 1;
    --q_len;
    HIPCHK(hipEventSynchronize(rb->ev[k]));
    const RedCtl& h = hc[k];
    const int32_t herr = h.err;
    if (h.done) break;
    if (h.need_more && !herr) {
      if (whole) return fail(PH0_EDEVICE, "reduction asked for columns past the last one");
      HIPCHK(hipStreamSynchronize(s));  // any queued burst found nothing to do
      q_len = 0;
      HIPCHK(next_chunk());
      ra.skeys = skeys;
      HIPCHK(launch_reduce_extend(ra, E_lim, R, s));
      prevF = -1;
      HIPCHK(issue_next());
      continue;
    }
    if (h.F <= prevF || herr) {
      HIPCHK(hipStreamSynchronize(s));
      return fail(PH0_EDEVICE, "reduction stalled at column %lld (err %d)", (long long)h.F,
                  herr);
    }
    prevF = h.F;
    // Bursts grow 2, 4, 8 (then stay): rounds queued past the end cost a few
    // launches each, so small problems queue few.  A burst is also cut to
    // the rounds still needed at the last burst's pivot rate, less those
    // already queued, plus one to finish the columns before the last pivot.
    // Once every pivot exists only those columns remain (a round or two), so
    // the bursts shrink to single rounds.
    pipelined = true;
    if (h.pivots >= n - 1) {
      burst = 1;
      if (q_len > 0) {
        last_round_queued = true;  // the queued burst's first round finishes
        continue;
      }
    } else {
      if (burst < 8) burst *= 2;
      const int64_t rate = (h.pivots - prev_piv) / std::max<int64_t>(1, h.round - prev_round);
      if (rate > 0) {
        const int64_t queued = q_len ? qburst[queue[q_head]] : 0;
        const int64_t need = (n - 1 - h.pivots + rate - 1) / rate + 1 - queued;
        burst = (int)std::max<int64_t>(1, std::min<int64_t>(burst, need));
      }
    }
    prev_piv = h.pivots;
    prev_round = h.round;
    if (q_len == 0) HIPCHK(issue_next());
  }
  S.sort_chunks = chunks;
  S.sorted_keys = E_lim;
  HIPCHK(launch_reduce_finish(ra, R, s));
  uint32_t* hw = rb->words;
  {
    Gather g;
    g.add(reduce_state(ra, R), hc, sizeof(RedCtl));
    g.add(serr, &hw[0], 4);
    HIPCHK(launch_gather(g, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  tm.mark();  // 4
  if (hw[0]) return fail(PH0_EDEVICE, "radix sort digit counts were inconsistent");
  const RedCtl* fin = hc;
  if (hc->err & 1) return fail(PH0_EDEVICE, "a reduced column did not have exactly two rows");
  if (fin->err & 2 || fin->pivots != n - 1)
    return fail(PH0_EDEVICE, "reduction ended with %lld pivots, expected %lld",
                (long long)fin->pivots, (long long)(n - 1));
  S.E_eff = fin->E_eff;
  S.additions_all = fin->additions_all;
  S.additions = fin->additions_all - fin->additions_overshoot;
  S.find_steps = fin->find_steps;
  S.words_read = fin->words_read;
  S.rounds = fin->round;

  // Grades over [0, E_eff), per-vertex deaths and the barcode, in one
  // ordered pass over the pivot positions (scratch: the spare key buffer).
  uint32_t* dbv = out.dbv ? out.dbv : static_cast<uint32_t*>(at(L.dbv));
  if (grades_work_bytes(fin->E_eff) > 8 * (size_t)std::max<int64_t>(L.E, 2 * n + 64))
    return fail(PH0_EDEVICE, "grade scratch does not fit the key buffer");
  const uint32_t *d_distinct = nullptr, *d_npiv = nullptr;
  HIPCHK(launch_grades_and_bars(skeys, fin->E_eff, 2 * ib, ra.killer, n, spare, dbv,
                                reinterpret_cast<uint32_t*>(out.bars), s, &d_distinct, &d_npiv));
  tm.mark();  // 5
  if (out.killer_pos || out.killer_edge || out.killer_sqdist || out.partner)
    HIPCHK(launch_pairs_detail(ra.killer, skeys, ib, ra.part, n, out.killer_pos,
                               out.killer_edge, out.killer_sqdist, out.partner, s));
  tm.mark();  // 6
  {
    Gather g;
    g.add(serr, &hw[0], 4);
    g.add(d_distinct, &hw[1], 4);
    g.add(d_npiv, &hw[2], 4);
    HIPCHK(launch_gather(g, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  drain.armed = false;
  const uint32_t distinct = hw[1], npiv = hw[2];
  if (hw[0]) return fail(PH0_EDEVICE, "radix sort digit counts were inconsistent");
  if (npiv != (uint32_t)(n - 1))
    return fail(PH0_EDEVICE, "found %u pivot columns, expected %lld", npiv, (long long)(n - 1));
  S.distinct_eff = 1 + distinct;
  if (st) {
    S.ms_keys = tm.ms(1, 2);
    S.ms_sort = tm.ms(2, 3);
    S.ms_reduce = tm.ms(3, 4);
    S.ms_rank = tm.ms(4, 5);
    S.ms_emit = tm.ms(5, 6);
    S.ms_total = tm.ms(0, 6);
    S.ms_walk_kernel = walk_clock.total_ms();
    S.walk_launches = walk_clock.launches();
    S.ms_radix_kernel = radix_clock.total_ms();
    S.radix_launches = radix_clock.launches();
    *st = S;
  }
  return PH0_OK;
}

// ---- batched path ----

struct BatchPlan {
  int64_t nclouds = 0, emax = 0, big_n = 0, blocks = 0;
  std::vector<int32_t> order;  // fused clouds, largest first
  std::vector<int32_t> big;    // clouds for the single-cloud path
  size_t offs = 0, ord = 0, errs = 0, queue = 0, scratch = 0, grades = 0, plain = 0,
         plain_bytes = 0, total = 0;
};

int device_cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// `cap_bytes` (0 = none) caps the workspace: the workgroup count is lowered
// until the per-workgroup scratch fits, and ENOMEM results when even one
// workgroup does not.
int plan_batch(const int64_t* offsets, int64_t nclouds, int32_t d, ph0_dtype dt,
               const ph0_batch_tuning* tune, BatchPlan* P, size_t cap_bytes = 0) {
  if (!offsets) return fail(PH0_EINVAL, "offsets pointer is NULL");
  if (nclouds < 1) return fail(PH0_EINVAL, "nclouds must be >= 1");
  if (d < 1) return fail(PH0_EINVAL, "d must be >= 1");
  if (dt != PH0_I8 && dt != PH0_I16) return fail(PH0_EINVAL, "dtype must be PH0_I8 or PH0_I16");
  if (offsets[0] != 0) return fail(PH0_EINVAL, "offsets[0] must be 0");
  if (tune && (tune->digit_bits < 0 || tune->digit_bits > 8))
    return fail(PH0_EINVAL, "tuning: digit_bits must be 0..8 (got %d)", tune->digit_bits);
  if (tune && tune->waves_per_cloud != 0 && tune->waves_per_cloud != 8 &&
      tune->waves_per_cloud != 16)
    return fail(PH0_EINVAL, "tuning: waves_per_cloud must be 0, 8 or 16 (got %d)",
                tune->waves_per_cloud);
  P->nclouds = nclouds;
  std::vector<std::pair<int64_t, int32_t>> bysize;
  for (int64_t c = 0; c < nclouds; ++c) {
    const int64_t n = offsets[c + 1] - offsets[c];
    if (n < 0) return fail(PH0_EINVAL, "offsets must be non-decreasing (cloud %lld)", (long long)c);
    if (n > kMaxN) return fail(PH0_EINVAL, "cloud %lld has n > %lld", (long long)c, (long long)kMaxN);
    if (n > kBatchMaxN || n * d > kBatchMaxPts || d > 64) {
      P->big.push_back((int32_t)c);
      P->big_n = std::max(P->big_n, n);
    } else {
      bysize.push_back({n, (int32_t)c});
      P->emax = std::max(P->emax, n * (n - 1) / 2);
    }
  }
  std::stable_sort(bysize.begin(), bysize.end(),
                   [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                     return x.first > y.first;
                   });
  for (auto& e : bysize) P->order.push_back(e.second);
  const int bpc = tune && tune->blocks_per_cu > 0 ? std::min(tune->blocks_per_cu, 2) : kBlocksPerCu;
  P->blocks = std::min<int64_t>((int64_t)device_cu_count() * bpc,
                                std::max<int64_t>((int64_t)P->order.size(), 1));
  if (P->big_n > 0) {
    if (ph0_workspace_bytes(P->big_n, d, dt, &P->plain_bytes) != PH0_OK) return PH0_EINVAL;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  P->offs = take(8 * (size_t)(nclouds + 1));
  P->ord = take(4 * std::max<size_t>(P->order.size(), 1));
  P->errs = take(4 * (size_t)nclouds);
  P->queue = take(4);
  const size_t per_block = 20 * (size_t)std::max<int64_t>(P->emax, 1);  // 2 keys + a grade
  if (cap_bytes) {
    const size_t fixed = o + 2 * kAlign + P->plain_bytes;
    const int64_t fit = cap_bytes > fixed ? (int64_t)((cap_bytes - fixed) / per_block) : 0;
    if (fit < 1)
      return fail(PH0_ENOMEM,
                  "the batch needs %zu bytes of fixed workspace plus %zu per workgroup; "
                  "only %zu are available", fixed, per_block, cap_bytes);
    P->blocks = std::min<int64_t>(P->blocks, fit);
  }
  P->scratch = take(16 * (size_t)std::max<int64_t>(P->emax, 1) * (size_t)P->blocks);
  P->grades = take(4 * (size_t)std::max<int64_t>(P->emax, 1) * (size_t)P->blocks);
  P->plain = take(P->plain_bytes);
  P->total = o;
  return PH0_OK;
}

// ---- H1 path ----

struct H1Layout {
  int64_t E = 0, T = 0, LWE = 0, cap = 0;
  size_t h0 = 0, h0_bytes = 0, keys = 0, inv = 0, grade = 0, cnt = 0, start = 0, scan = 0,
         tri = 0, owner = 0, lowc = 0, table = 0, surv = 0, clist = 0, wlist = 0, store = 0,
         sadds = 0, packed = 0,
         sorted = 0, rcounts = 0, rerr = 0, ctl = 0, total = 0;
};

int plan_h1(int64_t n, int32_t d, ph0_dtype dt, H1Layout* L) {
  L->E = n * (n - 1) / 2;
  L->T = n * (n - 1) * (n - 2) / 6;
  L->LWE = (L->E + 63) / 64;
  if (ph0_workspace_bytes(n, d, dt, &L->h0_bytes) != PH0_OK) return PH0_EINVAL;
  const int64_t E1 = std::max<int64_t>(L->E, 1), T1 = std::max<int64_t>(L->T, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L->h0 = take(L->h0_bytes);
  L->keys = take(8 * (size_t)E1);
  L->inv = take(4 * (size_t)E1);
  L->grade = take(4 * (size_t)E1);
  L->cnt = take(4 * (size_t)E1);
  L->start = take(4 * (size_t)(E1 + 1));
  L->scan = take(4 * (size_t)scan_totals_len(E1 + 1));
  L->tri = take(8 * (size_t)T1);
  L->owner = take(4 * (size_t)E1);
  L->lowc = take(8 * (size_t)E1);
  L->table = take(8 * (size_t)E1 * (size_t)std::max<int64_t>(L->LWE, 1));
  L->surv = take(8 * (size_t)T1);
  L->clist = take(8 * (size_t)E1);
  L->wlist = take(4 * (size_t)T1);
  L->cap = std::min<int64_t>(L->T, kH1StoreBytes / (8 * std::max<int64_t>(L->LWE, 1)));
  L->store = take(8 * (size_t)std::max<int64_t>(L->cap, 1) * (size_t)std::max<int64_t>(L->LWE, 1));
  L->sadds = take(4 * (size_t)std::max<int64_t>(L->cap, 1));
  L->packed = take(8 * (size_t)E1);
  L->sorted = take(8 * (size_t)E1);
  L->rcounts = take(4 * (size_t)radix_count_entries(E1));
  L->rerr = take(4);
  L->ctl = take(sizeof(H1Ctl));
  L->total = o;
  return PH0_OK;
}

int check_h1_args(const void* p, ph0_dtype dt, int64_t n, int32_t d) {
  int rc = check_args(p, dt, n, d);
  if (rc) return rc;
  if (n > kH1MaxN)
    return fail(PH0_ERANGE, "H1 supports n <= %lld (dense stored columns of n(n-1)/2 bits); "
                "got %lld", (long long)kH1MaxN, (long long)n);
  return PH0_OK;
}

struct DeviceBuffer {
  void* p = nullptr;
  ~DeviceBuffer() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

const char* ph0_last_error(void) { return g_err; }

int ph0_workspace_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes) {
  static const char probe = 0;
  int rc = check_args(&probe, dt, n, d);
  if (rc) return rc;
  if (!bytes) return fail(PH0_EINVAL, "bytes pointer is NULL");
  *bytes = make_layout(n, d).total;
  return PH0_OK;
}

int ph0_key_layout(int64_t n, int32_t d, ph0_dtype dt, int32_t* ibits, int32_t* dbits) {
  static const char probe = 0;
  int rc = check_args(&probe, dt, n, d);
  if (rc) return rc;
  const int ib = index_bits(n);
  const uint64_t span = dt == PH0_I8 ? 255 : 65535;
  unsigned __int128 bound = (unsigned __int128)d * span * span;
  int db = 0;
  while (db < 100 && (bound >> db) != 0) ++db;
  if (ibits) *ibits = ib;
  if (dbits) *dbits = db;
  if (2 * ib + db > 64)
    return fail(PH0_ERANGE, "full-range coordinates need %d + 2 x %d > 64 key bits", db, ib);
  return PH0_OK;
}

int ph0_workspace_bytes_f32(int64_t n, int32_t d, size_t* bytes) {
  size_t b = 0;
  const int rc = ph0_workspace_bytes(n, d, PH0_I16, &b);
  if (rc) return rc;
  if (!bytes) return fail(PH0_EINVAL, "bytes pointer is NULL");
  // The points on the int16 grid, the off-grid flag, then the int16 call's workspace.
  *bytes = align_up(2 * (size_t)n * (size_t)d) + align_up(4) + b;
  return PH0_OK;
}

int ph0_barcodes_f32_device(const float* d_points, int64_t n, int32_t d, double lo, double hi,
                            ph0_bar* d_out, void* d_ws, size_t ws_bytes, void* hip_stream,
                            ph0_stats* st) {
  if (!d_points) return fail(PH0_EINVAL, "points pointer is NULL");
  if (!d_out) return fail(PH0_EINVAL, "output pointer is NULL");
  if (!d_ws) return fail(PH0_EINVAL, "workspace pointer is NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi))
    return fail(PH0_EINVAL, "the coordinate interval needs finite lo < hi");
  size_t need = 0;
  int rc = ph0_workspace_bytes_f32(n, d, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return fail(PH0_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  char* ws = static_cast<char*>(d_ws);
  int16_t* q = reinterpret_cast<int16_t*>(ws);
  const size_t qb = align_up(2 * (size_t)n * (size_t)d);
  int32_t* qerr = reinterpret_cast<int32_t*>(ws + qb);
  char* rest = ws + qb + align_up(4);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  CtlReadback* rb = pinned_ctl();
  if (!rb) return fail(PH0_ENOMEM, "pinned host allocation failed");
  HIPCHK(launch_quantize_f32(d_points, n * (int64_t)d, lo, 32767.0 / (hi - lo), q, qerr, s));
  {
    Gather g;
    g.add(qerr, &rb->words[3], 4);
    HIPCHK(launch_gather(g, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (rb->words[3]) return fail(PH0_EINVAL, "a coordinate is outside [lo, hi] or not finite");
  Outputs o;
  o.bars = d_out;
  return run(q, PH0_I16, n, d, o, rest, ws_bytes - (size_t)(rest - ws), s, st, kStopAll);
}

int ph0_set_window(int64_t columns) {
  if (columns < 0) return fail(PH0_EINVAL, "window must be >= 0");
  g_window.store(columns);
  return PH0_OK;
}

int ph0_barcodes_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                        ph0_bar* d_out, void* d_ws, size_t ws_bytes, void* hip_stream,
                        ph0_stats* st) {
  if (!d_out) return fail(PH0_EINVAL, "output pointer is NULL");
  Outputs o;
  o.bars = d_out;
  return run(d_points, dt, n, d, o, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream), st,
             kStopAll);
}

int ph0_pairs_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                     uint32_t* d_death_by_vertex, int64_t* d_killer_pos,
                     uint64_t* d_killer_edge, int64_t* d_killer_sqdist, int32_t* d_partner,
                     void* d_ws, size_t ws_bytes, void* hip_stream, ph0_stats* st) {
  Outputs o;
  o.dbv = d_death_by_vertex;
  o.killer_pos = d_killer_pos;
  o.killer_edge = d_killer_edge;
  o.killer_sqdist = d_killer_sqdist;
  o.partner = d_partner;
  return run(d_points, dt, n, d, o, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream), st,
             kStopAll);
}

int ph0_keys_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d, uint64_t* d_keys,
                    void* d_ws, size_t ws_bytes, void* hip_stream) {
  if (!d_keys && n > 1) return fail(PH0_EINVAL, "keys pointer is NULL");
  Outputs o;
  o.keys = d_keys;
  return run(d_points, dt, n, d, o, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream),
             nullptr, kStopKeys);
}

int ph0_sorted_keys_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d,
                           uint64_t* d_keys, void* d_ws, size_t ws_bytes, void* hip_stream) {
  if (!d_keys && n > 1) return fail(PH0_EINVAL, "keys pointer is NULL");
  Outputs o;
  o.keys = d_keys;
  return run(d_points, dt, n, d, o, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream),
             nullptr, kStopSorted);
}

int ph0_batched_workspace_bytes(const int64_t* offsets, int64_t nclouds, int32_t d,
                                ph0_dtype dt, const ph0_batch_tuning* tune, size_t* bytes) {
  if (!bytes) return fail(PH0_EINVAL, "bytes pointer is NULL");
  BatchPlan P;
  int rc = plan_batch(offsets, nclouds, d, dt, tune, &P);
  if (rc) return rc;
  *bytes = P.total;
  return PH0_OK;
}

}  // extern "C"

namespace {

// The batched call once its plan is made and its workspace (P.total bytes
// at ws) is known: copies of the offsets and the processing order, the
// fused launch, the single-cloud path for the clouds it does not take, and
// the per-cloud error codes.
int batched_run(const void* d_points, ph0_dtype dt, const int64_t* offsets, int64_t nclouds,
                int32_t d, ph0_bar* d_out, char* ws, const BatchPlan& P,
                const ph0_batch_tuning* tune, hipStream_t s, ph0_stats* st) {
  int rc = PH0_OK;
  const int eb = dt == PH0_I8 ? 1 : 2;
  PoolScope pool_scope;
  StreamDrain drain(s);
  Timer tm(st != nullptr, s);
  tm.mark();
  HIPCHK(hipMemcpyAsync(ws + P.offs, offsets, 8 * (size_t)(nclouds + 1), hipMemcpyHostToDevice, s));
  if (!P.order.empty())
    HIPCHK(hipMemcpyAsync(ws + P.ord, P.order.data(), 4 * P.order.size(), hipMemcpyHostToDevice,
                          s));
  HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + P.errs), 0u, nclouds, s));
  HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + P.queue), 0u, 1, s));
  if (!P.order.empty()) {
    BatchArgs A;
    A.pts = d_points;
    A.elem_bytes = eb;
    A.d = d;
    A.offsets = reinterpret_cast<const int64_t*>(ws + P.offs);
    A.order = reinterpret_cast<const int32_t*>(ws + P.ord);
    A.nclouds = (int64_t)P.order.size();
    A.bars = reinterpret_cast<uint32_t*>(d_out);
    A.scratch = reinterpret_cast<uint64_t*>(ws + P.scratch);
    A.grades = reinterpret_cast<uint32_t*>(ws + P.grades);
    A.emax = std::max<int64_t>(P.emax, 1);
    A.queue = reinterpret_cast<uint32_t*>(ws + P.queue);
    A.errs = reinterpret_cast<int32_t*>(ws + P.errs);
    for (int b = 0; b < 4; ++b)
      A.chunk_mult[b] = tune && tune->chunk_mult[b] > 0 ? tune->chunk_mult[b] : kChunkMult[b];
    A.digit_bits = tune && tune->digit_bits > 0 ? tune->digit_bits : kDigitBits;
    A.threads = 64 * (tune && tune->waves_per_cloud > 0 ? tune->waves_per_cloud : kWavesPerCloud);
    HIPCHK(launch_batched(A, (int)P.blocks, s));
  }
  tm.mark();
  for (int32_t c : P.big) {
    const int64_t n = offsets[c + 1] - offsets[c];
    Outputs o;
    o.bars = d_out + offsets[c];
    rc = run(static_cast<const char*>(d_points) + offsets[c] * d * eb, dt, n, d, o, ws + P.plain,
             P.plain_bytes, s, nullptr, kStopAll);
    if (rc) return rc;
  }
  tm.mark();
  std::vector<int32_t> errs((size_t)nclouds);
  HIPCHK(hipMemcpyAsync(errs.data(), ws + P.errs, 4 * (size_t)nclouds, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  drain.armed = false;
  for (int64_t c = 0; c < nclouds; ++c)
    if (errs[c])
      return fail(errs[c] == 3 ? PH0_ERANGE : PH0_EDEVICE,
                  "cloud %lld failed in the batched kernel (code %d)", (long long)c, errs[c]);
  if (st) {
    ph0_stats S = {};
    S.n = offsets[nclouds];
    S.ms_reduce = tm.ms(0, 1);
    S.ms_emit = tm.ms(1, 2);
    S.ms_total = tm.ms(0, 2);
    *st = S;
  }
  return PH0_OK;
}

}  // namespace

extern "C" {

int ph0_barcodes_batched_device(const void* d_points, ph0_dtype dt, const int64_t* offsets,
                                int64_t nclouds, int32_t d, ph0_bar* d_out, void* d_ws,
                                size_t ws_bytes, const ph0_batch_tuning* tune,
                                void* hip_stream, ph0_stats* st) {
  if (!d_points) return fail(PH0_EINVAL, "points pointer is NULL");
  if (!d_out) return fail(PH0_EINVAL, "output pointer is NULL");
  if (!d_ws) return fail(PH0_EINVAL, "workspace pointer is NULL");
  BatchPlan P;
  int rc = plan_batch(offsets, nclouds, d, dt, tune, &P);
  if (rc) return rc;
  if (ws_bytes < P.total)
    return fail(PH0_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
  return batched_run(d_points, dt, offsets, nclouds, d, d_out, static_cast<char*>(d_ws), P, tune,
                     static_cast<hipStream_t>(hip_stream), st);
}

}  // extern "C"

// Workspace of ph0_barcodes_batched_device_noalloc: a fixed device array, so
// that the call allocates nothing.  Host code never passes this name to a
// kernel or a copy (in host code it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// Address of `scratch` on the current device (each device holds its own copy
// of the array), looked up on the first call made on that device.
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PH0_EDEVICE, "device %d is beyond the %d devices supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PH0_EDEVICE, "no device address for the fixed scratch array");
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return PH0_OK;
}

}  // namespace

extern "C" {

int ph0_barcodes_batched_device_noalloc(const void* d_points, ph0_dtype dt,
                                        const int64_t* offsets, int64_t nclouds, int32_t d,
                                        ph0_bar* d_out, const ph0_batch_tuning* tune,
                                        void* hip_stream) {
  if (!d_points) return fail(PH0_EINVAL, "points pointer is NULL");
  if (!d_out) return fail(PH0_EINVAL, "output pointer is NULL");
  BatchPlan P;
  int rc = plan_batch(offsets, nclouds, d, dt, tune, &P);
  if (rc) return rc;
  if (!P.big.empty()) {
    const int32_t c = P.big.front();
    return fail(PH0_EINVAL,
                "cloud %d (n = %lld, d = %d) is too large for the allocation-free call: it "
                "takes clouds with n <= %d, n * d <= %d and d <= 64 only",
                c, (long long)(offsets[c + 1] - offsets[c]), d, kBatchMaxN, kBatchMaxPts);
  }
  P = BatchPlan();
  if ((rc = plan_batch(offsets, nclouds, d, dt, tune, &P, kNoAllocScratchBytes))) return rc;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return batched_run(d_points, dt, offsets, nclouds, d, d_out, static_cast<char*>(ws), P, tune,
                     static_cast<hipStream_t>(hip_stream), nullptr);
}

int ph0_h1_workspace_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes) {
  static const char probe = 0;
  int rc = check_h1_args(&probe, dt, n, d);
  if (rc) return rc;
  if (!bytes) return fail(PH0_EINVAL, "bytes pointer is NULL");
  H1Layout L;
  if ((rc = plan_h1(n, d, dt, &L))) return rc;
  *bytes = L.total;
  return PH0_OK;
}

int ph0_h1_device(const void* d_points, ph0_dtype dt, int64_t n, int32_t d, ph0_bar* d_bars,
                  int64_t* d_tri_of_edge, int64_t* n_bars, void* d_ws, size_t ws_bytes,
                  void* hip_stream, ph0_h1_stats* st) {
  int rc = check_h1_args(d_points, dt, n, d);
  if (rc) return rc;
  if (!n_bars) return fail(PH0_EINVAL, "n_bars pointer is NULL");
  if (!d_ws) return fail(PH0_EINVAL, "workspace pointer is NULL");
  H1Layout L;
  if ((rc = plan_h1(n, d, dt, &L))) return rc;
  if (ws_bytes < L.total)
    return fail(PH0_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  if (!d_bars && L.E - n + 1 > 0) return fail(PH0_EINVAL, "bars pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char* ws = static_cast<char*>(d_ws);
  auto at = [&](size_t off) { return static_cast<void*>(ws + off); };
  ph0_h1_stats S = {};
  S.E = L.E;
  S.T = L.T;
  *n_bars = 0;
  PoolScope pool_scope;
  StreamDrain drain(s);
  Timer tm(st != nullptr, s);
  tm.mark();
  if (n < 3) {  // no triangle, no cycle
    if (d_tri_of_edge && L.E > 0) HIPCHK(launch_fill_u64((uint64_t*)d_tri_of_edge, ~0ull, L.E, s));
    HIPCHK(hipStreamSynchronize(s));
    drain.armed = false;
    if (st) *st = S;
    return PH0_OK;
  }
  uint64_t* keys = static_cast<uint64_t*>(at(L.keys));
  if ((rc = ph0_sorted_keys_device(d_points, dt, n, d, keys, at(L.h0), L.h0_bytes, s)))
    return rc;
  H1Args A;
  A.keys = keys;
  A.ib = index_bits(n);
  A.n = n;
  A.E = L.E;
  A.T = L.T;
  A.LWE = L.LWE;
  A.inv = static_cast<int32_t*>(at(L.inv));
  A.grade = static_cast<uint32_t*>(at(L.grade));
  A.cnt = static_cast<uint32_t*>(at(L.cnt));
  A.start = static_cast<uint32_t*>(at(L.start));
  A.scan_tmp = static_cast<uint32_t*>(at(L.scan));
  A.tri = static_cast<uint64_t*>(at(L.tri));
  A.owner = static_cast<int32_t*>(at(L.owner));
  A.lowc = static_cast<uint64_t*>(at(L.lowc));
  A.table = static_cast<uint64_t*>(at(L.table));
  A.surv = static_cast<uint64_t*>(at(L.surv));
  A.clist = static_cast<uint64_t*>(at(L.clist));
  A.wlist = static_cast<uint32_t*>(at(L.wlist));
  A.store = static_cast<uint64_t*>(at(L.store));
  A.sadds = static_cast<uint32_t*>(at(L.sadds));
  A.cap = L.cap;
  A.nsurv_host = 0;
  A.cus = device_cu_count();
  A.ctl = static_cast<H1Ctl*>(at(L.ctl));
  H1Ctl c0 = {};
  c0.T = L.T;
  c0.firstdup = ~0ull;
  HIPCHK(hipMemcpyAsync(A.ctl, &c0, sizeof(c0), hipMemcpyHostToDevice, s));
  HIPCHK(launch_h1_setup(A, s));
  tm.mark();
  // Rounds until every column is final.  Every round after the first
  // commits at least its smallest live survivor, so there are at most
  // E - n + 2 of them.
  H1Ctl hc = {};
  uint32_t tcount = 0;
  HIPCHK(hipMemcpyAsync(&tcount, A.start + L.E, 4, hipMemcpyDeviceToHost, s));
  int64_t rounds = 0;
  for (bool first = true;; first = false) {
    HIPCHK(launch_h1_round(A, first, s));
    ++rounds;
    HIPCHK(hipMemcpyAsync(&hc, A.ctl, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hc.err)
      return fail(PH0_EDEVICE, "H1 reduction: %s (round %lld)",
                  (hc.err & 2) ? "a stored column's top bit is not its row" :
                                 "a repeated walk diverged", (long long)rounds);
    if (hc.live == 0) break;
    if (rounds > L.E - n + 2)
      return fail(PH0_EDEVICE, "H1 reduction made no progress after %lld rounds",
                  (long long)rounds);
    A.nsurv_host = hc.nsurv;
  }
  if ((int64_t)tcount != L.T)
    return fail(PH0_EDEVICE, "H1 triangle count %u != %lld", tcount, (long long)L.T);
  tm.mark();
  uint64_t* packed = static_cast<uint64_t*>(at(L.packed));
  HIPCHK(launch_h1_bars(A, packed, s));
  HIPCHK(hipMemcpyAsync(&hc, A.ctl, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hc.stored != L.E - n + 1)
    return fail(PH0_EDEVICE, "H1 reduction stored %lld pivots, expected E - n + 1 = %lld",
                (long long)hc.stored, (long long)(L.E - n + 1));
  const int64_t m = hc.nbars;
  // Canonical order: (birth, death) ascending, by LSD passes over the
  // packed birth << 20 | death (grades are below 2^20 for n <= 512).
  uint64_t* src = packed;
  uint64_t* dst = static_cast<uint64_t*>(at(L.sorted));
  if (m > 1) {
    for (int sh = 0; sh < 40; sh += 8) {
      HIPCHK(launch_radix_pass(src, dst, m, sh, 8, static_cast<uint32_t*>(at(L.rcounts)),
                               static_cast<int32_t*>(at(L.rerr)), s));
      std::swap(src, dst);
    }
  }
  HIPCHK(launch_h1_bars_out(src, m, reinterpret_cast<uint32_t*>(d_bars), s));
  if (d_tri_of_edge) HIPCHK(launch_h1_owner_out(A.owner, L.E, d_tri_of_edge, s));
  tm.mark();
  HIPCHK(hipStreamSynchronize(s));
  drain.armed = false;
  *n_bars = m;
  if (st) {
    S.rounds = rounds;
    S.pivots = hc.stored;
    S.emergent = hc.stored - hc.pivots;
    S.bars = m;
    S.zero_length = hc.stored - m;
    S.additions = hc.additions;
    S.walks = hc.walks;
    S.ms_setup = tm.ms(0, 1);
    S.ms_reduce = tm.ms(1, 2);
    S.ms_total = tm.ms(0, 3);
    *st = S;
  }
  return PH0_OK;
}

}  // extern "C"

namespace {

// Tuning text of ph0_barcodes_batched: a JSON object whose only members are
// "chunk_mult" (an array of up to four non-negative integers),
// "blocks_per_cu", "digit_bits" and "waves_per_cloud" (non-negative
// integers), e.g.
//   {"chunk_mult": [6, 6, 8, 48], "blocks_per_cu": 2, "digit_bits": 8, "waves_per_cloud": 8}
// Anything else is rejected, so a misspelt key cannot pass silently.
struct JsonCursor {
  const char* p;
  void ws() {
    while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
  }
  bool eat(char c) {
    ws();
    if (*p != c) return false;
    ++p;
    return true;
  }
  bool integer(int32_t* v) {
    ws();
    if (*p < '0' || *p > '9') return false;
    int64_t x = 0;
    while (*p >= '0' && *p <= '9') {
      x = 10 * x + (*p++ - '0');
      if (x > 1000000) return false;
    }
    *v = (int32_t)x;
    return true;
  }
  bool key(char* buf, size_t cap) {
    if (!eat('"')) return false;
    size_t k = 0;
    while (*p && *p != '"') {
      if (k + 1 >= cap) return false;
      buf[k++] = *p++;
    }
    buf[k] = 0;
    if (*p != '"') return false;
    ++p;
    return true;
  }
};

int parse_tuning(const char* text, ph0_batch_tuning* t) {
  *t = ph0_batch_tuning{};
  JsonCursor c{text};
  if (!c.eat('{')) return fail(PH0_EINVAL, "tuning: expected a JSON object");
  bool closed = c.eat('}');
  while (!closed) {
    char k[32];
    if (!c.key(k, sizeof(k)) || !c.eat(':')) return fail(PH0_EINVAL, "tuning: expected \"key\":");
    if (!strcmp(k, "chunk_mult")) {
      if (!c.eat('[')) return fail(PH0_EINVAL, "tuning: chunk_mult must be an array");
      int m = 0;
      if (!c.eat(']')) {
        while (true) {
          if (m >= 4 || !c.integer(&t->chunk_mult[m++]))
            return fail(PH0_EINVAL, "tuning: chunk_mult takes up to 4 non-negative integers");
          if (c.eat(']')) break;
          if (!c.eat(',')) return fail(PH0_EINVAL, "tuning: expected ',' or ']'");
        }
      }
    } else if (!strcmp(k, "blocks_per_cu")) {
      if (!c.integer(&t->blocks_per_cu))
        return fail(PH0_EINVAL, "tuning: blocks_per_cu must be a non-negative integer");
    } else if (!strcmp(k, "digit_bits")) {
      if (!c.integer(&t->digit_bits))
        return fail(PH0_EINVAL, "tuning: digit_bits must be a non-negative integer");
    } else if (!strcmp(k, "waves_per_cloud")) {
      if (!c.integer(&t->waves_per_cloud))
        return fail(PH0_EINVAL, "tuning: waves_per_cloud must be a non-negative integer");
    } else {
      return fail(PH0_EINVAL, "tuning: unknown key \"%s\"", k);
    }
    if (c.eat('}')) closed = true;
    else if (!c.eat(',')) return fail(PH0_EINVAL, "tuning: expected ',' or '}'");
  }
  c.ws();
  if (*c.p) return fail(PH0_EINVAL, "tuning: trailing text after the object");
  return PH0_OK;
}

}  // namespace

extern "C" {

int ph0_barcodes_batched(const void* points, ph0_dtype dt, const int64_t* offsets,
                         int64_t nclouds, int32_t d, ph0_bar* out, const char* tune_json,
                         ph0_stats* st) {
  if (!points) return fail(PH0_EINVAL, "points pointer is NULL");
  if (!out) return fail(PH0_EINVAL, "output pointer is NULL");
  ph0_batch_tuning tune = {};
  int rc = PH0_OK;
  if (tune_json && (rc = parse_tuning(tune_json, &tune))) return rc;
  size_t ws = 0;
  if ((rc = ph0_batched_workspace_bytes(offsets, nclouds, d, dt, &tune, &ws))) return rc;
  const int64_t rows = offsets[nclouds];
  const size_t pbytes = (size_t)rows * d * (dt == PH0_I8 ? 1 : 2);
  const size_t obytes = 8 * (size_t)rows;
  DeviceBuffer dp, dout, dws;
  if (hipMalloc(&dp.p, std::max<size_t>(pbytes, 1)) != hipSuccess ||
      hipMalloc(&dout.p, std::max<size_t>(obytes, 8)) != hipSuccess ||
      hipMalloc(&dws.p, ws) != hipSuccess)
    return fail(PH0_ENOMEM, "device allocation of %zu bytes failed", ws + pbytes + obytes);
  hipStream_t s;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (pbytes && hipMemcpyAsync(dp.p, points, pbytes, hipMemcpyHostToDevice, s) != hipSuccess)
    rc = fail(PH0_EDEVICE, "copy of points to the device failed");
  if (!rc)
    rc = ph0_barcodes_batched_device(dp.p, dt, offsets, nclouds, d,
                                     static_cast<ph0_bar*>(dout.p), dws.p, ws, &tune, s, st);
  if (!rc && obytes &&
      (hipMemcpyAsync(out, dout.p, obytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    rc = fail(PH0_EDEVICE, "copy of the barcodes to the host failed");
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

int ph0_barcodes(const void* points, ph0_dtype dt, int64_t n, int32_t d, ph0_bar* out,
                 ph0_stats* st) {
  int rc = check_args(points, dt, n, d);
  if (rc) return rc;
  if (!out) return fail(PH0_EINVAL, "output pointer is NULL");
  size_t ws = 0;
  if ((rc = ph0_workspace_bytes(n, d, dt, &ws))) return rc;
  const size_t pbytes = (size_t)n * d * (dt == PH0_I8 ? 1 : 2);
  DeviceBuffer dp, dout, dws;
  if (hipMalloc(&dp.p, pbytes) != hipSuccess || hipMalloc(&dout.p, 8 * (size_t)n) != hipSuccess ||
      hipMalloc(&dws.p, ws) != hipSuccess)
    return fail(PH0_ENOMEM, "device allocation of %zu bytes failed", ws + pbytes + 8 * n);
  hipStream_t s;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  rc = PH0_OK;
  if (hipMemcpyAsync(dp.p, points, pbytes, hipMemcpyHostToDevice, s) != hipSuccess)
    rc = fail(PH0_EDEVICE, "copy of points to the device failed");
  if (!rc)
    rc = ph0_barcodes_device(dp.p, dt, n, d, static_cast<ph0_bar*>(dout.p), dws.p, ws, s, st);
  if (!rc && (hipMemcpyAsync(out, dout.p, 8 * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = fail(PH0_EDEVICE, "copy of the barcode to the host failed");
  (void)hipStreamDestroy(s);
  return rc;
}

}  // extern "C"

// ---- serving ----

namespace {

struct Request {
  uint64_t tag = 0;
  int64_t n = 0;
  int32_t d = 0;
  ph0_dtype dt = PH0_I8;
  std::vector<char> pts;
  std::vector<ph0_bar> bars;
  int32_t status = PH0_OK;
  size_t off = 0, bytes = 0;  // pool region
};

// First-fit allocator over [0, size) of the device pool.
class PoolAllocator {
 public:
  explicit PoolAllocator(size_t size) { free_[0] = size; }
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

size_t request_bytes(int64_t n, int32_t d, ph0_dtype dt) {
  size_t ws = 0;
  if (ph0_workspace_bytes(n, d, dt, &ws) != PH0_OK) return 0;
  return align_up((size_t)n * d * (dt == PH0_I8 ? 1 : 2)) + align_up(8 * (size_t)n) + ws;
}

}  // namespace

struct ph0_server {
  size_t budget = 0;
  char* pool = nullptr;
  PoolAllocator* alloc = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;   // admitted, waiting for a worker
  std::deque<Request*> finished;  // done, waiting for poll
  std::vector<std::thread> workers;
  int32_t slots = 0;
  int32_t busy = 0;  // admitted and not finished
  int64_t in_flight = 0;
  bool stop = false;
};

namespace {

void serve_worker(ph0_server* S) {
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  while (true) {
    Request* R = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->pending.empty(); });
      if (S->pending.empty()) break;
      R = S->pending.front();
      S->pending.pop_front();
    }
    char* base = S->pool + R->off;
    const size_t pbytes = (size_t)R->n * R->d * (R->dt == PH0_I8 ? 1 : 2);
    char* dpts = base;
    ph0_bar* dout = reinterpret_cast<ph0_bar*>(base + align_up(pbytes));
    char* ws = base + align_up(pbytes) + align_up(8 * (size_t)R->n);
    const size_t ws_bytes = R->bytes - align_up(pbytes) - align_up(8 * (size_t)R->n);
    int rc = PH0_OK;
    if (!s) rc = fail(PH0_EDEVICE, "stream creation failed");
    if (!rc && hipMemcpyAsync(dpts, R->pts.data(), pbytes, hipMemcpyHostToDevice, s) != hipSuccess)
      rc = fail(PH0_EDEVICE, "copy of points failed");
    if (!rc) {
      Outputs o;
      o.bars = dout;
      rc = run(dpts, R->dt, R->n, R->d, o, ws, ws_bytes, s, nullptr, kStopAll);
    }
    R->bars.resize((size_t)R->n);
    if (!rc && (hipMemcpyAsync(R->bars.data(), dout, 8 * (size_t)R->n, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
      rc = fail(PH0_EDEVICE, "copy of the barcode failed");
    // Whatever the outcome, nothing of this request may still run on the
    // stream when its pool region goes to the next request.
    if (s) (void)hipStreamSynchronize(s);
    R->status = rc;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->alloc->give(R->off, R->bytes);
      S->busy -= 1;
      S->finished.push_back(R);
    }
  }
  if (s) (void)hipStreamDestroy(s);
  release_thread_resources();
}

}  // namespace

extern "C" {

int ph0_server_request_bytes(int64_t n, int32_t d, ph0_dtype dt, size_t* bytes) {
  static const char probe = 0;
  int rc = check_args(&probe, dt, n, d);
  if (rc) return rc;
  if (!bytes) return fail(PH0_EINVAL, "bytes pointer is NULL");
  *bytes = request_bytes(n, d, dt);
  return PH0_OK;
}

int ph0_server_create(size_t mem_budget_bytes, int32_t max_slots, ph0_server** srv) {
  if (!srv) return fail(PH0_EINVAL, "server pointer is NULL");
  if (max_slots < 1 || max_slots > 64) return fail(PH0_EINVAL, "max_slots must be in 1..64");
  if (mem_budget_bytes < 4096) return fail(PH0_EINVAL, "memory budget too small");
  ph0_server* S = new ph0_server();
  S->budget = mem_budget_bytes;
  if (hipMalloc((void**)&S->pool, mem_budget_bytes) != hipSuccess) {
    delete S;
    return fail(PH0_ENOMEM, "device pool of %zu bytes could not be allocated", mem_budget_bytes);
  }
  S->alloc = new PoolAllocator(mem_budget_bytes);
  S->slots = max_slots;
  for (int k = 0; k < max_slots; ++k) S->workers.emplace_back(serve_worker, S);
  *srv = S;
  return PH0_OK;
}

int ph0_server_submit(ph0_server* S, const void* points, ph0_dtype dt, int64_t n, int32_t d,
                      uint64_t tag) {
  if (!S) return fail(PH0_EINVAL, "server is NULL");
  int rc = check_args(points, dt, n, d);
  if (rc) return rc;
  const size_t need = request_bytes(n, d, dt);
  if (need > S->budget)
    return fail(PH0_ENOMEM, "request needs %zu bytes, the pool holds %zu", need, S->budget);
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->busy >= S->slots) return fail(PH0_EBUSY, "all %d slots are busy", S->slots);
  size_t off = 0;
  if (!S->alloc->take(need, &off)) return fail(PH0_EBUSY, "not enough free pool memory now");
  Request* R = new Request();
  R->tag = tag;
  R->n = n;
  R->d = d;
  R->dt = dt;
  R->off = off;
  R->bytes = need;
  const size_t pbytes = (size_t)n * d * (dt == PH0_I8 ? 1 : 2);
  R->pts.assign(static_cast<const char*>(points), static_cast<const char*>(points) + pbytes);
  S->busy += 1;
  S->in_flight += 1;
  S->pending.push_back(R);
  lk.unlock();
  S->cv.notify_one();
  return PH0_OK;
}

int ph0_server_poll(ph0_server* S, uint64_t* tag, int32_t* status, ph0_bar* out, int64_t out_cap,
                    int64_t* n_out) {
  if (!S) return fail(PH0_EINVAL, "server is NULL");
  Request* R = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->finished.empty()) return 0;
    R = S->finished.front();
    S->finished.pop_front();
    S->in_flight -= 1;
  }
  if (tag) *tag = R->tag;
  if (status) *status = R->status;
  if (n_out) *n_out = R->n;
  if (out && R->status == PH0_OK)
    std::memcpy(out, R->bars.data(), 8 * (size_t)std::min<int64_t>(out_cap, R->n));
  delete R;
  return 1;
}

int64_t ph0_server_in_flight(ph0_server* S) {
  if (!S) return 0;
  std::lock_guard<std::mutex> lk(S->mu);
  return S->in_flight;
}

void ph0_server_destroy(ph0_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  for (Request* R : S->finished) delete R;
  if (S->pool) (void)hipFree(S->pool);
  delete S->alloc;
  delete S;
}

}  // extern "C"
