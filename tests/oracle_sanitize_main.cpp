// Driver for the sanitizer build of the CPU oracle (tests/test_oracle_sanitize.py):
// the oracle compiled with -fsanitize=address,undefined runs every entry point
// on small seeded clouds (tiny, tie-heavy, int8 extremes, int16 spreads) and
// checks the invariants every barcode has: n bars, one infinite, n - 1 pivots,
// literal mode equal to early exit; H1 gives E - n + 1 pairs and the same bars
// in both modes.  Any memory or
// undefined-behaviour error aborts the run with the sanitizer's report.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

extern "C" {
typedef struct {
  int64_t E, E_eff, distinct, additions, pivots, columns, late_nonzero, not_two_sparse;
  double s_dist, s_sort, s_rank, s_reduce, s_emit;
} ph0o_stats;
typedef struct {
  int64_t E, T, T_eff, additions, pivots, zero_length, columns;
} ph0o_h1_stats;
int ph0o_sorted_edges(const void*, int, int64_t, int32_t, int64_t*, int64_t*, int32_t*, int32_t*,
                      uint32_t*, int64_t*);
int ph0o_barcode(const void*, int, int64_t, int32_t, int, uint32_t*, uint32_t*, int64_t*, int32_t*,
                 ph0o_stats*);
int ph0o_h1(const void*, int, int64_t, int32_t, int, int64_t*, uint32_t*, uint32_t*, int64_t,
            int64_t*, ph0o_h1_stats*);
}

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) {  // [lo, hi]
  return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1));
}

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

static int one(int eb, int64_t n, int32_t d, int64_t lo, int64_t hi) {
  std::vector<int8_t> p8;
  std::vector<int16_t> p16;
  if (eb == 1)
    for (int64_t k = 0; k < n * d; ++k) p8.push_back((int8_t)uniform(lo, hi));
  else
    for (int64_t k = 0; k < n * d; ++k) p16.push_back((int16_t)uniform(lo, hi));
  const void* pts = eb == 1 ? (const void*)p8.data() : (const void*)p16.data();
  const int64_t E = n * (n - 1) / 2;
  std::vector<uint32_t> dv(n), can(n), dv2(n), can2(n);
  std::vector<int64_t> kp(n), kp2(n);
  std::vector<int32_t> par(n), par2(n);
  ph0o_stats a, b;
  CHECK(ph0o_barcode(pts, eb, n, d, 1, dv.data(), can.data(), kp.data(), par.data(), &a) == 0);
  CHECK(ph0o_barcode(pts, eb, n, d, 0, dv2.data(), can2.data(), kp2.data(), par2.data(), &b) == 0);
  CHECK(a.E == E && a.pivots == n - 1 && b.pivots == n - 1);
  CHECK(b.late_nonzero == 0 && a.not_two_sparse == 0 && b.not_two_sparse == 0);
  CHECK(can[n - 1] == 0xFFFFFFFFu);
  for (int64_t k = 0; k + 1 < n; ++k) CHECK(can[k] != 0xFFFFFFFFu && can[k] <= can[k + 1]);
  for (int64_t k = 0; k < n; ++k) CHECK(can[k] == can2[k] && dv[k] == dv2[k] && par[k] == par2[k]);
  std::vector<int64_t> cd(E), de(E);
  std::vector<int32_t> jj(E), ii(E);
  std::vector<uint32_t> gg(E);
  int64_t nd = 0;
  CHECK(ph0o_sorted_edges(pts, eb, n, d, cd.data(), de.data(), jj.data(), ii.data(), gg.data(),
                          &nd) == 0);
  CHECK(nd == a.distinct);
  if (n <= 24) {
    const int64_t cap = E - n + 1 > 0 ? E - n + 1 : 0;
    std::vector<int64_t> toe(E > 0 ? E : 1);
    std::vector<uint32_t> hb(cap > 0 ? cap : 1), hd(cap > 0 ? cap : 1);
    int64_t nb = 0;
    ph0o_h1_stats hs, hs2;
    CHECK(ph0o_h1(pts, eb, n, d, 1, toe.data(), hb.data(), hd.data(), cap, &nb, &hs) == 0);
    CHECK(hs.pivots == cap);
    std::vector<uint32_t> hb2(hb.size()), hd2(hd.size());
    int64_t nb2 = 0;
    CHECK(ph0o_h1(pts, eb, n, d, 0, toe.data(), hb2.data(), hd2.data(), cap, &nb2, &hs2) == 0);
    CHECK(nb2 == nb && hs2.pivots == cap);
    for (int64_t k = 0; k < nb; ++k) CHECK(hb[k] == hb2[k] && hd[k] == hd2[k] && hb[k] < hd[k]);
  }
  return 0;
}

int main() {
  int cases = 0;
  for (int rep = 0; rep < 40; ++rep) {
    const int64_t n = uniform(1, 40);
    const int32_t d = (int32_t)uniform(1, 6);
    if (one(1, n, d, 0, 2)) return 1;          // heavy ties, duplicate points
    if (one(1, n, d, -128, 127)) return 1;     // int8 extremes
    if (one(2, n, d, -16000, 16000)) return 1;  // wide int16
    cases += 3;
  }
  if (one(1, 300, 16, -128, 127)) return 1;
  if (one(2, 257, 3, -100, 100)) return 1;
  printf("sanitized oracle: %d cases ok\n", cases + 2);
  return 0;
}
