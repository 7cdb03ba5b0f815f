// ph0_omp.cpp -- CPU TIMING BASELINE (test and benchmark infrastructure only).
//
// The multi-core CPU scheme of Section 3 ("Multi-Core CPU Parallelization")
// of Rawson, "Linear Run Time of Persistent Homology Computation with GPU
// Parallelization": the barcode algorithm of Section 2 with OpenMP
// work-sharing loops.  The pairwise distances are a parallel loop.  The column
// reduction keeps its outer loop over columns sequential (column p needs every
// earlier column reduced), and the loops inside it -- adding a stored column
// to the current one and finding the new lowest entry -- are work-shared, so
// every column addition opens one parallel region: the per-addition thread
// cost that Section 3 identifies as the limit of this scheme.
//
// Only the test suite and the benchmark's CPU legs load this file; the GPU
// library never does and shares no code with it.  It is written apart from
// the single-threaded oracle (ph0_oracle.cpp) too: columns here are dense
// arrays of N one-byte F2 coefficients, one per vertex row (a plain dense
// matrix column, as Section 2 describes M), not bitsets.  The tests require
// identical barcodes, per-vertex deaths and addition counts from both.
//
// Readings shared with the oracle (Section 2 is silent on them): squared
// distances; ties ordered by (j, i) with i < j; the low of a column is its
// largest row index; the vertex that never becomes a pivot carries the
// infinite bar; deaths are 1-based grades (indices in D).  Sorting is
// std::sort: Section 3 parallelizes loops only.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Pair {
  int64_t delta;
  int32_t j, i;  // i < j
};

double since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

template <typename T>
void distances(const T* x, int64_t n, int32_t d, std::vector<Pair>& out, int threads) {
  out.resize(static_cast<size_t>(n * (n - 1) / 2));
#pragma omp parallel for schedule(dynamic, 8) num_threads(threads)
  for (int64_t j = 1; j < n; ++j) {
    const int64_t base = j * (j - 1) / 2;
    for (int64_t i = 0; i < j; ++i) {
      int64_t s = 0;
      for (int32_t k = 0; k < d; ++k) {
        const int64_t t = static_cast<int64_t>(x[i * d + k]) - static_cast<int64_t>(x[j * d + k]);
        s += t * t;
      }
      out[static_cast<size_t>(base + i)] = Pair{s, static_cast<int32_t>(j), static_cast<int32_t>(i)};
    }
  }
}

}  // namespace

extern "C" {

#define PH0P_INF 0xFFFFFFFFu

typedef struct {
  int64_t E, E_eff, distinct, additions, pivots;
  int32_t threads;  // threads the parallel regions ran with
  int32_t reserved;
  double s_dist, s_sort, s_rank, s_reduce, s_emit;
} ph0p_stats;

// points: n x d int8 (elem_bytes 1) or int16 (2), row-major.  threads >= 1.
// early_exit != 0 stops the column loop at the (n-1)-th pivot (every later
// column reduces to zero).  death_by_vertex[n] and canonical[n] (deaths
// ascending, infinite last) may be NULL.  Returns 0, or -1 on bad arguments.
int ph0p_barcode(const void* points, int elem_bytes, int64_t n, int32_t d, int threads,
                 int early_exit, uint32_t* death_by_vertex, uint32_t* canonical,
                 ph0p_stats* st) {
  if (!points || (elem_bytes != 1 && elem_bytes != 2) || n < 1 || d < 1 || threads < 1)
    return -1;
  ph0p_stats s;
  std::memset(&s, 0, sizeof(s));
  s.E = n * (n - 1) / 2;
  s.threads = threads;

  auto t0 = std::chrono::steady_clock::now();
  std::vector<Pair> e;
  if (elem_bytes == 1)
    distances(static_cast<const int8_t*>(points), n, d, e, threads);
  else
    distances(static_cast<const int16_t*>(points), n, d, e, threads);
  s.s_dist = since(t0);

  t0 = std::chrono::steady_clock::now();
  std::sort(e.begin(), e.end(), [](const Pair& a, const Pair& b) {
    return a.delta != b.delta ? a.delta < b.delta : (a.j != b.j ? a.j < b.j : a.i < b.i);
  });
  s.s_sort = since(t0);

  // Grades: 1 + number of distance changes up to each sorted position.
  t0 = std::chrono::steady_clock::now();
  std::vector<uint32_t> grade(e.size());
  uint32_t g = 0;
  for (size_t p = 0; p < e.size(); ++p) {
    if (p == 0 || e[p].delta != e[p - 1].delta) ++g;
    grade[p] = g;
  }
  s.distinct = g;
  s.s_rank = since(t0);

  // Dense reduction: stored[r] is the reduced column whose low is r (n bytes).
  t0 = std::chrono::steady_clock::now();
  std::vector<uint8_t> stored(static_cast<size_t>(n * n), 0);
  std::vector<uint8_t> has(static_cast<size_t>(n), 0);
  std::vector<uint32_t> death(static_cast<size_t>(n), PH0P_INF);
  std::vector<uint8_t> col(static_cast<size_t>(n), 0);
  for (size_t p = 0; p < e.size(); ++p) {
    if (early_exit && s.pivots == n - 1) break;
    col[e[p].i] = 1;
    col[e[p].j] = 1;
    int64_t low = e[p].j;
    while (low >= 0 && has[low]) {
      const uint8_t* src = &stored[static_cast<size_t>(low * n)];
      uint8_t* c = col.data();
      int64_t next = -1;
      // One column addition: XOR the stored column in and find the new low.
#pragma omp parallel for reduction(max : next) num_threads(threads)
      for (int64_t v = 0; v < n; ++v) {
        c[v] ^= src[v];
        if (c[v] && v > next) next = v;
      }
      low = next;
      ++s.additions;
    }
    if (low >= 0) {
      std::memcpy(&stored[static_cast<size_t>(low * n)], col.data(), static_cast<size_t>(n));
      has[low] = 1;
      death[low] = grade[p];
      ++s.pivots;
      s.E_eff = static_cast<int64_t>(p) + 1;
      std::fill(col.begin(), col.end(), 0);
    }
    // a zero column leaves col all zero
  }
  s.s_reduce = since(t0);

  t0 = std::chrono::steady_clock::now();
  std::vector<uint32_t> sorted(death);
  std::sort(sorted.begin(), sorted.end());
  for (int64_t r = 0; r < n; ++r) {
    if (death_by_vertex) death_by_vertex[r] = death[r];
    if (canonical) canonical[r] = sorted[r];
  }
  s.s_emit = since(t0);
  if (st) *st = s;
  return 0;
}

}  // extern "C"
