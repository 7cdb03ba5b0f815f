// ph0_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU oracle for the 0th persistent homology
// barcode of a Vietoris-Rips filtration, written from Section 2 ("Barcode
// Algorithm") of Rawson, "Linear Run Time of Persistent Homology Computation
// with GPU Parallelization".  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the GPU library never does,
// and it shares no code, header or table with the GPU library.
//
// The steps, in the paper's order (Section 2; the GPU step list of Section 4):
//   1. distance of every pair of points            (squared Euclidean, int64)
//   2. sort the distance list E increasingly       (std::sort on (delta, j, i))
//   3. remove duplicates -> D; grade of edge = 1-based index of its distance in D
//   4. boundary matrix M: one column per edge, one row per vertex, entries
//      t^a at the edge's two vertices (t-grading carried as the column grade)
//   5. column-reduce M left to right until every nonzero column has a
//      distinct lowest entry (the "lower triangular" form)
//   6. each surviving pivot t^b gives the interval (0, b)
//
// Readings where the paper is silent (each also listed in the design notes):
//   * squared distances instead of distances: the square root is monotone,
//     so the sorted order, the duplicates and the grades are unchanged, and
//     integer arithmetic stays exact;
//   * equal distances are ordered by (j, i) with i < j (colex edge order);
//   * the lowest entry ("low") of a column is its largest row index, and only
//     earlier columns are added to later ones; "pivoting" = finding the
//     stored column that owns the current low;
//   * the vertex whose row never becomes a pivot gets the infinite bar;
//   * deaths are reported as the 1-based grade b (index in D).
//
// Columns are dense bitsets of N bits (ceil(N/64) words); a column addition
// XORs all words and the low is found by scanning from the top word down.
// Over F2 the powers of t only travel along: every entry of a column keeps
// the column's own grade (the added columns are earlier, hence of lower or
// equal grade, and the shift t^(a_j - a_k) restores the grade), so the
// reduction is carried out on the coefficient pattern and the grade of the
// column supplies b.
//
// Parity unpinned: none.  Every output is pinned in the test suite against
// something other than this file (Kruskal and union-find, brute-force
// component counts, closed forms, library distance/sort routines; for H1,
// persistent Betti numbers, the rank form of the pairing lemma and a
// set-based reduction).  The PH0O_PLANT_* switches plant known mistakes for
// the tests that show those pins catch them; the library is never built
// with them.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Edge {
  int64_t delta;
  int32_t j;  // larger endpoint
  int32_t i;  // smaller endpoint
};

bool edge_less(const Edge& a, const Edge& b) {
  if (a.delta != b.delta) return a.delta < b.delta;
  if (a.j != b.j) return a.j < b.j;
  return a.i < b.i;
}

int64_t coord(const void* pts, int elem_bytes, int64_t idx) {
  if (elem_bytes == 1) return static_cast<const int8_t*>(pts)[idx];
  return static_cast<const int16_t*>(pts)[idx];
}

// Step 1: squared Euclidean distance of every pair i < j, in colex order
// (j ascending, then i ascending).
std::vector<Edge> all_pairs(const void* pts, int elem_bytes, int64_t n, int32_t d) {
  std::vector<Edge> edges;
  if (n < 2) return edges;
  edges.reserve(static_cast<size_t>(n * (n - 1) / 2));
  for (int64_t j = 1; j < n; ++j) {
    for (int64_t i = 0; i < j; ++i) {
      int64_t s = 0;
      for (int32_t k = 0; k < d; ++k) {
        int64_t diff = coord(pts, elem_bytes, i * d + k) - coord(pts, elem_bytes, j * d + k);
        s += diff * diff;
      }
      edges.push_back(Edge{s, static_cast<int32_t>(j), static_cast<int32_t>(i)});
    }
  }
  return edges;
}

// Step 3: 1-based index in D of each sorted edge's distance.
std::vector<uint32_t> grades(const std::vector<Edge>& sorted, int64_t* distinct) {
  std::vector<uint32_t> g(sorted.size());
  uint32_t cur = 0;
  for (size_t p = 0; p < sorted.size(); ++p) {
    if (p == 0 || sorted[p].delta != sorted[p - 1].delta) ++cur;
    g[p] = cur;
  }
  *distinct = cur;
  return g;
}

// Highest set bit of a dense column, or -1 for the zero column.
int64_t low_of(const std::vector<uint64_t>& col) {
  for (int64_t w = static_cast<int64_t>(col.size()) - 1; w >= 0; --w) {
    if (col[w] != 0) return 64 * w + 63 - __builtin_clzll(col[w]);
  }
  return -1;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

#define PH0O_INF 0xFFFFFFFFu

typedef struct {
  int64_t E;          // number of edges N(N-1)/2
  int64_t E_eff;      // sorted position of the last pivot + 1
  int64_t distinct;   // |D|
  int64_t additions;  // column additions performed by the reduction
  int64_t pivots;     // nonzero reduced columns (N-1 for N >= 1)
  int64_t columns;    // columns visited by the reduction
  int64_t late_nonzero;  // literal mode: nonzero columns after E_eff (must be 0)
  int64_t not_two_sparse;  // reduced columns with a weight other than 2 (must be 0)
  double s_dist, s_sort, s_rank, s_reduce, s_emit;
} ph0o_stats;

// Steps 1-3 only.  Writes the sorted edge list and the grade of each edge;
// any output pointer may be NULL.  Returns 0, or -1 on bad arguments.
int ph0o_sorted_edges(const void* points, int elem_bytes, int64_t n, int32_t d,
                      int64_t* colex_delta, int64_t* delta, int32_t* j, int32_t* i,
                      uint32_t* grade, int64_t* distinct) {
  if (!points || (elem_bytes != 1 && elem_bytes != 2) || n < 1 || d < 1) return -1;
  std::vector<Edge> edges = all_pairs(points, elem_bytes, n, d);
  if (colex_delta)
    for (size_t p = 0; p < edges.size(); ++p) colex_delta[p] = edges[p].delta;
  std::sort(edges.begin(), edges.end(), edge_less);
  int64_t nd = 0;
  std::vector<uint32_t> g = grades(edges, &nd);
  for (size_t p = 0; p < edges.size(); ++p) {
    if (delta) delta[p] = edges[p].delta;
    if (j) j[p] = edges[p].j;
    if (i) i[p] = edges[p].i;
    if (grade) grade[p] = g[p];
  }
  if (distinct) *distinct = nd;
  return 0;
}

// The whole algorithm.  Outputs (NULL allowed except where noted):
//   death_by_vertex[n]  grade b of the pivot in row r, PH0O_INF if row r never
//                       became a pivot
//   canonical[n]        the barcode's deaths sorted ascending, PH0O_INF last
//   killer_pos[n]       sorted position of the column whose pivot is row r, -1
//   partner[n]          the other nonzero row of the reduced column stored for
//                       row r (the stored columns have weight 2), -1 if none
// early_exit != 0 stops after N-1 pivots; otherwise every column is reduced
// and stats->late_nonzero counts nonzero columns found after the last pivot.
int ph0o_barcode(const void* points, int elem_bytes, int64_t n, int32_t d, int early_exit,
                 uint32_t* death_by_vertex, uint32_t* canonical, int64_t* killer_pos,
                 int32_t* partner, ph0o_stats* st) {
  if (!points || (elem_bytes != 1 && elem_bytes != 2) || n < 1 || d < 1) return -1;
  ph0o_stats s;
  std::memset(&s, 0, sizeof(s));
  s.E = n * (n - 1) / 2;

  auto t0 = std::chrono::steady_clock::now();
  std::vector<Edge> edges = all_pairs(points, elem_bytes, n, d);  // step 1
  s.s_dist = seconds_since(t0);

  t0 = std::chrono::steady_clock::now();
  std::sort(edges.begin(), edges.end(), edge_less);  // step 2
  s.s_sort = seconds_since(t0);

  t0 = std::chrono::steady_clock::now();
  std::vector<uint32_t> g = grades(edges, &s.distinct);  // step 3
  s.s_rank = seconds_since(t0);

  // Steps 4-5: dense F2 columns, reduced left to right.
  t0 = std::chrono::steady_clock::now();
  const int64_t words = (n + 63) / 64;
  std::vector<std::vector<uint64_t>> slot(static_cast<size_t>(n));  // empty = no pivot
  std::vector<uint32_t> death(static_cast<size_t>(n), PH0O_INF);
  std::vector<int64_t> killer(static_cast<size_t>(n), -1);
  std::vector<uint64_t> col(static_cast<size_t>(words));
  for (size_t p = 0; p < edges.size(); ++p) {
    if (early_exit && s.pivots == n - 1) break;
    ++s.columns;
    std::fill(col.begin(), col.end(), 0);
    col[edges[p].i / 64] ^= 1ull << (edges[p].i % 64);  // step 4: column p of M
    col[edges[p].j / 64] ^= 1ull << (edges[p].j % 64);
    int64_t low = low_of(col);
    while (low >= 0 && !slot[low].empty()) {
      for (int64_t w = 0; w < words; ++w) col[w] ^= slot[low][w];
      ++s.additions;
      low = low_of(col);
    }
    if (low >= 0) {
      if (s.pivots == n - 1) {  // only reachable in literal mode
        ++s.late_nonzero;
        continue;
      }
      slot[low] = col;
      death[low] = g[p];
      killer[low] = static_cast<int64_t>(p);
      ++s.pivots;
      s.E_eff = static_cast<int64_t>(p) + 1;
    }
  }
  s.s_reduce = seconds_since(t0);

  // Step 6: one interval (0, b) per pivot, plus the essential class.
  t0 = std::chrono::steady_clock::now();
  std::vector<uint32_t> bars(death);
  std::sort(bars.begin(), bars.end());
  for (int64_t r = 0; r < n; ++r) {
    int32_t other = -1;
    if (!slot[r].empty()) {
      int weight = 0;
      for (int64_t w = 0; w < words; ++w) weight += __builtin_popcountll(slot[r][w]);
      if (weight != 2) ++s.not_two_sparse;
      for (int64_t v = 0; v < r; ++v)
        if ((slot[r][v / 64] >> (v % 64)) & 1ull) other = static_cast<int32_t>(v);
    }
    if (death_by_vertex) death_by_vertex[r] = death[r];
    if (canonical) canonical[r] = bars[r];
    if (killer_pos) killer_pos[r] = killer[r];
    if (partner) partner[r] = other;
  }
  s.s_emit = seconds_since(t0);
  if (st) *st = s;
  return 0;
}

// ---- H1: the edge-by-triangle boundary matrix ----
//
// The 1st persistent homology of the same filtration, the higher-dimension
// repetition Section 3 anticipates and the conclusion leaves to future work.
// Readings (the paper gives no H1 details):
//   * the 2-skeleton of the Vietoris-Rips complex: a triangle {a, b, c}
//     enters with its latest edge, the one of its three edges that comes last
//     in the H0 edge order (delta, j, i); its grade is that edge's grade;
//   * triangles are ordered by (position of the latest edge, third vertex),
//     which lists every face before its cofaces;
//   * the boundary matrix has one row per edge (in edge order) and one
//     column per triangle (in triangle order), the triangle's three edges;
//     columns are reduced left to right over F2, low = largest edge position;
//   * a reduced column with low e pairs edge e with the triangle: the H1
//     interval [grade(e), grade(triangle)); intervals of length 0 are not
//     bars.  The complete 2-skeleton has no H1, so exactly E - N + 1 pairs
//     exist and no interval is infinite; early_exit stops at the last one.
// Columns are dense bitsets of E bits.  Outputs (NULL allowed):
//   tri_of_edge[E]   for the edge at sorted position q, the index (in
//                    triangle order) of the triangle it pairs with, -1 if none
//   birth[cap], death[cap]  the bars (birth < death), sorted by (birth, death);
//                    *nbars receives their number (at most E - N + 1)
// Returns 0, -1 on bad arguments, -2 when cap is too small.
typedef struct {
  int64_t E, T, T_eff, additions, pivots, zero_length, columns;
} ph0o_h1_stats;

int ph0o_h1(const void* points, int elem_bytes, int64_t n, int32_t d, int early_exit,
            int64_t* tri_of_edge, uint32_t* birth, uint32_t* death, int64_t cap,
            int64_t* nbars, ph0o_h1_stats* st) {
  if (!points || (elem_bytes != 1 && elem_bytes != 2) || n < 1 || d < 1 || cap < 0) return -1;
  ph0o_h1_stats s;
  std::memset(&s, 0, sizeof(s));
  std::vector<Edge> edges = all_pairs(points, elem_bytes, n, d);
  std::sort(edges.begin(), edges.end(), edge_less);
  int64_t distinct = 0;
  std::vector<uint32_t> g = grades(edges, &distinct);
  const int64_t E = static_cast<int64_t>(edges.size());
  s.E = E;
  // Sorted position of edge {i, j}, i < j.
  std::vector<int64_t> pos(static_cast<size_t>(n * n), -1);
  for (int64_t q = 0; q < E; ++q) {
    pos[static_cast<size_t>(edges[q].i * n + edges[q].j)] = q;
    pos[static_cast<size_t>(edges[q].j * n + edges[q].i)] = q;
  }
  // Triangles with their three edge positions, in (latest edge, third vertex) order.
  struct Tri {
    int64_t e0, e1, e2;  // e2 = latest edge; e0 < e1 < e2
    int32_t k;           // vertex not on the latest edge
  };
  std::vector<Tri> tris;
  tris.reserve(static_cast<size_t>(n * (n - 1) * (n - 2) / 6));
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a + 1; b < n; ++b)
      for (int64_t c = b + 1; c < n; ++c) {
        int64_t e[3] = {pos[a * n + b], pos[a * n + c], pos[b * n + c]};
        std::sort(e, e + 3);
        const int64_t third = e[2] == pos[a * n + b] ? c : e[2] == pos[a * n + c] ? b : a;
        tris.push_back(Tri{e[0], e[1], e[2], static_cast<int32_t>(third)});
      }
  std::sort(tris.begin(), tris.end(), [](const Tri& x, const Tri& y) {
#ifdef PH0O_PLANT_H1_ORDER  // planted mistake for the pin tests only: ties by third
    return x.e2 != y.e2 ? x.e2 < y.e2 : x.k > y.k;  // vertex descending
#else
    return x.e2 != y.e2 ? x.e2 < y.e2 : x.k < y.k;
#endif
  });
  s.T = static_cast<int64_t>(tris.size());

  const int64_t words = (E + 63) / 64;
  std::vector<std::vector<uint64_t>> slot(static_cast<size_t>(E));
  std::vector<int64_t> paired(static_cast<size_t>(E), -1);
  std::vector<uint64_t> col(static_cast<size_t>(words));
  const int64_t want = E - (n - 1);
  for (int64_t t = 0; t < s.T; ++t) {
    if (early_exit && s.pivots == want) break;
    ++s.columns;
    std::fill(col.begin(), col.end(), 0);
    for (int64_t e : {tris[t].e0, tris[t].e1, tris[t].e2}) col[e / 64] ^= 1ull << (e % 64);
    int64_t low = low_of(col);
    while (low >= 0 && !slot[low].empty()) {
      for (int64_t w = 0; w < words; ++w) col[w] ^= slot[low][w];
      low = low_of(col);
#ifdef PH0O_PLANT_H1_COUNT  // planted mistake for the pin tests only: the addition
      if (low >= 0)          // that clears a column goes uncounted
#endif
      ++s.additions;
    }
    if (low >= 0) {
      slot[low] = col;
      paired[low] = t;
      ++s.pivots;
      s.T_eff = t + 1;
    }
  }
  std::vector<std::pair<uint32_t, uint32_t>> bars;
  for (int64_t q = 0; q < E; ++q) {
    if (tri_of_edge) tri_of_edge[q] = paired[q];
    if (paired[q] < 0) continue;
    const uint32_t b = g[q], dd = g[tris[paired[q]].e2];
    if (b == dd)
      ++s.zero_length;
    else
      bars.push_back({b, dd});
  }
  std::sort(bars.begin(), bars.end());
  if (nbars) *nbars = static_cast<int64_t>(bars.size());
  if (st) *st = s;
  if (static_cast<int64_t>(bars.size()) > cap && (birth || death)) return -2;
  for (size_t k = 0; k < bars.size(); ++k) {
    if (birth) birth[k] = bars[k].first;
    if (death) death[k] = bars[k].second;
  }
  return 0;
}

}  // extern "C"
