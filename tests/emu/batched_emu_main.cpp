// CPU driver of the batched kernel's emulation (tests/test_batched_emulation.py).
// It includes a copy of csrc/batched.hip in which every LDS array is bounds
// checked (the test rewrites the source), lays out the launch the way
// ph0_barcodes_batched_device does for the clouds the fused kernel takes
// (largest first; n <= 512, n * d <= 8192, d <= 64), gives every
// workgroup's key and grade scratch an ASan-poisoned tail so that any access
// past its emax entries aborts, runs the kernel on two workgroups of host
// threads, and writes the bars and the per-cloud error codes.
#include <sanitizer/asan_interface.h>

#include <algorithm>
#include <utility>

#include BATCHED_SOURCE

using namespace ph0;

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[10];  // nclouds, d, elem_bytes, blocks, chunk_mult[4], digit_bits, threads
  if (fread(hdr, 8, 10, f) != 10) return 2;
  const int64_t nclouds = hdr[0], d = hdr[1], eb = hdr[2], blocks = hdr[3];
  std::vector<int64_t> offsets(nclouds + 1);
  if (fread(offsets.data(), 8, nclouds + 1, f) != (size_t)(nclouds + 1)) return 2;
  const int64_t rows = offsets[nclouds];
  std::vector<char> pts((size_t)(rows * d * eb) + 1);
  if (fread(pts.data(), 1, rows * d * eb, f) != (size_t)(rows * d * eb)) return 2;
  fclose(f);

  // The fused clouds, largest first (stable), and the largest edge count.
  std::vector<std::pair<int64_t, int32_t>> bysize;
  int64_t emax = 1;
  for (int64_t c = 0; c < nclouds; ++c) {
    const int64_t n = offsets[c + 1] - offsets[c];
    if (n > kBatchMaxN || n * d > kBatchMaxPts || d > 64) continue;
    bysize.push_back({n, (int32_t)c});
    emax = std::max(emax, n * (n - 1) / 2);
  }
  std::stable_sort(bysize.begin(), bysize.end(),
                   [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                     return x.first > y.first;
                   });
  std::vector<int32_t> order;
  for (auto& e : bysize) order.push_back(e.second);

  // Scratch regions of emax entries, each followed by a poisoned gap: the
  // kernel is told the region stride (emax + gap) and uses emax entries.
  const int64_t gap = 64;
  const int64_t stride = emax + gap;
  std::vector<uint64_t> scratch((size_t)(2 * stride * blocks));
  std::vector<uint32_t> grades((size_t)(stride * blocks));
  for (int64_t b = 0; b < 2 * blocks; ++b)
    ASAN_POISON_MEMORY_REGION(scratch.data() + b * stride + emax, gap * 8);
  for (int64_t b = 0; b < blocks; ++b)
    ASAN_POISON_MEMORY_REGION(grades.data() + b * stride + emax, gap * 4);
  std::vector<uint32_t> bars((size_t)(2 * rows) + 1, 0xDEADBEEFu);
  std::vector<int32_t> errs((size_t)nclouds, 0);
  uint32_t queue = 0;

  BatchArgs A;
  A.pts = pts.data();
  A.elem_bytes = (int)eb;
  A.d = (int32_t)d;
  A.offsets = offsets.data();
  A.order = order.data();
  A.nclouds = (int64_t)order.size();
  A.bars = bars.data();
  A.scratch = scratch.data();
  A.grades = grades.data();
  A.emax = stride;
  A.queue = &queue;
  A.errs = errs.data();
  for (int b = 0; b < 4; ++b) A.chunk_mult[b] = (int32_t)hdr[4 + b];
  A.digit_bits = (int32_t)hdr[8];
  A.threads = (int32_t)hdr[9];
  if (!order.empty() && launch_batched(A, (int)blocks, nullptr) != hipSuccess) return 3;

  FILE* g = fopen(argv[2], "wb");
  if (!g) return 2;
  fwrite(bars.data(), 4, 2 * rows, g);
  fwrite(errs.data(), 4, nclouds, g);
  fclose(g);
  printf("emulated %zu fused clouds on %lld workgroups\n", order.size(), (long long)blocks);
  return 0;
}
