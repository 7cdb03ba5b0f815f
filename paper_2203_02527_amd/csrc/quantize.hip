// quantize.hip -- real-valued points onto the int16 grid of an interval, for
// the real-valued entry point (the paper's workload, Section 4.1, is points
// drawn uniformly from the unit square; the barcode is defined on exact
// integer distances, so the coordinates are put on a fixed grid first).
#include "ph0_internal.h"

namespace ph0 {

namespace {

// Real coordinates onto the int16 grid: q = rint((x - lo) * scale) in fp64
// (one subtraction, one multiplication, round half to even); a value off
// [0, 32767] (a coordinate outside [lo, hi], or not finite) sets *err and
// stores 0.
__global__ void k_quantize_f32(const float* __restrict__ x, int64_t count, double lo,
                               double scale, int16_t* __restrict__ q, int32_t* err) {
  bool bad = false;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double r = rint(((double)x[k] - lo) * scale);
    const bool ok = r >= 0.0 && r <= 32767.0;  // false for NaN
    q[k] = ok ? (int16_t)r : (int16_t)0;
    bad |= !ok;
  }
  if (bad) atomicOr(err, 1);
}

}  // namespace

hipError_t launch_quantize_f32(const float* x, int64_t count, double lo, double scale, int16_t* q,
                               int32_t* err, hipStream_t s) {
  const hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(err), 0u, 1, s);
  if (e != hipSuccess || count <= 0) return e;
  int64_t g = (count + 256 * 8 - 1) / (256 * 8);
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_quantize_f32, dim3((unsigned)g), dim3(256), 0, s, x, count, lo, scale, q,
                     err);
  return hipGetLastError();
}

}  // namespace ph0
