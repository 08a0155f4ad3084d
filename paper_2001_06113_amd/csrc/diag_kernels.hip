// Diagnostics of a run, gfx950: the failure guard (non-finite entries and
// the squared norm of the carried state) and the relative difference of two
// mode arrays (the drift of a stored history entry against its FP64
// recomputation).  Each is a grid-stride reduction: per-workgroup sums in
// LDS, then one device-scope atomic per workgroup into acc (cleared by a
// kernel of its own first, so the sequence can be captured in a graph).
#include <hip/hip_runtime.h>

#include "tdse_internal.h"

namespace tdse {

namespace {

constexpr int DT = 256;

__device__ __forceinline__ void block_add(double a, double b, unsigned bad, double* acc, unsigned* flag) {
  __shared__ double sa[DT], sb[DT];
  __shared__ unsigned sf[DT];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  sf[threadIdx.x] = bad;
  __syncthreads();
  for (int w = DT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
      sf[threadIdx.x] |= sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(acc, sa[0]);
    atomicAdd(acc + 1, sb[0]);
    if (sf[0]) atomicOr(flag, 1u);
  }
}

}  // namespace

__global__ __launch_bounds__(DT) void k_diag_clear(double* acc, unsigned* flag) {
  if (threadIdx.x == 0) {
    acc[0] = 0.0;
    acc[1] = 0.0;
    *flag = 0u;
  }
}

// acc[0] += sum |x_i|^2 over n doubles; flag |= 1 if any x_i is not finite
__global__ __launch_bounds__(DT) void k_guard(const double* __restrict__ x, int64_t n, double* acc, unsigned* flag) {
  double s = 0.0;
  unsigned bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT) {
    const double v = x[i];
    if (!isfinite(v)) bad = 1;
    else s += v * v;
  }
  block_add(s, 0.0, bad, acc, flag);
}

// acc[0] += sum |a_i - b_i|^2, acc[1] += sum |b_i|^2 over n complex entries;
// a is complex64 (a32) or complex128 (a64), b complex128
__global__ __launch_bounds__(DT) void k_diffnorm(const float2* __restrict__ a32, const double2* __restrict__ a64,
                                                 const double2* __restrict__ b, int64_t n, double* acc,
                                                 unsigned* flag) {
  double s = 0.0, t = 0.0;
  unsigned bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT) {
    const double2 y = b[i];
    const double2 x = a32 ? double2{(double)a32[i].x, (double)a32[i].y} : a64[i];
    const double dx = x.x - y.x, dy = x.y - y.y;
    s += dx * dx + dy * dy;
    t += y.x * y.x + y.y * y.y;
    if (!isfinite(s) || !isfinite(t)) bad = 1;
  }
  block_add(s, t, bad, acc, flag);
}

static int diag_blocks(int64_t n) {
  const int64_t b = (n + DT - 1) / DT;
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

hipError_t launch_guard(const double* x, int64_t n, double* acc, unsigned* flag, bool clear, hipStream_t s) {
  if (clear) hipLaunchKernelGGL(k_diag_clear, dim3(1), dim3(DT), 0, s, acc, flag);
  hipLaunchKernelGGL(k_guard, dim3(diag_blocks(n)), dim3(DT), 0, s, x, n, acc, flag);
  return hipGetLastError();
}

hipError_t launch_diffnorm(const float2* a32, const double2* a64, const double2* b, int64_t n, double* acc,
                           unsigned* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_clear, dim3(1), dim3(DT), 0, s, acc, flag);
  hipLaunchKernelGGL(k_diffnorm, dim3(diag_blocks(n)), dim3(DT), 0, s, a32, a64, b, n, acc, flag);
  return hipGetLastError();
}

}  // namespace tdse
