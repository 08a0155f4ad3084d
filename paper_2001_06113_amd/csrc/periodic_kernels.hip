// HIP kernels of the periodic marching scheme, gfx950: the per-instance
// column and row passes (bodies in periodic_body.h), the middle-axis FFT
// passes of 3D grids, their dispatch over line lengths, and the
// complex128 -> complex64 narrowing.
#include <hip/hip_ext.h>

#include "periodic_body.h"

namespace tdse {

// ------------------------------------------------------------- column pass

template <typename C, int N, int LPW, int TL>
__global__ __launch_bounds__(LPW * TL, (sizeof(C) == sizeof(double2) && N >= 256 && N <= 1024 && (N & (N - 1)) == 0) ? 4 : 1) void k_col(LineArgs a) {
  __shared__ C lds[col_lds<C, N, LPW>::elems];
  // tiles sharing a 128-byte line of the potential share an XCD
  const int tile = xcd_tile<(16 / LPW > 1 ? 16 / LPW : 1)>(blockIdx.x, gridDim.x);
  col_body<C, N, LPW, TL>(a, tile * LPW, blockIdx.x, gridDim.x, lds);
}

// FFT-only pass over the middle axis of a 3D grid, in the transform precision
template <typename C, int N, int LPW, int TL, bool INV>
__global__ __launch_bounds__(LPW * TL) void k_mid(LineArgs a) {
  __shared__ C lds[col_lds<C, N, LPW>::elems];
  const int tile = xcd_tile<(16 / LPW > 1 ? 16 / LPW : 1)>(blockIdx.x, gridDim.x);
  mid_body<C, N, LPW, TL, INV>(a, tile * LPW, lds);
}

// ---------------------------------------------------------------- row pass

template <typename C, int N, int LPW, int TL, bool PW = false>
__global__ __launch_bounds__(LPW * TL) void k_row(LineArgs a) {
  __shared__ C lds[row_lds<C, N, LPW>::elems];
  row_body<C, N, LPW, TL, PW>(a, blockIdx.x * LPW, lds);
}

// ---------------------------------------------------------------- dispatch

// Column pass: EPT elements per thread (4 for lengths 256..1024, 8 otherwise,
// 12 with a factor 3, 6 at 384), LPW columns per workgroup (2 from length
// 256: enough workgroups to fill the chip at 512 columns), padded LDS lines.
constexpr int col_ept(int N) {
  return N == 1 ? 1
                : (N % 3 == 0 ? (N < 12 ? N : (N == 384 ? 6 : 12))
                              : (N < 8 ? N : (N >= 256 && N <= 1024 ? 4 : 8)));
}
constexpr int col_tl(int N) { return N / col_ept(N); }
constexpr int col_lpw(int N) {
  return N == 1 ? 256 : (N > 1536 ? 1 : (N >= 256 ? 2 : (64 / col_tl(N) > 2 ? 64 / col_tl(N) : 2)));
}
// Row pass: EPT 4 (12 with a factor 3, 6 at 384 and 768: twice the threads
// for the history loads of an Adams step, 13-17 % faster there than 12
// despite three more radix-2 passes; 8 from 2048). At least 128 threads
// below length 256; from 256 on, one wave is enough, so 256-, 384- and
// 768-point rows take one line per workgroup (a 384-row grid: 384
// workgroups, against 96 of four lines with EPT 12 and 128 threads).
constexpr int row_ept(int N) {
  return N % 3 == 0 ? (N < 12 ? N : (N == 384 || N == 768 ? 6 : 12)) : (N >= 2048 ? 8 : (N < 4 ? N : 4));
}
constexpr int row_tl(int N) { return N / row_ept(N); }
constexpr int row_lpw(int N) {
  return (N >= 256 ? 64 : 128) / row_tl(N) > 1 ? (N >= 256 ? 64 : 128) / row_tl(N) : 1;
}

#define TDSE_LINE_SIZES(X) \
  X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) \
  X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)

bool line_length_supported(int N) {
  switch (N) {
#define X(n) case n:
    TDSE_LINE_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

// With events e0/e1 the launch records them at the kernel's own start and
// end (hipExtLaunchKernelGGL), which times the kernel without launch gaps.
#define TDSE_LAUNCH(K, G, B, S, E0, E1, A)                        \
  do {                                                            \
    if (E0) hipExtLaunchKernelGGL(K, G, B, 0, S, E0, E1, 0, A);   \
    else hipLaunchKernelGGL(K, G, B, 0, S, A);                    \
  } while (0)

// The pointwise pass of a 1D problem (length 1) fills one workgroup with its
// M2 points; it gets extra, inactive workgroups so that the next row pass's
// phase table has one entry per thread.
inline int64_t col_blocks(int N, const LineArgs& a, int L, int T) {
  int64_t nb = (a.nlines + L - 1) / L;
  if (N == 1) {
    const int64_t entries = (int64_t)a.req.nj * (a.M1 + a.M2);
    nb = std::max<int64_t>(nb, std::min<int64_t>((entries + L * T - 1) / (L * T), 1024));
  }
  return nb;
}

template <typename C>
hipError_t col_pass(int N, const LineArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (N) {
#define X(n)                                                                                      \
  case n: {                                                                                       \
    constexpr int L = (sizeof(C) == sizeof(float2) && n == 128) ? 16 : col_lpw(n), T = col_tl(n);                                                \
    TDSE_LAUNCH((k_col<C, n, L, T>), dim3((unsigned)col_blocks(n, a, L, T)), dim3(L * T), s, e0, e1, a); \
    break;                                                                                        \
  }
    X(1)
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// middle-axis pass: the column pass's schedules (the lines are strided the same way)
template <typename C>
hipError_t mid_pass(int N, bool inverse, const LineArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.slab_lines < 1) return hipErrorInvalidValue;
  switch (N) {
#define X(n)                                                                                          \
  case n: {                                                                                           \
    constexpr int L = (sizeof(C) == sizeof(float2) && n == 128) ? 16 : col_lpw(n), T = col_tl(n);                                                    \
    const dim3 g((unsigned)((a.nlines + L - 1) / L));                                                 \
    if (inverse) TDSE_LAUNCH((k_mid<C, n, L, T, true>), g, dim3(L * T), s, e0, e1, a);               \
    else TDSE_LAUNCH((k_mid<C, n, L, T, false>), g, dim3(L * T), s, e0, e1, a);                      \
    break;                                                                                            \
  }
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename C>
hipError_t row_pass(int N, const LineArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (N) {
#define X(n)                                                                                      \
  case n: {                                                                                       \
    constexpr int L = row_lpw(n), T = row_tl(n);                                                  \
    if (a.pf_pow) {                                                                               \
      TDSE_LAUNCH((k_row<C, n, L, T, true>), dim3((a.nlines + L - 1) / L), dim3(L * T), s, e0, e1, a); \
      break;                                                                                      \
    }                                                                                             \
    TDSE_LAUNCH((k_row<C, n, L, T>), dim3((a.nlines + L - 1) / L), dim3(L * T), s, e0, e1, a);   \
    break;                                                                                        \
  }
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_narrow(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = float2{(float)src[i].x, (float)src[i].y};
}

hipError_t launch_narrow(const double2* src, float2* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}


hipError_t launch_col_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return prec == P_SPLIT ? col_pass<float2>(N, a, s, e0, e1) : col_pass<double2>(N, a, s, e0, e1);
}
hipError_t launch_mid_pass(int prec, int N, bool inverse, const LineArgs& a, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  return prec == P_SPLIT ? mid_pass<float2>(N, inverse, a, s, e0, e1) : mid_pass<double2>(N, inverse, a, s, e0, e1);
}
hipError_t launch_row_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return prec == P_SPLIT ? row_pass<float2>(N, a, s, e0, e1) : row_pass<double2>(N, a, s, e0, e1);
}

}  // namespace tdse
