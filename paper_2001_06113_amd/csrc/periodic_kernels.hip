// HIP kernels of the periodic marching scheme (FP64), gfx950.
//
// One implicit step (Section 2.2, eq. (uadamsk)) on an M1 x M2 grid is two
// passes over HBM, each an LDS-staged line FFT with the pointwise work of the
// step fused in:
//
//  column pass (axis 0, lines are columns, LPW columns per workgroup):
//     load the column tile (row segments of LPW*16 bytes, coalesced)
//     inverse FFT along axis 0                      -> w = F^-1 B on the grid
//     u = w / (1 + i mu_0 dt V(x,t_n))                 (diagonal solve, Remark 2.1)
//     g = V(x,t_n) u / (M1 M2)
//     forward FFT along axis 0, store the tile
//     (and the per-axis phase factors of the next row pass)
//  row pass (axis 1, contiguous rows):
//     forward FFT along axis 1                      -> What_n = F(V u_n)
//     uhat_n = B_n - i mu_0 dt What_n, What_n into the history ring,
//     B_{n+1} = E^(1) uhat_n - i dt sum_{j>=1} mu_j E^(j) What_{n+1-j}
//     inverse FFT along axis 1, store
//
// with E^(j)(k1,k2) = T1_j[k1] T2_j[k2] and
// T_a,j[k] = exp(-i k^2 j dt + i k (phi_a(t_{n+1}) - phi_a(t_{n+1-j}))), the
// factorised phase of Lemma 1.  A 1D problem is the case M1 = 1.
#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

// FFT index -> integer mode in [-M/2, M/2) (M even; M = 1 is the single mode 0)
__device__ __forceinline__ int signed_mode(int idx, int M) { return idx < ((M + 1) >> 1) ? idx : idx - M; }

__device__ __forceinline__ double potential(const LineArgs& a, int64_t g) {
  double v = 0.0;
  for (int r = 0; r < a.nV; ++r) v += a.fV[r] * a.V[r * a.vstride + g];
  return v;
}

// (-i c) * z
__device__ __forceinline__ double2 mul_mi(double c, double2 z) { return double2{c * z.y, -c * z.x}; }

// Per-axis phase table of the next row pass (spread over all workgroups).
__device__ __forceinline__ void build_phase_table(const LineArgs& a, int nthreads) {
  const int per = a.M1 + a.M2;
  const int total = a.req.nj * per;
  for (int idx = blockIdx.x * nthreads + threadIdx.x; idx < total; idx += gridDim.x * nthreads) {
    const int j = idx / per;
    const int kk = idx - j * per;
    double k, dphi;
    if (kk < a.M1) {
      k = (double)signed_mode(kk, a.M1);
      dphi = a.req.dphi1[j];
    } else {
      k = (double)signed_mode(kk - a.M1, a.M2);
      dphi = a.req.dphi2[j];
    }
    const double th = -(k * k) * a.req.tau[j] + k * dphi;
    double s, c;
    sincos(th, &s, &c);
    a.ph[idx] = double2{c, s};
  }
}

// ------------------------------------------------------------- column pass

template <int N, int LPW, int NT>
__global__ __launch_bounds__(NT) void k_col(LineArgs a) {
  static_assert(NT % LPW == 0, "threads must split evenly over lines");
  constexpr int TL = NT / LPW;
  __shared__ double2 lds[LPW * N];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * LPW;
  const int nl = min(LPW, a.nlines - l0);
  const int mode = a.mode;

  if (a.req.nj > 0) build_phase_table(a, NT);

  // load: consecutive threads take consecutive columns of one row
  for (int f = tid; f < LPW * N; f += NT) {
    const int i = f % LPW, e = f / LPW;
    if (i < nl) {
      const int64_t g = (int64_t)(l0 + i) * a.line_stride + (int64_t)e * a.elem_stride;
      double2 v = a.src[g];
      if (mode == C_FWD) {
        const double Vs = potential(a, g);
        const double cr = a.alpha_re + a.beta_re * Vs, ci = a.alpha_im + a.beta_im * Vs;
        v = double2{(cr * v.x - ci * v.y) * a.scale, (cr * v.y + ci * v.x) * a.scale};
      }
      lds[i * N + e] = v;
    }
  }
  __syncthreads();
  const int li = tid / TL, lt = tid % TL;
  double2* line = &lds[li * N];
  if (mode == C_SOLVE) {
    fft_line<N, true, TL>(line, lt, a.tw);
    for (int f = tid; f < LPW * N; f += NT) {
      const int i = f % LPW, e = f / LPW;
      if (i < nl) {
        const int64_t g = (int64_t)(l0 + i) * a.line_stride + (int64_t)e * a.elem_stride;
        const double2 w = lds[i * N + e];
        const double Vs = potential(a, g);
        const double q = a.csolve * Vs;
        const double inv = 1.0 / (1.0 + q * q);
        // u = w (1 - i q) / (1 + q^2)
        const double2 u = double2{(w.x + q * w.y) * inv, (w.y - q * w.x) * inv};
        if (a.uout) a.uout[g] = u;
        if (a.uacc) {
          double2 acc = a.acc_first ? double2{0.0, 0.0} : a.uacc[g];
          acc.x += a.wacc * u.x;
          acc.y += a.wacc * u.y;
          a.uacc[g] = acc;
        }
        const double s = Vs * a.scale;
        lds[i * N + e] = double2{s * u.x, s * u.y};
      }
    }
    __syncthreads();
  }
  fft_line<N, false, TL>(line, lt, a.tw);
  for (int f = tid; f < LPW * N; f += NT) {
    const int i = f % LPW, e = f / LPW;
    if (i < nl) {
      const int64_t g = (int64_t)(l0 + i) * a.line_stride + (int64_t)e * a.elem_stride;
      a.dst[g] = lds[i * N + e];
    }
  }
}

// ---------------------------------------------------------------- row pass

template <int N, int LPW, int NT>
__global__ __launch_bounds__(NT) void k_row(LineArgs a) {
  static_assert(NT % LPW == 0, "threads must split evenly over lines");
  constexpr int TL = NT / LPW;
  __shared__ double2 lds[LPW * N];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * LPW;
  const int nl = min(LPW, a.nlines - l0);
  const int mode = a.mode;
  const int per = a.M1 + a.M2;

  for (int f = tid; f < LPW * N; f += NT) {
    const int e = f % N, i = f / N;
    if (i < nl) {
      const int64_t g = (int64_t)(l0 + i) * a.line_stride + (int64_t)e * a.elem_stride;
      lds[i * N + e] = a.src[g];
    }
  }
  __syncthreads();
  const int li = tid / TL, lt = tid % TL;
  double2* line = &lds[li * N];
  fft_line<N, false, TL>(line, lt, a.tw);

  for (int f = tid; f < LPW * N; f += NT) {
    const int e = f % N, i = f / N;
    if (i < nl) {
      const int k1 = l0 + i;
      const int64_t g = (int64_t)k1 * a.line_stride + (int64_t)e * a.elem_stride;
      const double2 W = lds[i * N + e];
      if (mode == R_FWD) {
        a.fdst[g] = W;
        continue;
      }
      const double2 E1 = cmul(a.ph[k1], a.ph[a.M1 + e]);
      double2 acc;
      if (mode == R_INIT) {
        acc = cmul(E1, W);
      } else if (mode == R_FORM) {
        acc = cmul(E1, W);
        for (int j = 1; j <= a.nh; ++j) {
          const double2 Ej = cmul(a.ph[(j - 1) * per + k1], a.ph[(j - 1) * per + a.M1 + e]);
          const double2 Wj = a.ring[a.slot_r[j] * a.ring_stride + g];
          acc = cadd(acc, cmul(Ej, mul_mi(a.ch[j], Wj)));
        }
      } else {  // R_AM
        const double2 B = a.Bm[g];
        const double2 uh = cadd(B, mul_mi(a.c0, W));
        if (a.slot_w >= 0) a.ring[a.slot_w * a.ring_stride + g] = W;
        acc = cmul(E1, cadd(uh, mul_mi(a.ch[1], W)));
        for (int j = 2; j <= a.nh; ++j) {
          const double2 Ej = cmul(a.ph[(j - 1) * per + k1], a.ph[(j - 1) * per + a.M1 + e]);
          const double2 Wj = a.ring[a.slot_r[j] * a.ring_stride + g];
          acc = cadd(acc, cmul(Ej, mul_mi(a.ch[j], Wj)));
        }
      }
      a.Bm[g] = acc;
      lds[i * N + e] = acc;
    }
  }
  __syncthreads();
  if (mode == R_FWD) return;
  fft_line<N, true, TL>(line, lt, a.tw);
  for (int f = tid; f < LPW * N; f += NT) {
    const int e = f % N, i = f / N;
    if (i < nl) {
      const int64_t g = (int64_t)(l0 + i) * a.line_stride + (int64_t)e * a.elem_stride;
      a.dst[g] = lds[i * N + e];
    }
  }
}

// ---------------------------------------------------------------- dispatch

// Column tiles hold LPW whole columns (at most 64 KiB of LDS); a row segment
// of LPW*16 bytes is one coalesced access.
constexpr int col_lpw(int N) { return N == 1 ? 256 : (N <= 512 ? 8 : (N <= 1024 ? 4 : (N <= 2048 ? 2 : 1))); }
constexpr int col_nt(int N) { return 256; }
// Row tiles: at least 512 elements per workgroup, about 8 elements per thread.
constexpr int pow2_floor(int x) { return x >= 64 ? 64 : x >= 32 ? 32 : x >= 16 ? 16 : x >= 8 ? 8 : x >= 4 ? 4 : x >= 2 ? 2 : 1; }
constexpr int row_lpw(int N) { return N >= 512 ? 1 : pow2_floor(512 / N); }
constexpr int row_nt(int N) {
  return ((N * row_lpw(N) / 8 + 63) / 64) * 64 < 64 ? 64 : ((N * row_lpw(N) / 8 + 63) / 64) * 64;
}

int col_lines_per_block(int N) { return col_lpw(N); }
int row_lines_per_block(int N) { return row_lpw(N); }

#define TDSE_LINE_SIZES(X) \
  X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) \
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

hipError_t launch_col_pass(int N, const LineArgs& a, hipStream_t s) {
  switch (N) {
    case 1: {
      constexpr int L = col_lpw(1), T = col_nt(1);
      hipLaunchKernelGGL((k_col<1, L, T>), dim3((a.nlines + L - 1) / L), dim3(T), 0, s, a);
      break;
    }
#define X(n)                                                                               \
  case n: {                                                                                \
    constexpr int L = col_lpw(n), T = col_nt(n);                                           \
    hipLaunchKernelGGL((k_col<n, L, T>), dim3((a.nlines + L - 1) / L), dim3(T), 0, s, a); \
    break;                                                                                 \
  }
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_pass(int N, const LineArgs& a, hipStream_t s) {
  switch (N) {
#define X(n)                                                                               \
  case n: {                                                                                \
    constexpr int L = row_lpw(n), T = row_nt(n);                                           \
    hipLaunchKernelGGL((k_row<n, L, T>), dim3((a.nlines + L - 1) / L), dim3(T), 0, s, a); \
    break;                                                                                 \
  }
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tdse
