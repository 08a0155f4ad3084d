// HIP kernels of the free-space complex-frequency scheme (FP64), gfx950.
//
// Per axis the modes sit on the contour Gamma (Section 3.4) in the order
// E1 | A1 C A3 | E3: N_E equispaced nodes on each horizontal ray, 2p + N_C
// Alpert and Gauss nodes in between ("dense" modes).  One line transform
// (Section 4.1):
//   forward  fhat_k = (2/M) sum_j exp(-i zeta_k x_j) f_j
//     E3: pre-multiply f by exp(-2i alpha j/M - H x_j), zero-pad to nu, FFT_nu,
//         keep outputs e < N_E, post-multiply by (2/M) exp(i alpha + i e h);
//     E1: the mirror image through an inverse FFT_nu (mode N_E-1-e);
//     dense modes: direct sums with a precomputed (2p + N_C) x M matrix;
//   inverse  u_j = (1/2pi) sum_k w_k exp(i zeta_k x_j) uhat_k
//     the same three parts in the opposite directions, weights folded into
//     the pre-multipliers and the dense matrix.
// alpha = H + kappa h, h = pi M / nu.  The ν-point FFTs are the
// register-resident Stockham transforms of fft_lds.h, one line per block.
//
// Row pass (axis 1, one mode row k1 per block): forward transform of the
// column-pass output, the implicit Adams recurrence on the row's N2 modes,
// inverse transform into the tile buffer.  Column pass (axis 0, one physical
// column per block): inverse transform, diagonal solve, forward transform.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

__device__ __forceinline__ double2 fs_mul_mi(double c, double2 z) { return double2{c * z.y, -c * z.x}; }

// Per-axis phase factors exp(i(-zeta^2 tau_j + zeta dphi_j)) for complex
// nodes zeta (|.| != 1 off the real axis), table ph[(j-1)(N1+N2) + k].
__device__ __forceinline__ void build_phase_table_fs(const FSArgs& a, int nthreads) {
  const int per = a.N1 + a.N2;
  const int total = a.req.nj * per;
  for (int idx = blockIdx.x * nthreads + threadIdx.x; idx < total; idx += gridDim.x * nthreads) {
    const int j = idx / per;
    const int kk = idx - j * per;
    double2 z;
    double dphi;
    if (kk < a.N1) {
      z = a.ax1.zeta ? a.ax1.zeta[kk] : double2{0.0, 0.0};
      dphi = a.req.dphi1[j];
    } else {
      z = a.ax2.zeta[kk - a.N1];
      dphi = a.req.dphi2[j];
    }
    const double2 z2 = cmul(z, z);
    // theta = -z^2 tau + z dphi (complex); exp(i theta)
    const double tr = -z2.x * a.req.tau[j] + z.x * dphi;
    const double ti = -z2.y * a.req.tau[j] + z.y * dphi;
    const double mag = exp(-ti);
    double s, c;
    sincos(tr, &s, &c);
    a.ph[idx] = double2{mag * c, mag * s};
  }
}

// forward transform of f[0..M) (LDS) into out[0..N) (LDS); every thread calls
template <int NU, int TL>
__device__ void cf_forward(const double2* f, double2* out, double2* fline, const CFAxis& ax, int t) {
  constexpr int EPT = NU / TL;
  const int M = ax.M, N = ax.N, NE = ax.NE, ND = ax.ND;
  double2 v[EPT];
  // E3 branch
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v[m] = e < M ? cmul(ax.pre3[e], f[e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, false>(v, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < NE) out[N - NE + e] = cmul(ax.post3[e], v[m]);
  }
  // E1 branch
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v[m] = e < M ? cmul(ax.pre1[e], f[e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, true>(v, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < NE) out[NE - 1 - e] = cmul(ax.post1[e], v[m]);
  }
  // dense modes
  for (int q = t; q < ND; q += TL) {
    const double2* row = ax.Dfwd + (int64_t)q * M;
    double2 s = {0.0, 0.0};
    for (int j = 0; j < M; ++j) s = cadd(s, cmul(row[j], f[j]));
    out[NE + q] = s;
  }
  __syncthreads();
}

// inverse transform of g[0..N) (LDS) into acc[m] = u(t + TL m), m < EPT
// (only elements < M are meaningful); every thread calls
template <int NU, int TL>
__device__ void cf_inverse(const double2* g, double2* acc, double2* fline, const CFAxis& ax, int t) {
  constexpr int EPT = NU / TL;
  const int M = ax.M, N = ax.N, NE = ax.NE, ND = ax.ND;
  double2 v[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) acc[m] = double2{0.0, 0.0};
  // E3 branch: inverse FFT
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v[m] = e < NE ? cmul(ax.ipre3[e], g[N - NE + e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, true>(v, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M) acc[m] = cadd(acc[m], cmul(ax.ipost3[e], v[m]));
  }
  // E1 branch: forward FFT
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v[m] = e < NE ? cmul(ax.ipre1[e], g[NE - 1 - e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, false>(v, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M) acc[m] = cadd(acc[m], cmul(ax.ipost1[e], v[m]));
  }
  // dense modes
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M) {
      const double2* row = ax.Dinv + (int64_t)e * ND;
      double2 s = acc[m];
      for (int q = 0; q < ND; ++q) s = cadd(s, cmul(row[q], g[NE + q]));
      acc[m] = s;
    }
  }
}

// E^(j) at (k1, k2) from the per-axis phase table
__device__ __forceinline__ double2 fs_phase(const double2* ph, int per, int M1, int j, int k1, int k2) {
  return cmul(ph[(j - 1) * per + k1], ph[(j - 1) * per + M1 + k2]);
}

// ---------------------------------------------------------------- row pass

template <int NU, int MAXN>
__global__ __launch_bounds__(NU / 8) void k_fs_row(FSArgs a) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  __shared__ double2 fin[NU];                  // physical row (M2 <= NU)
  __shared__ double2 modes[MAXN];              // the row's N2 modes
  __shared__ double2 fline[lds_line_len(NU)];  // FFT exchange buffer
  const CFAxis& ax = a.ax2;
  const int t = threadIdx.x;
  const int k1 = blockIdx.x;
  const int mode = a.mode;
  const int M2 = ax.M, N2 = ax.N;
  const int per = a.N1 + a.N2;
  const int64_t row_m = (int64_t)k1 * N2;   // mode row
  const int64_t row_p = (int64_t)k1 * M2;   // tile row (physical axis 1)

  const bool need_fwd = (mode == R_AM || mode == R_FWD || mode == R_UHACC);
  if (need_fwd) {
    for (int j = t; j < M2; j += TL) fin[j] = a.src[row_p + j];
    __syncthreads();
    cf_forward<NU, TL>(fin, modes, fline, ax, t);
  }
  if (mode == R_FWD) {
    for (int k = t; k < N2; k += TL) a.fdst[row_m + k] = modes[k];
    return;
  }
  // per-mode work
  for (int k = t; k < N2; k += TL) {
    const int64_t g = row_m + k;
    double2 acc;
    if (mode == R_AM) {
      const double2 W = modes[k];
      const double2 uh = cadd(a.Bm[g], fs_mul_mi(a.c0, W));
      acc = cmul(fs_phase(a.ph, per, a.N1, 1, k1, k), cadd(uh, fs_mul_mi(a.ch[1], W)));
      for (int j = 2; j <= a.nh; ++j) {
        const double2 Wj = a.ring[a.slot_r[j] * a.ring_stride + g];
        acc = cadd(acc, cmul(fs_phase(a.ph, per, a.N1, j, k1, k), fs_mul_mi(a.ch[j], Wj)));
      }
      if (a.slot_w >= 0) a.ring[a.slot_w * a.ring_stride + g] = W;
      a.Bm[g] = acc;
    } else if (mode == R_BINIT) {
      // B = P (uhat - i c What) with What from the ring
      const double2 W = a.ring[a.slot_r[1] * a.ring_stride + g];
      acc = cmul(fs_phase(a.ph, per, a.N1, 1, k1, k), cadd(a.UH[g], fs_mul_mi(a.c0, W)));
      a.Bm[g] = acc;
    } else if (mode == R_UHACC) {
      // uhat^(l) = B - i c What, accumulated with its Richardson weight
      const double2 uh = cadd(a.Bm[g], fs_mul_mi(a.c0, modes[k]));
      double2 s = a.acc_first ? double2{0.0, 0.0} : a.UHacc[g];
      s.x += a.wacc * uh.x;
      s.y += a.wacc * uh.y;
      a.UHacc[g] = s;
      continue;
    } else {  // R_FORM: B from uhat (stored) and the history
      acc = cmul(fs_phase(a.ph, per, a.N1, 1, k1, k), a.UH[g]);
      for (int j = 1; j <= a.nh; ++j) {
        const double2 Wj = a.ring[a.slot_r[j] * a.ring_stride + g];
        acc = cadd(acc, cmul(fs_phase(a.ph, per, a.N1, j, k1, k), fs_mul_mi(a.ch[j], Wj)));
      }
      a.Bm[g] = acc;
    }
    modes[k] = acc;
  }
  if (mode == R_UHACC) return;
  __syncthreads();
  double2 acc[EPT];
  cf_inverse<NU, TL>(modes, acc, fline, ax, t);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M2) a.dst[row_p + e] = acc[m];
  }
}

// ------------------------------------------------------------- column pass

template <int NU, int MAXN>
__global__ __launch_bounds__(NU / 8) void k_fs_col(FSArgs a) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  __shared__ double2 fin[NU];                  // physical column (M1 <= NU)
  __shared__ double2 modes[MAXN];              // the column's N1 modes
  __shared__ double2 fline[lds_line_len(NU)];
  const CFAxis& ax = a.ax1;
  const int t = threadIdx.x;
  const int y = blockIdx.x;                    // physical column index (axis 1)
  const int mode = a.mode;
  const int M1 = ax.M, N1 = ax.N;
  const int M2 = a.ax2.M;

  if (a.req.nj > 0) build_phase_table_fs(a, TL);
  if (mode == C_SOLVE) {
    for (int k = t; k < N1; k += TL) modes[k] = a.src[(int64_t)k * M2 + y];
    __syncthreads();
    double2 w[EPT];
    cf_inverse<NU, TL>(modes, w, fline, ax, t);
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < M1) {
        const int64_t g = (int64_t)e * M2 + y;
        double Vs = 0.0;
        for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + g];
        const double q = a.csolve * Vs;
        const double inv = 1.0 / (1.0 + q * q);
        const double2 u = double2{(w[m].x + q * w[m].y) * inv, (w[m].y - q * w[m].x) * inv};
        if (a.uout) a.uout[g] = u;
        if (a.uacc) {
          double2 s = a.acc_first ? double2{0.0, 0.0} : a.uacc[g];
          s.x += a.wacc * u.x;
          s.y += a.wacc * u.y;
          a.uacc[g] = s;
        }
        fin[e] = double2{Vs * u.x, Vs * u.y};
      }
    }
  } else {  // C_FWD: (alpha + beta V) u from the physical solution
    for (int e = t; e < M1; e += TL) {
      const int64_t g = (int64_t)e * M2 + y;
      double Vs = 0.0;
      for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + g];
      const double2 u = a.usrc[g];
      const double cr = a.alpha_re + a.beta_re * Vs, ci = a.alpha_im + a.beta_im * Vs;
      fin[e] = double2{cr * u.x - ci * u.y, cr * u.y + ci * u.x};
    }
  }
  __syncthreads();
  cf_forward<NU, TL>(fin, modes, fline, ax, t);
  for (int k = t; k < N1; k += TL) a.dst[(int64_t)k * M2 + y] = modes[k];
}

// --------------------------------------------------- pointwise column pass (1D)

// The 1D problem has no axis-0 transform: the "column pass" is the diagonal
// solve (or the pre-multiply) on the M2 grid points of the single row.
__global__ __launch_bounds__(256) void k_fs_point(FSArgs a) {
  if (a.req.nj > 0) build_phase_table_fs(a, 256);
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int M2 = a.ax2.M;
  if (e >= M2) return;
  double Vs = 0.0;
  for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + e];
  if (a.mode == C_SOLVE) {
    const double2 w = a.src[e];
    const double q = a.csolve * Vs;
    const double inv = 1.0 / (1.0 + q * q);
    const double2 u = double2{(w.x + q * w.y) * inv, (w.y - q * w.x) * inv};
    if (a.uout) a.uout[e] = u;
    if (a.uacc) {
      double2 s = a.acc_first ? double2{0.0, 0.0} : a.uacc[e];
      s.x += a.wacc * u.x;
      s.y += a.wacc * u.y;
      a.uacc[e] = s;
    }
    a.dst[e] = double2{Vs * u.x, Vs * u.y};
  } else {
    const double2 u = a.usrc[e];
    const double cr = a.alpha_re + a.beta_re * Vs, ci = a.alpha_im + a.beta_im * Vs;
    a.dst[e] = double2{cr * u.x - ci * u.y, cr * u.y + ci * u.x};
  }
}

// phase table only (before a row pass that has no transform-carrying column pass)
__global__ __launch_bounds__(256) void k_fs_phase(FSArgs a) { build_phase_table_fs(a, 256); }

// ---------------------------------------------------------------- dispatch

#define TDSE_FS_NU(X) X(256) X(512) X(1024) X(2048)

// non-null events are recorded at the kernel's own start and end
#define TDSE_FS_LAUNCH(K, G, B, S, E0, E1, A)                     \
  do {                                                            \
    if (E0) hipExtLaunchKernelGGL(K, G, B, 0, S, E0, E1, 0, A);   \
    else hipLaunchKernelGGL(K, G, B, 0, S, A);                    \
  } while (0)

bool fs_nu_supported(int nu) {
  switch (nu) {
#define X(n) case n:
    TDSE_FS_NU(X)
#undef X
    return true;
    default:
      return false;
  }
}

int fs_max_modes(int nu) { return nu + 64; }

hipError_t launch_fs_row(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    TDSE_FS_LAUNCH((k_fs_row<n, n + 64>), dim3(a.N1), dim3(n / 8), s, e0, e1, a);         \
    break;
    TDSE_FS_NU(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_col(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nu == 0) {   // 1D: pointwise
    TDSE_FS_LAUNCH(k_fs_point, dim3((a.ax2.M + 255) / 256), dim3(256), s, e0, e1, a);
    return hipGetLastError();
  }
  switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    TDSE_FS_LAUNCH((k_fs_col<n, n + 64>), dim3(a.ax2.M), dim3(n / 8), s, e0, e1, a);      \
    break;
    TDSE_FS_NU(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_phase(const FSArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fs_phase, dim3(8), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tdse
