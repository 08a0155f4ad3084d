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
//     the pre-multipliers and the dense matrix (stored [N_D][M]).
// alpha = H + kappa h, h = pi M / nu.  The nu-point FFTs are the
// register-resident Stockham transforms of fft_lds.h, one line per workgroup,
// and the ray modes stay in the registers the FFT leaves them in.
//
// Row pass (axis 1, one mode row k1 per workgroup): forward transform of the
// column-pass output, the implicit Adams recurrence on the row's N2 modes,
// inverse transform into the tile buffer.  Column pass (axis 0, one physical
// column per workgroup): inverse transform, diagonal solve, forward transform.
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

// Line transforms with the ray modes in registers.  Thread t holds, for
// e = t + TL m (m < EPT = 8): v3[m] = mode N - N_E + e (E3 ray) and
// v1[m] = mode N_E - 1 - e (E1 ray), zero for e >= N_E, which is the layout
// the nu-point FFT leaves them in; the N_D dense modes N_E + q live in LDS
// (dm).  The dense block's forward sums are split over (mode, chunk) pairs
// and reduced through LDS (part, N_D * max(1, TL / N_D) entries).

// forward transform of f[0..M) (LDS); ends with dm complete (a barrier)
template <int NU>
__device__ __forceinline__ void cf_forward(const double2* f, double2 (&v3)[8], double2 (&v1)[8], double2* dm,
                                           double2* part, double2* fline, const CFAxis& ax, int t) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND;
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v3[m] = e < M ? cmul(ax.pre3[e], f[e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, false>(v3, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v3[m] = e < NE ? cmul(ax.post3[e], v3[m]) : double2{0.0, 0.0};
  }
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v1[m] = e < M ? cmul(ax.pre1[e], f[e]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, true>(v1, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v1[m] = e < NE ? cmul(ax.post1[e], v1[m]) : double2{0.0, 0.0};
  }
  // dense modes: thread (q, c) sums j = c, c + C, ... (lanes of one q read consecutive j)
  const int C = TL / ND > 1 ? TL / ND : 1;
  for (int i = t; i < ND * C; i += TL) {   // more dense modes than threads: several pairs per thread
    const int q = i / C, c = i - q * C;
    const double2* row = ax.Dfwd + (int64_t)q * M;
    double2 acc = {0.0, 0.0};
    for (int j = c; j < M; j += C) acc = cadd(acc, cmul(row[j], f[j]));
    part[i] = acc;
  }
  __syncthreads();
  for (int q = t; q < ND; q += TL) {
    double2 acc = {0.0, 0.0};
    for (int c = 0; c < C; ++c) acc = cadd(acc, part[q * C + c]);
    dm[q] = acc;
  }
  __syncthreads();
}

// inverse transform of the modes (v3, v1 registers, dm LDS) into
// out[m] = u(t + TL m) for t + TL m < M; v3 and v1 are overwritten
template <int NU>
__device__ __forceinline__ void cf_inverse(double2 (&v3)[8], double2 (&v1)[8], const double2* dm, double2* fline,
                                           const CFAxis& ax, int t, double2 (&out)[8]) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND;
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    v3[m] = e < NE ? cmul(ax.ipre3[e], v3[m]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, true>(v3, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    out[m] = e < M ? cmul(ax.ipost3[e], v3[m]) : double2{0.0, 0.0};
    v1[m] = e < NE ? cmul(ax.ipre1[e], v1[m]) : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, false>(v1, t, fline, ax.tw);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M) {
      double2 s = cadd(out[m], cmul(ax.ipost1[e], v1[m]));
      for (int q = 0; q < ND; ++q) s = cadd(s, cmul(ax.Dinv[(int64_t)q * M + e], dm[q]));
      out[m] = s;
    }
  }
}

// dynamic LDS of a line kernel: f[M] | FFT exchange line | dm[ND] | part[ND * C]
__host__ __device__ constexpr int fs_part_len(int TL, int ND) { return ND * (TL / ND > 1 ? TL / ND : 1); }
template <int NU>
size_t fs_lds_bytes(int M, int ND) {
  return sizeof(double2) * (size_t)(M + lds_line_len(NU) + ND + fs_part_len(NU / 8, ND));
}

// The per-mode step of the row pass for mode g = row_m + k; W is the mode of
// the forward transform (R_AM, R_UHACC).  Returns the new B (R_UHACC: unused).
__device__ __forceinline__ double2 fs_mode_update(const FSArgs& a, int k1, int per, int k, int64_t g, double2 W) {
  const int mode = a.mode;
  const double2* ph = a.ph;
  const int N1 = a.N1;
  // E^(j) = T1_j[k1] T2_j[k]; the first factor is uniform over the workgroup
  auto E = [ph, per, N1, k1, k](int j) { return cmul(ph[(j - 1) * per + k1], ph[(j - 1) * per + N1 + k]); };
  double2 acc;
  if (mode == R_AM) {
    const double2 uh = cadd(a.Bm[g], fs_mul_mi(a.c0, W));
    acc = cmul(E(1), cadd(uh, fs_mul_mi(a.ch[1], W)));
    for (int j = 2; j <= a.nh; ++j) acc = cadd(acc, cmul(E(j), fs_mul_mi(a.ch[j], a.ring[a.slot_r[j] * a.ring_stride + g])));
    if (a.slot_w >= 0) a.ring[a.slot_w * a.ring_stride + g] = W;
    a.Bm[g] = acc;
  } else if (mode == R_BINIT) {
    const double2 Wr = a.ring[a.slot_r[1] * a.ring_stride + g];
    acc = cmul(E(1), cadd(a.UH[g], fs_mul_mi(a.c0, Wr)));
    a.Bm[g] = acc;
  } else if (mode == R_UHACC) {
    const double2 uh = cadd(a.Bm[g], fs_mul_mi(a.c0, W));
    double2 s = a.acc_first ? double2{0.0, 0.0} : a.UHacc[g];
    s.x += a.wacc * uh.x;
    s.y += a.wacc * uh.y;
    a.UHacc[g] = s;
    acc = s;
  } else {  // R_FORM
    acc = cmul(E(1), a.UH[g]);
    for (int j = 1; j <= a.nh; ++j) acc = cadd(acc, cmul(E(j), fs_mul_mi(a.ch[j], a.ring[a.slot_r[j] * a.ring_stride + g])));
    a.Bm[g] = acc;
  }
  return acc;
}

// ---------------------------------------------------------------- row pass

// Three workgroups per CU (a register budget of 168; the few values that
// spill cost less than the latency a third wave per SIMD hides in the
// per-mode updates).
template <int NU>
__global__ __launch_bounds__(NU / 8) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_fs_row(FSArgs a) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  const CFAxis& ax = a.ax2;
  const int M2 = ax.M, N2 = ax.N, NE = ax.NE, ND = ax.ND;
  double2* fin = fs_lds;
  double2* fline = fin + M2;
  double2* dm = fline + lds_line_len(NU);
  double2* part = dm + ND;
  const int t = threadIdx.x;
  const int k1 = blockIdx.x;
  const int mode = a.mode;
  const int per = a.N1 + a.N2;
  const int64_t row_m = (int64_t)k1 * N2;   // mode row
  const int64_t row_p = (int64_t)k1 * M2;   // tile row (physical axis 1)

  double2 v3[EPT], v1[EPT];
  const bool need_fwd = (mode == R_AM || mode == R_FWD || mode == R_UHACC);
  if (need_fwd) {
    for (int j = t; j < M2; j += TL) fin[j] = a.src[row_p + j];
    __syncthreads();
    cf_forward<NU>(fin, v3, v1, dm, part, fline, ax, t);
  } else {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v3[m] = v1[m] = double2{0.0, 0.0};
  }
  if (mode == R_FWD) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < NE) {
        a.fdst[row_m + N2 - NE + e] = v3[m];
        a.fdst[row_m + NE - 1 - e] = v1[m];
      }
    }
    for (int q = t; q < ND; q += TL) a.fdst[row_m + NE + q] = dm[q];
    return;
  }
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < NE) {
      v3[m] = fs_mode_update(a, k1, per, N2 - NE + e, row_m + N2 - NE + e, v3[m]);
      v1[m] = fs_mode_update(a, k1, per, NE - 1 - e, row_m + NE - 1 - e, v1[m]);
    }
  }
  for (int q = t; q < ND; q += TL)
    dm[q] = fs_mode_update(a, k1, per, NE + q, row_m + NE + q, need_fwd ? dm[q] : double2{0.0, 0.0});
  if (mode == R_UHACC) return;
  __syncthreads();
  double2 out[EPT];
  cf_inverse<NU>(v3, v1, dm, fline, ax, t, out);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M2) a.dst[row_p + e] = out[m];
  }
}

// ------------------------------------------------------------- column pass

// Columns sharing a 128-byte line of the tile (8 complex128) are dealt to the
// same XCD (workgroups b, b + 8, ...), so their strided accesses meet in one L2.
__device__ __forceinline__ int fs_col_of(int b, int nb) {
  if (nb % 64) return b;
  const int x = b & 7, s = b >> 3;
  return 8 * ((s / 8) * 8 + x) + (s % 8);
}

template <int NU>
__global__ __launch_bounds__(NU / 8) void k_fs_col(FSArgs a) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  const CFAxis& ax = a.ax1;
  const int M1 = ax.M, N1 = ax.N, NE = ax.NE, ND = ax.ND;
  const int M2 = a.ax2.M;
  double2* fin = fs_lds;
  double2* fline = fin + M1;
  double2* dm = fline + lds_line_len(NU);
  double2* part = dm + ND;
  const int t = threadIdx.x;
  const int y = fs_col_of(blockIdx.x, gridDim.x);   // physical column (axis 1)
  const int mode = a.mode;

  if (a.req.nj > 0) build_phase_table_fs(a, TL);
  double2 v3[EPT], v1[EPT];
  if (mode == C_SOLVE) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      v3[m] = e < NE ? a.src[(int64_t)(N1 - NE + e) * M2 + y] : double2{0.0, 0.0};
      v1[m] = e < NE ? a.src[(int64_t)(NE - 1 - e) * M2 + y] : double2{0.0, 0.0};
    }
    for (int q = t; q < ND; q += TL) dm[q] = a.src[(int64_t)(NE + q) * M2 + y];
    __syncthreads();
    double2 w[EPT];
    cf_inverse<NU>(v3, v1, dm, fline, ax, t, w);
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
  cf_forward<NU>(fin, v3, v1, dm, part, fline, ax, t);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < NE) {
      a.dst[(int64_t)(N1 - NE + e) * M2 + y] = v3[m];
      a.dst[(int64_t)(NE - 1 - e) * M2 + y] = v1[m];
    }
  }
  for (int q = t; q < ND; q += TL) a.dst[(int64_t)(NE + q) * M2 + y] = dm[q];
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
#define TDSE_FS_LAUNCH_SH(K, G, B, SH, S, E0, E1, A)               \
  do {                                                             \
    if (E0) hipExtLaunchKernelGGL(K, G, B, SH, S, E0, E1, 0, A);   \
    else hipLaunchKernelGGL(K, G, B, SH, S, A);                    \
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

size_t fs_line_lds_bytes(int nu, int M, int ND) {
  switch (nu) {
#define X(n) case n: return fs_lds_bytes<n>(M, ND);
    TDSE_FS_NU(X)
#undef X
    default:
      return 0;
  }
}

hipError_t launch_fs_row(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    TDSE_FS_LAUNCH_SH((k_fs_row<n>), dim3(a.N1), dim3(n / 8), fs_lds_bytes<n>(a.ax2.M, a.ax2.ND), s, e0, e1, a); \
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
    TDSE_FS_LAUNCH_SH((k_fs_col<n>), dim3(a.ax2.M), dim3(n / 8), fs_lds_bytes<n>(a.ax1.M, a.ax1.ND), s, e0, e1, a); \
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
