// HIP kernels of the periodic marching scheme (FP64), gfx950.
//
// One implicit step (Section 2.2, eq. (uadamsk)) on an M1 x M2 grid is two
// passes over HBM, each a register-resident line FFT (fft_lds.h) with the
// pointwise work of the step fused in:
//
//  column pass (axis 0; LPW columns per workgroup, lanes run across columns
//  so each row segment is one coalesced access):
//     inverse FFT along axis 0                      -> w = F^-1 B on the grid
//     u = w / (1 + i mu_0 dt V(x,t_n))                 (diagonal solve, Section 2.1 remark)
//     g = V(x,t_n) u / (M1 M2)
//     forward FFT along axis 0
//     (the block also writes the per-axis phase factors of the next row pass)
//  row pass (axis 1, contiguous rows):
//     forward FFT along axis 1                      -> What_n = F(V u_n)
//     uhat_n = B_n - i mu_0 dt What_n, What_n into the history ring,
//     B_{n+1} = E^(1) uhat_n - i dt sum_{j>=1} mu_j E^(j) What_{n+1-j}
//     inverse FFT along axis 1
//
// with E^(j)(k1,k2) = T1_j[k1] T2_j[k2] and
// T_a,j[k] = exp(-i k^2 j dt + i k (phi_a(t_{n+1}) - phi_a(t_{n+1-j}))), the
// factorised phase of Lemma 1.  A 1D problem is the case M1 = 1.
//
// Every global load a pass needs (tile, potential, B, history, phase factors)
// is issued before its first FFT so their latencies overlap.
#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

// FFT index -> integer mode in [-M/2, M/2) (M even; M = 1 is the single mode 0)
__device__ __forceinline__ int signed_mode(int idx, int M) { return idx < ((M + 1) >> 1) ? idx : idx - M; }

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

// Workgroups are dealt to the eight XCDs round-robin.  Neighbouring column
// tiles share 128-byte lines (of the tile data and of the potential), so the
// G tiles Gq..Gq+G-1 go to workgroups b, b+8, ..., b+8(G-1), which sit on the
// same XCD and L2.
template <int G>
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb % (8 * G)) return b;
  const int x = b & 7, s = b >> 3;
  return G * ((s / G) * 8 + x) + (s % G);
}

// ------------------------------------------------------------- column pass

template <int N, int LPW, int TL>
__global__ __launch_bounds__(LPW * TL) void k_col(LineArgs a) {
  constexpr int NT = LPW * TL;
  constexpr int EPT = N / TL;
  constexpr int PITCH = N > 1 ? lds_line_len(N) + 1 : 1;   // +1 spreads the LPW lines over banks
  constexpr bool TWL = (N > 1 && N <= 1024);
  __shared__ double2 lds[LPW * PITCH];
  __shared__ double2 twl[TWL ? N : 1];
  const int tid = threadIdx.x;
  const int i = tid % LPW, t = tid / LPW;
  // tiles sharing a 128-byte line of the potential (8-byte elements) share an XCD
  const int line = xcd_tile<(16 / LPW > 1 ? 16 / LPW : 1)>(blockIdx.x, gridDim.x) * LPW + i;
  const bool active = line < a.nlines;
  const int mode = a.mode;

  double2 v[EPT];
  double vv[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    v[m] = double2{0.0, 0.0};
    vv[m] = 0.0;
    if (active) {
      const int64_t g = (int64_t)line * a.line_stride + (int64_t)(t + TL * m) * a.elem_stride;
      v[m] = a.src[g];
      double p = 0.0;
      for (int r = 0; r < a.nV; ++r) p += a.fV[r] * a.V[r * a.vstride + g];
      vv[m] = p;
    }
  }
  if constexpr (TWL) {
    for (int q = tid; q < N; q += NT) twl[q] = a.tw[q];
  }
  if (a.req.nj > 0) build_phase_table(a, NT);
  if constexpr (TWL) __syncthreads();
  const double2* tw = TWL ? twl : a.tw;
  double2* myline = &lds[i * PITCH];

  if (mode == C_FWD) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double cr = a.alpha_re + a.beta_re * vv[m], ci = a.alpha_im + a.beta_im * vv[m];
      const double2 u = v[m];
      v[m] = double2{(cr * u.x - ci * u.y) * a.scale, (cr * u.y + ci * u.x) * a.scale};
    }
  } else {  // C_SOLVE
    fft_regs<N, TL, true>(v, t, myline, tw);
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double2 w = v[m];
      const double q = a.csolve * vv[m];
      const double inv = 1.0 / (1.0 + q * q);
      // u = w (1 - i q) / (1 + q^2)
      const double2 u = double2{(w.x + q * w.y) * inv, (w.y - q * w.x) * inv};
      if (active) {
        const int64_t g = (int64_t)line * a.line_stride + (int64_t)(t + TL * m) * a.elem_stride;
        if (a.uout) a.uout[g] = u;
        if (a.uacc) {
          double2 acc = a.acc_first ? double2{0.0, 0.0} : a.uacc[g];
          acc.x += a.wacc * u.x;
          acc.y += a.wacc * u.y;
          a.uacc[g] = acc;
        }
      }
      const double s = vv[m] * a.scale;
      v[m] = double2{s * u.x, s * u.y};
    }
  }
  fft_regs<N, TL, false>(v, t, myline, tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int64_t g = (int64_t)line * a.line_stride + (int64_t)(t + TL * m) * a.elem_stride;
      a.dst[g] = v[m];
    }
  }
}

// ---------------------------------------------------------------- row pass

template <int N, int LPW, int TL>
__global__ __launch_bounds__(LPW * TL) void k_row(LineArgs a) {
  constexpr int NT = LPW * TL;
  constexpr int EPT = N / TL;
  constexpr int NH = MAXH - 1;    // history terms of the order-8 rule (j = 1..7)
  constexpr bool PF = EPT <= 4;   // prefetch history and phases into registers
  constexpr bool TWL = (N <= 1024);
  constexpr int PITCH = lds_line_len(N);
  __shared__ double2 lds[LPW * PITCH];
  __shared__ double2 twl[TWL ? N : 1];
  const int tid = threadIdx.x;
  const int i = tid / TL, t = tid % TL;
  const int k1 = blockIdx.x * LPW + i;
  const bool active = k1 < a.nlines;
  const int mode = a.mode;
  const int per = a.M1 + a.M2;
  const int nh = a.nh;
  const int64_t row0 = (int64_t)k1 * a.line_stride;

  double2 v[EPT];
  double2 Bp[EPT];
  double2 Wr[PF ? NH - 1 : 1][EPT];
  double2 T2[PF ? NH : 1][EPT];
  double2 T1[NH];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    v[m] = double2{0.0, 0.0};
    if (active) v[m] = a.src[row0 + (t + TL * m)];
  }
  if (active && mode == R_AM) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) Bp[m] = a.Bm[row0 + (t + TL * m)];
    if constexpr (PF) {
#pragma unroll
      for (int j = 2; j <= NH; ++j) {
        if (j <= nh) {
#pragma unroll
          for (int m = 0; m < EPT; ++m) Wr[j - 2][m] = a.ring[a.slot_r[j] * a.ring_stride + row0 + (t + TL * m)];
        }
      }
    }
  }
  if (active && mode != R_FWD) {
    const int nj = (mode == R_INIT) ? 1 : nh;
#pragma unroll
    for (int j = 1; j <= NH; ++j) {
      if (j <= nj) {
        T1[j - 1] = a.ph[(j - 1) * per + k1];
        if constexpr (PF) {
#pragma unroll
          for (int m = 0; m < EPT; ++m) T2[j - 1][m] = a.ph[(j - 1) * per + a.M1 + (t + TL * m)];
        }
      }
    }
  }
  // Phase factor E^(j) and history term What_{n+1-j} at element m, from
  // registers (PF) or from memory.  Only plain locals are captured: taking the
  // address of the by-value kernel argument would copy it to scratch.
  const double2* __restrict__ ph = a.ph;
  const double2* __restrict__ ring = a.ring;
  const int64_t rstride = a.ring_stride;
  const int M1 = a.M1;
  int slot_r[MAXH + 1];
#pragma unroll
  for (int j = 0; j <= MAXH; ++j) slot_r[j] = a.slot_r[j];
  auto E = [&T1, &T2, ph, per, M1, t](int j, int m) -> double2 {
    if constexpr (PF) return cmul(T1[j - 1], T2[j - 1][m]);
    else return cmul(T1[j - 1], ph[(j - 1) * per + M1 + (t + TL * m)]);
  };
  auto Wh = [&Wr, &slot_r, ring, rstride, row0, t](int j, int m) -> double2 {
    if constexpr (PF) return Wr[j - 2][m];
    else return ring[slot_r[j] * rstride + row0 + (t + TL * m)];
  };
  if constexpr (TWL) {
    for (int q = tid; q < N; q += NT) twl[q] = a.tw[q];
    __syncthreads();
  }
  const double2* tw = TWL ? twl : a.tw;
  double2* myline = &lds[i * PITCH];

  fft_regs<N, TL, false>(v, t, myline, tw);

  if (mode == R_FWD) {
    if (active) {
#pragma unroll
      for (int m = 0; m < EPT; ++m) a.fdst[row0 + (t + TL * m)] = v[m];
    }
    return;
  }
  // fused recurrence; lanes past the last line (ragged tile) only keep the
  // FFT barriers company and touch no memory
  if (!active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = double2{0.0, 0.0};
  } else if (mode == R_AM) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double2 W = v[m];
      const double2 uh = cadd(Bp[m], mul_mi(a.c0, W));
      double2 acc = cmul(E(1, m), cadd(uh, mul_mi(a.ch[1], W)));
#pragma unroll
      for (int j = 2; j <= NH; ++j) {
        if (j <= nh) acc = cadd(acc, cmul(E(j, m), mul_mi(a.ch[j], Wh(j, m))));
      }
      const int64_t g = row0 + (t + TL * m);
      if (a.slot_w >= 0) a.ring[a.slot_w * a.ring_stride + g] = W;
      a.Bm[g] = acc;
      v[m] = acc;
    }
  } else if (mode == R_INIT) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double2 acc = cmul(E(1, m), v[m]);
      a.Bm[row0 + (t + TL * m)] = acc;
      v[m] = acc;
    }
  } else {  // R_FORM: B from uhat (this FFT) and nh history terms, all from the ring
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      double2 acc = cmul(E(1, m), v[m]);
      const int64_t g = row0 + (t + TL * m);
#pragma unroll
      for (int j = 1; j <= NH; ++j) {  // static j: registers stay registers
        if (j <= nh) {
          const double2 Wj = ring[slot_r[j] * rstride + g];
          acc = cadd(acc, cmul(E(j, m), mul_mi(a.ch[j], Wj)));
        }
      }
      a.Bm[g] = acc;
      v[m] = acc;
    }
  }
  fft_regs<N, TL, true>(v, t, myline, tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) a.dst[row0 + (t + TL * m)] = v[m];
  }
}

// ---------------------------------------------------------------- dispatch

// Column pass: EPT elements per thread (8, or 12 for lengths with a factor
// 3), LPW columns per workgroup (2 from length 256: enough workgroups to fill
// the chip at 512 columns), padded LDS lines.
constexpr int col_ept(int N) { return N == 1 ? 1 : (N % 3 == 0 ? (N < 12 ? N : 12) : (N < 8 ? N : (N >= 256 && N <= 1024 ? 4 : 8))); }
constexpr int col_tl(int N) { return N / col_ept(N); }
constexpr int col_lpw(int N) {
  return N == 1 ? 256 : (N > 1536 ? 1 : (N >= 256 ? 2 : (64 / col_tl(N) > 2 ? 64 / col_tl(N) : 2)));
}
// Row pass: EPT 4 (12 with a factor 3, 8 from 2048), at least 128 threads.
constexpr int row_ept(int N) { return N % 3 == 0 ? (N < 12 ? N : 12) : (N >= 2048 ? 8 : (N < 4 ? N : 4)); }
constexpr int row_tl(int N) { return N / row_ept(N); }
constexpr int row_lpw(int N) { return 128 / row_tl(N) > 1 ? 128 / row_tl(N) : 1; }

int col_lines_per_block(int N) { return col_lpw(N); }
int row_lines_per_block(int N) { return row_lpw(N); }

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

hipError_t launch_col_pass(int N, const LineArgs& a, hipStream_t s) {
  switch (N) {
#define X(n)                                                                                   \
  case n: {                                                                                    \
    constexpr int L = col_lpw(n), T = col_tl(n);                                               \
    hipLaunchKernelGGL((k_col<n, L, T>), dim3((a.nlines + L - 1) / L), dim3(L * T), 0, s, a); \
    break;                                                                                     \
  }
    X(1)
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_pass(int N, const LineArgs& a, hipStream_t s) {
  switch (N) {
#define X(n)                                                                                   \
  case n: {                                                                                    \
    constexpr int L = row_lpw(n), T = row_tl(n);                                               \
    hipLaunchKernelGGL((k_row<n, L, T>), dim3((a.nlines + L - 1) / L), dim3(L * T), 0, s, a); \
    break;                                                                                     \
  }
    TDSE_LINE_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tdse
