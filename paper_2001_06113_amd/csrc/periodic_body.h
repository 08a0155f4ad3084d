// Pass bodies of the periodic marching scheme, shared by the per-instance
// kernels (periodic_kernels.hip) and the batched kernels (batch_kernels.h).
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
// Every kernel is a template on the transform type C: double2 (FP64) or
// float2 (split precision).  In the split form the FFTs, the tile buffer,
// the history ring, the diagonal solve and the products E^(j) What (j >= 2)
// are complex64, while B, E^(1) uhat, the dt mu_j weighting and sum of the
// history products, the phase factors, the potential, the Richardson
// accumulator and the physical solution stay FP64.  (A weight or a
// potential rounded to FP32 is the same perturbation of the scheme at every
// step, so its error would grow linearly in time rather than as a random
// walk.)
//
// Every global load a pass needs (tile, potential, B, history, phase factors)
// is issued before its first FFT so their latencies overlap, in the order of
// first use: a wave's loads complete in issue order, so waiting for one
// waits for all loads issued before it.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {


template <typename C>
struct real_of;
template <>
struct real_of<double2> { using type = double; };
template <>
struct real_of<float2> { using type = float; };

template <typename C>
__device__ __forceinline__ C from_d(double2 z) {
  using R = typename real_of<C>::type;
  return C{(R)z.x, (R)z.y};
}
template <typename C>
__device__ __forceinline__ double2 to_d(C z) { return double2{(double)z.x, (double)z.y}; }

// FFT index -> integer mode in [-M/2, M/2) (M even; M = 1 is the single mode 0)
__device__ __forceinline__ int signed_mode(int idx, int M) { return idx < ((M + 1) >> 1) ? idx : idx - M; }

// (-i c) * z
template <typename C>
__device__ __forceinline__ C mul_mi(double c, C z) {
  using R = typename real_of<C>::type;
  const R cc = (R)c;
  return C{cc * z.y, -cc * z.x};
}

// Per-axis phase table of the next row pass, spread over the nblk workgroups
// of the instance's column pass (blk = this workgroup's index), FP64, and
// rounded to complex64 into ph32 for the split form.
__device__ __forceinline__ void build_phase_table(const LineArgs& a, int nthreads, int blk, int nblk) {
  const int per = a.M1 + a.M2;
  const int total = a.req.nj * per;
  for (int idx = blk * nthreads + threadIdx.x; idx < total; idx += nblk * nthreads) {
    const int j = idx / per;
    const int kk = idx - j * per;
    double th;
    if (kk >= a.M1) {
      const double k = (double)signed_mode(kk - a.M1, a.M2);
      th = -(k * k) * a.req.tau[j] + k * a.req.dphi2[j];
    } else if (a.Mmid == 0) {
      const double k = (double)signed_mode(kk, a.M1);
      th = -(k * k) * a.req.tau[j] + k * a.req.dphi1[j];
    } else {   // 3D row (k0, k1)
      const int i0 = kk / a.Mmid;
      const double k0 = (double)signed_mode(i0, a.M0), k1 = (double)signed_mode(kk - i0 * a.Mmid, a.Mmid);
      th = -(k0 * k0 + k1 * k1) * a.req.tau[j] + k0 * a.req.dphi0[j] + k1 * a.req.dphi1[j];
    }
    double s, c;
    sincos(th, &s, &c);
    a.ph[idx] = double2{c, s};
    if (a.ph32) a.ph32[idx] = float2{(float)c, (float)s};
  }
}

// Moving periodic Gaussian well (Example 1 of Section 6), one axis:
// sum_{|k| <= K} exp(-(d + 2 pi k)^2 s) for the offset d = x - centre
// wrapped into [-pi, pi), s = 1/(2 beta^2).  The host picks K so that every
// image within 9.2 beta of x is kept; the ones left out are below
// exp(-42) ~ 4e-19 of the well depth.
__device__ __forceinline__ double well_images(double d, double s, int K) {
  constexpr double TWO_PI = 6.28318530717958647692528676655900577;
  d -= TWO_PI * floor((d + 0.5 * TWO_PI) / TWO_PI);
  double acc = exp(-(d * d) * s);
  for (int k = 1; k <= K; ++k) {
    const double y1 = d + TWO_PI * k, y2 = d - TWO_PI * k;
    acc += exp(-(y1 * y1) * s) + exp(-(y2 * y2) * s);
  }
  return acc;
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

template <typename C, int N, int LPW>
struct col_lds {
  static constexpr int PITCH = N > 1 ? lds_line_len(N) + 1 : 1;   // +1 spreads the LPW lines over banks
  static constexpr bool TWL = (N > 1 && N <= 1024);
  static constexpr int elems = LPW * PITCH + (TWL ? N : 0);      // line buffers, then the twiddles
};

// Column pass over lines line0 .. line0+LPW-1 of one instance; blk/nblk
// place this workgroup among the instance's column-pass workgroups (for the
// phase table).  lds holds col_lds<C,N,LPW>::elems elements.
template <typename C, int N, int LPW, int TL>
__device__ __forceinline__ void col_body(const LineArgs& a, int line0, int blk, int nblk, C* lds) {
  using R = typename real_of<C>::type;
  constexpr int NT = LPW * TL;
  constexpr int EPT = N / TL;
  constexpr int PITCH = col_lds<C, N, LPW>::PITCH;
  constexpr bool TWL = col_lds<C, N, LPW>::TWL;
  C* twl = lds + LPW * PITCH;
  const int tid = threadIdx.x;
  const int i = tid % LPW, t = tid / LPW;
  const int line = line0 + i;
  const bool active = line < a.nlines;
  const int mode = a.mode;
  const double* __restrict__ V = (const double*)a.V;

  C v[EPT];
  double2 u0[EPT];   // C_FWD reads the complex128 physical solution
  double vv[EPT];   // potential fields after the first (summed at first use)
  const int64_t g0 = (int64_t)line * a.line_stride + (int64_t)t * a.elem_stride;
  const int64_t gs = (int64_t)TL * a.elem_stride;
  // loads in the order of first use (they complete in order): twiddles,
  // tile, then the potential, which is needed only after the first FFT
  constexpr int TWN = TWL ? (N + NT - 1) / NT : 1;
  C twr[TWN];
  if constexpr (TWL) {
#pragma unroll
    for (int k = 0; k < TWN; ++k) {
      const int q = tid + k * NT;
      if (N % NT == 0 || q < N) twr[k] = ((const C*)a.tw)[q];
    }
  }
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    v[m] = C{0, 0};
    u0[m] = double2{0.0, 0.0};
    vv[m] = 0.0;
  }
  // In FP64 the tile and the physical solution have one element type: one
  // load serves both modes (a per-mode choice between two loaded copies
  // would wait for the data at once)
  constexpr bool F64 = sizeof(C) == sizeof(double2);
  if (active) {
    if (F64 || mode != C_FWD) {
#pragma unroll
      for (int m = 0; m < EPT; ++m) v[m] = ((const C*)a.src)[g0 + m * gs];
    } else {
#pragma unroll
      for (int m = 0; m < EPT; ++m) u0[m] = ((const double2*)a.src)[g0 + m * gs];
    }
  }
  if constexpr (TWL) {
#pragma unroll
    for (int k = 0; k < TWN; ++k) {
      const int q = tid + k * NT;
      if (N % NT == 0 || q < N) twl[q] = twr[k];
    }
  }
  // potential: the first field's loads stay in flight through the first
  // FFT (its product is formed at first use); further fields, if any, are
  // summed into vv just before the pointwise step
  double v0[EPT];
  const double f0 = a.nV > 0 ? a.fV[0] : 0.0;
#pragma unroll
  for (int m = 0; m < EPT; ++m) v0[m] = 0.0;
  if (active && a.nV > 0) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v0[m] = V[g0 + m * gs];
  }
  // moving well: V = -V0 prod_axes well_images(x_a - centre_a); the last
  // axis' factor is fixed along a column (x of the column index, or of the
  // point itself for a 1D problem)
  constexpr double PI = 3.14159265358979323846264338327950288;
  const bool well = a.vkind == 1;
  const int wK = well ? (int)a.fV[4] : 0;
  const double wline = well ? a.fV[0] * well_images(-PI + 2.0 * PI * line / a.M2 - a.fV[3], a.fV[1], wK) : 0.0;
  auto V_at = [&](int m) -> double {
    if (!well) return vv[m] + f0 * v0[m];
    if (a.M1 == 1) return wline;
    return wline * well_images(-PI + 2.0 * PI * (t + TL * m) / a.M1 - a.fV[2], a.fV[1], wK);
  };
  auto more_fields = [&]() {
    if (!active) return;
    for (int r = 1; r < a.nV; ++r) {
      double vr[EPT];
#pragma unroll
      for (int m = 0; m < EPT; ++m) vr[m] = V[r * a.vstride + g0 + m * gs];
#pragma unroll
      for (int m = 0; m < EPT; ++m) vv[m] += a.fV[r] * vr[m];
    }
  };
  if constexpr (TWL) __syncthreads();
  const C* tw = TWL ? twl : (const C*)a.tw;
  C* myline = &lds[i * PITCH];

  if (mode == C_FWD) {
    more_fields();
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double Vs = V_at(m);
      const double cr = a.alpha_re + a.beta_re * Vs, ci = a.alpha_im + a.beta_im * Vs;
      const double2 u = F64 ? to_d(v[m]) : u0[m];
      v[m] = from_d<C>(double2{(cr * u.x - ci * u.y) * a.scale, (cr * u.y + ci * u.x) * a.scale});
    }
  } else {  // C_SOLVE
    fft_regs<N, TL, true>(v, t, myline, tw);
    more_fields();
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const C w = v[m];
      const double Vs = V_at(m);
      const R q = (R)(a.csolve * Vs);
      const R inv = R(1) / (R(1) + q * q);
      // u = w (1 - i q) / (1 + q^2)
      const C u = C{(w.x + q * w.y) * inv, (w.y - q * w.x) * inv};
      if (active) {
        const int64_t g = (int64_t)line * a.line_stride + (int64_t)(t + TL * m) * a.elem_stride;
        const double2 ud = to_d(u);
        if (a.uout) a.uout[g] = ud;
        if (a.uacc) {
          double2 acc = a.acc_first ? double2{0.0, 0.0} : a.uacc[g];
          acc.x += a.wacc * ud.x;
          acc.y += a.wacc * ud.y;
          a.uacc[g] = acc;
        }
      }
      const R s = (R)(Vs * a.scale);
      v[m] = C{s * u.x, s * u.y};
    }
  }
  fft_regs<N, TL, false>(v, t, myline, tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int64_t g = (int64_t)line * a.line_stride + (int64_t)(t + TL * m) * a.elem_stride;
      ((C*)a.dst)[g] = v[m];
    }
  }
  // last, so that its loads and waits delay none of the pass's own
  if (a.req.nj > 0) build_phase_table(a, NT, blk, nblk);
}


// Middle-axis pass of a 3D grid: FFT along axis 1 only (inverse before the
// column pass, forward after it), in place.  Lines (i0, i2) of N elements at
// stride elem_stride = M2, grouped in slabs of slab_lines = M2 lines per i0
// (line l starts at (l / M2) slab_stride + l mod M2); lanes run across
// consecutive lines as in the column pass.
template <typename C, int N, int LPW, int TL, bool INV>
__device__ __forceinline__ void mid_body(const LineArgs& a, int line0, C* lds) {
  constexpr int NT = LPW * TL;
  constexpr int EPT = N / TL;
  constexpr int PITCH = col_lds<C, N, LPW>::PITCH;
  constexpr bool TWL = col_lds<C, N, LPW>::TWL;
  C* twl = lds + LPW * PITCH;
  const int tid = threadIdx.x;
  const int i = tid % LPW, t = tid / LPW;
  const int line = line0 + i;
  const bool active = line < a.nlines;
  const int64_t base = (int64_t)(line / a.slab_lines) * a.slab_stride + (int64_t)(line % a.slab_lines) * a.line_stride;
  constexpr int TWN = TWL ? (N + NT - 1) / NT : 1;
  C twr[TWN];
  if constexpr (TWL) {
#pragma unroll
    for (int k = 0; k < TWN; ++k) {
      const int q = tid + k * NT;
      if (N % NT == 0 || q < N) twr[k] = ((const C*)a.tw)[q];
    }
  }
  C v[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) v[m] = C{0, 0};
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = ((const C*)a.src)[base + (int64_t)(t + TL * m) * a.elem_stride];
  }
  if constexpr (TWL) {
#pragma unroll
    for (int k = 0; k < TWN; ++k) {
      const int q = tid + k * NT;
      if (N % NT == 0 || q < N) twl[q] = twr[k];
    }
    __syncthreads();
  }
  const C* tw = TWL ? twl : (const C*)a.tw;
  fft_regs<N, TL, INV>(v, t, &lds[i * PITCH], tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) ((C*)a.dst)[base + (int64_t)(t + TL * m) * a.elem_stride] = v[m];
  }
}


// ---------------------------------------------------------------- row pass

template <typename C, int N, int LPW>
struct row_lds {
  static constexpr int PITCH = lds_line_len(N);
  static constexpr bool TWL = (N <= 1024);
  static constexpr int elems = LPW * PITCH + (TWL ? N : 0);
};

// Row pass over rows k1 = line0 .. line0+LPW-1 of one instance; lds holds
// row_lds<C,N,LPW>::elems elements.
template <typename C, int N, int LPW, int TL, bool PW = false>
__device__ __forceinline__ void row_body(const LineArgs& a, int line0, C* lds) {
  constexpr int NT = LPW * TL;
  constexpr int EPT = N / TL;
  constexpr int NH = MAXH - 1;    // history terms of the order-8 rule (j = 1..7)
  constexpr bool PF = EPT <= 4;   // prefetch history and phases into registers
  constexpr bool TWL = row_lds<C, N, LPW>::TWL;
  constexpr int PITCH = row_lds<C, N, LPW>::PITCH;
  C* twl = lds + LPW * PITCH;
  const int tid = threadIdx.x;
  const int i = tid / TL, t = tid % TL;
  const int k1 = line0 + i;
  const bool active = k1 < a.nlines;
  const int mode = a.mode;
  const int per = a.M1 + a.M2;
  const int nh = a.nh;
  const int64_t row0 = (int64_t)k1 * a.line_stride;
  const C* __restrict__ src = (const C*)a.src;
  const double2* __restrict__ ph = a.ph;
  const C* __restrict__ ring = (const C*)a.ring;
  const int64_t rstride = a.ring_stride;
  const int M1 = a.M1;
  int slot_r[MAXH + 1];
#pragma unroll
  for (int j = 0; j <= MAXH; ++j) slot_r[j] = a.slot_r[j];

  C v[EPT];
  double2 Bp[EPT];
  C Wr[PF ? NH - 1 : 1][EPT];
  // E^(1) = T1[0] P1 in FP64 (it multiplies uhat), formed only after the
  // forward FFT: a product taken here would wait for its loads, and loads
  // complete in order, so for every load issued before them
  double2 P1[EPT];
  // axis-2 factors of E^(j), j >= 2, transform precision; PW (no field along
  // axis 2): exp(-i k^2 j dt) = P1^j, formed by FP64 products instead (the
  // split form rounds E^(j) to complex64 once, as it rounds the table)
  C T2[PF && !PW ? NH - 1 : 1][EPT];
  double2 T1[NH];
  constexpr bool F64 = sizeof(C) == sizeof(double2);
  // Loads are issued in the order their values are first needed, since
  // they complete in order: twiddles (staged into LDS), the row factors T1
  // (uniform along the row), the tile, then B, the history and the axis-2
  // factors, which are used only after the forward FFT.
  constexpr int TWN = TWL ? (N + NT - 1) / NT : 1;
  C twr[TWN];
  if constexpr (TWL) {
#pragma unroll
    for (int i = 0; i < TWN; ++i) {
      const int q = tid + i * NT;
      if (N % NT == 0 || q < N) twr[i] = ((const C*)a.tw)[q];
    }
  }
  const bool phases = active && mode != R_FWD && mode != R_INV;
  const int nj = (mode == R_INIT) ? 1 : nh;
  if (phases) {
    // unconditional (entries past nj repeat entry nj and go unused), so the
    // loads share one block and one wait
    const int njc = nj > 1 ? nj : 1;
#pragma unroll
    for (int j = 1; j <= NH; ++j) T1[j - 1] = ph[((j < njc ? j : njc) - 1) * per + k1];
  }
#pragma unroll
  for (int m = 0; m < EPT; ++m) v[m] = C{0, 0};
  if (active) {
    // one loop per source: a per-element choice would wait for the data
    if (mode == R_INV) {
#pragma unroll
      for (int m = 0; m < EPT; ++m) v[m] = from_d<C>(a.Bm[row0 + (t + TL * m)]);
    } else {
#pragma unroll
      for (int m = 0; m < EPT; ++m) v[m] = src[row0 + (t + TL * m)];
    }
  }
  // twiddles into LDS before the later loads are issued: waiting for them
  // then never waits for those
  if constexpr (TWL) {
#pragma unroll
    for (int i = 0; i < TWN; ++i) {
      const int q = tid + i * NT;
      if (N % NT == 0 || q < N) twl[q] = twr[i];
    }
  }
  if (active && mode == R_AM) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) Bp[m] = a.Bm[row0 + (t + TL * m)];
    if constexpr (PF) {
#pragma unroll
      for (int j = 2; j <= NH; ++j) {
        if (j <= nh) {
#pragma unroll
          for (int m = 0; m < EPT; ++m) Wr[j - 2][m] = ring[slot_r[j] * rstride + row0 + (t + TL * m)];
        }
      }
    }
  }
  if (phases) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) P1[m] = ph[M1 + (t + TL * m)];
    if constexpr (PF && !PW) {
      // the split form reads the complex64 copy: no conversion waits here
      const C* __restrict__ tpj = F64 ? (const C*)ph : (const C*)a.ph32;
#pragma unroll
      for (int j = 2; j <= NH; ++j) {
        if (j <= nj) {
#pragma unroll
          for (int m = 0; m < EPT; ++m) T2[j - 2][m] = tpj[(j - 1) * per + M1 + (t + TL * m)];
        }
      }
    }
  }
  // E^(j), j >= 2, and the history term What_{n+1-j} at element m, from
  // registers (PF) or memory.  Only plain locals are captured: taking the
  // address of the by-value kernel argument would copy it to scratch.
  auto Ej = [&T1, &T2, ph, per, M1, t](int j, int m) -> C {
    if constexpr (PF && !PW) return cmul(from_d<C>(T1[j - 1]), T2[j - 2][m]);
    else return from_d<C>(cmul(T1[j - 1], ph[(j - 1) * per + M1 + (t + TL * m)]));
  };
  auto Wh = [&Wr, &slot_r, ring, rstride, row0, t](int j, int m) -> C {
    if constexpr (PF) return Wr[j - 2][m];
    else return ring[slot_r[j] * rstride + row0 + (t + TL * m)];
  };
  if constexpr (TWL) __syncthreads();
  const C* tw = TWL ? twl : (const C*)a.tw;
  C* myline = &lds[i * PITCH];

  if (mode != R_INV) fft_regs<N, TL, false>(v, t, myline, tw);

  if (mode == R_FWD) {
    if (active) {
#pragma unroll
      for (int m = 0; m < EPT; ++m) ((C*)a.fdst)[row0 + (t + TL * m)] = v[m];
    }
    return;
  }
  // fused recurrence; lanes past the last line (ragged tile) only keep the
  // FFT barriers company and touch no memory
  if (!active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = C{0, 0};
  } else if (mode == R_INV) {
    // v already holds the row of B
  } else if (mode == R_AM) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const C W = v[m];
      const double2 Wd = to_d(W);
      const double2 uh = cadd(Bp[m], mul_mi(a.c0, Wd));
      double2 acc = cmul(cmul(T1[0], P1[m]), cadd(uh, mul_mi(a.ch[1], Wd)));
      // products E^(j) What in the transform precision, weighted by dt mu_j
      // and summed in FP64
      double2 hist = double2{0.0, 0.0};
      if constexpr (PW) {
        double2 R = P1[m];
#pragma unroll
        for (int j = 2; j <= NH; ++j) {
          if (j <= nh) {
            R = cmul(R, P1[m]);
            if constexpr (F64) hist = cadd(hist, mul_mi(a.ch[j], cmul(cmul(T1[j - 1], R), to_d(Wh(j, m)))));
            else hist = cadd(hist, mul_mi(a.ch[j], to_d(cmul(from_d<C>(cmul(T1[j - 1], R)), Wh(j, m)))));
          }
        }
      } else {
#pragma unroll
        for (int j = 2; j <= NH; ++j) {
          if (j <= nh) hist = cadd(hist, mul_mi(a.ch[j], to_d(cmul(Ej(j, m), Wh(j, m)))));
        }
      }
      acc = cadd(acc, hist);
      const int64_t g = row0 + (t + TL * m);
      if (a.slot_w >= 0) ((C*)a.ring)[a.slot_w * rstride + g] = W;
      a.Bm[g] = acc;
      v[m] = from_d<C>(acc);
    }
  } else if (mode == R_INIT) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double2 acc = cmul(cmul(T1[0], P1[m]), to_d(v[m]));
      a.Bm[row0 + (t + TL * m)] = acc;
      v[m] = from_d<C>(acc);
    }
  } else {  // R_FORM: B from uhat (this FFT) and nh history terms, all from the ring
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double2 E1 = cmul(T1[0], P1[m]);
      double2 acc = cmul(E1, to_d(v[m]));
      const int64_t g = row0 + (t + TL * m);
      acc = cadd(acc, cmul(E1, mul_mi(a.ch[1], to_d(ring[slot_r[1] * rstride + g]))));
      double2 hist = double2{0.0, 0.0};
#pragma unroll
      for (int j = 2; j <= NH; ++j) {  // static j: registers stay registers
        if (j <= nh) hist = cadd(hist, mul_mi(a.ch[j], to_d(cmul(Ej(j, m), ring[slot_r[j] * rstride + g]))));
      }
      acc = cadd(acc, hist);
      a.Bm[g] = acc;
      v[m] = from_d<C>(acc);
    }
  }
  fft_regs<N, TL, true>(v, t, myline, tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) ((C*)a.dst)[row0 + (t + TL * m)] = v[m];
  }
}


}  // namespace tdse
