// One-workgroup run of a 1D periodic problem, gfx950: every time step of a
// tdse_step call (the Richardson start-up of Section 2.2 and the implicit
// Adams steps of eq. (uadamsk)) inside one kernel.
//
// A 1D line of N <= 512 points fits one workgroup, so the two passes per
// step of the multi-launch path (a pointwise pass and a row pass, each a
// kernel launch) become one loop in which the line never leaves the
// workgroup: the physical values and the carried state B sit in registers
// (thread t holds elements t + TL m, the layout of fft_lds.h), the FFTs
// exchange through LDS, and only the history ring (read ahead, before the
// transforms that precede its use) goes through memory, where it stays in
// the cache.  Per step the same arithmetic as the multi-launch path:
//   w = F^-1 B,  u = w / (1 + i mu_0 dt V(t_m)),  What_m = F(V(t_m) u),
//   uhat_m = B - i mu_0 dt What_m,
//   B_{m+1} = E^(1)(uhat_m - i dt mu_1 What_m) - i dt sum_{j>=2} mu_j E^(j) What_{m+1-j}.
// The phase factor of Lemma 1 over [t_{m+1-j}, t_{m+1}] is taken as
//   E^(j)[k] = exp(-i k^2 j dt) prod_{i=m+2-j}^{m+1} exp(i k (phi(t_i) - phi(t_{i-1}))),
// a static factor (a table built once per plan in extended precision) times
// the product of per-step increments, each computed from its own small
// argument and kept in registers as a shift register over the last n-1
// steps: no factor is ever raised to a power, so no angle error grows
// with k or with the step count.  With A = 0 the increments are 1.
//
// The start-up step from t_{m-1} runs, for each level l, 2^l order-2
// sub-steps of eq. (utrapk) with delta = dt / 2^l, chained through B in
// mode space as in the multi-launch path, and adds the level's result with
// its folded Richardson weight.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

namespace {

__device__ __forceinline__ int mode_of(int idx, int N) { return idx < (N >> 1) ? idx : idx - N; }

// (-i c) z
__device__ __forceinline__ double2 mi(double c, double2 z) { return double2{c * z.y, -c * z.x}; }

}  // namespace

// PH: the field A is nonzero, so the phase factors carry increments
template <int N, int TL, bool PH>
__global__ __launch_bounds__(TL) void k_run1d(Run1DArgs a) {
  constexpr int EPT = N / TL;
  constexpr int H = MAXH - 1;   // history terms of the order-8 rule
  constexpr double PI = 3.14159265358979323846264338327950288;
  HIP_DYNAMIC_SHARED(double2, run1d_lds)
  double2* line = run1d_lds;                       // FFT exchange line
  double2* twl = line + lds_line_len(N);           // twiddles
  double2* stab = twl + N;                         // static phase factors [rows][N]
  double* Vl = (double*)(stab + a.stab_rows * N);  // potential fields [nV][N]
  const int t = threadIdx.x;
  const int n = a.order, nh = n - 1;
  const double* __restrict__ tab = a.tab;

  // twiddles, static phase factors and potential fields into LDS
  for (int q = t; q < N; q += TL) twl[q] = a.tw[q];
  for (int q = t; q < a.stab_rows * N; q += TL) stab[q] = a.stab[q];
  for (int r = 0; r < a.nV; ++r)
    for (int q = t; q < N; q += TL) Vl[r * N + q] = a.V[r * a.vstride + q];
  __syncthreads();

  // the potential at element m for the time factors fV (stored fields, or
  // the moving well with fV = {-V0, 1/(2 beta^2), -, centre, images})
  auto Vat = [&](const double* fV, int m) -> double {
    const int idx = t + TL * m;
    if (a.vkind == 1) {
      double d = -PI + 2.0 * PI * idx / N - fV[3];
      d -= 2.0 * PI * floor((d + PI) / (2.0 * PI));
      const double s = fV[1];
      double acc = exp(-(d * d) * s);
      const int K = (int)fV[4];
      for (int k = 1; k <= K; ++k) {
        const double y1 = d + 2.0 * PI * k, y2 = d - 2.0 * PI * k;
        acc += exp(-(y1 * y1) * s) + exp(-(y2 * y2) * s);
      }
      return fV[0] * acc;
    }
    double v = 0.0;
    for (int r = 0; r < a.nV; ++r) v += fV[r] * Vl[r * N + idx];
    return v;
  };
  const double scale = 1.0 / N;
  auto fwd = [&](double2* v) { fft_regs<N, TL, false>(v, t, line, twl); };
  auto inv = [&](double2* v) { fft_regs<N, TL, true>(v, t, line, twl); };
  // What = F(V(fV) u), into ring slot s
  auto history = [&](const double2* u, const double* fV, int s) {
    double2 w[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const double vs = Vat(fV, m) * scale;
      w[m] = double2{vs * u[m].x, vs * u[m].y};
    }
    fwd(w);
#pragma unroll
    for (int m = 0; m < EPT; ++m) a.ring[(int64_t)s * N + t + TL * m] = w[m];
  };
  // exp(i k dphi) at element m
  auto incr = [&](double dphi, int m) -> double2 {
    double s, c;
    sincos((double)mode_of(t + TL * m, N) * dphi, &s, &c);
    return double2{c, s};
  };

  double2 u[EPT], B[EPT];
  const int ns = a.ns;
  int m = a.m0 + 1;
  // ------------------------------------------------ Richardson start-up
  if (m <= ns || (m == ns + 1 && m <= a.m1)) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) u[q] = a.u_in[t + TL * q];
  }
  for (; m <= a.m1 && m <= ns; ++m) {
    if (m == 1) history(u, tab + a.oH, 0);
    const double* fpre = tab + a.oH + 8 * (m - 1);
    const double* lev = tab + a.oR + (int64_t)(m - 1) * 9 * ((1 << a.L) - 1);
    double2 acc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) acc[q] = double2{0.0, 0.0};
    for (int l = 0; l < a.L; ++l) {
      const int nsub = 1 << l;
      const double hd = 0.5 * a.dt / nsub;   // delta / 2
      const double* sub = lev + 9 * (nsub - 1);
      const double2* Sl = stab + (a.stab_rows - a.L + l) * N;
      double2 v[EPT];
      // v = F((1 - i delta/2 V(t)) u)
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const double ci = -hd * Vat(fpre, q);
        v[q] = double2{(u[q].x - ci * u[q].y) * scale, (u[q].y + ci * u[q].x) * scale};
      }
      fwd(v);
      double2 Bs[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        double2 E = Sl[t + TL * q];
        if (PH) E = cmul(E, incr(sub[8], q));
        Bs[q] = cmul(E, v[q]);
      }
      for (int k = 0; k < nsub; ++k) {
        const double* fpost = sub + 9 * k;
#pragma unroll
        for (int q = 0; q < EPT; ++q) v[q] = Bs[q];
        inv(v);
        double2 W[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const double Vs = Vat(fpost, q);
          const double qq = hd * Vs;
          const double iv = 1.0 / (1.0 + qq * qq);
          const double2 uu = double2{(v[q].x + qq * v[q].y) * iv, (v[q].y - qq * v[q].x) * iv};
          if (k == nsub - 1) {
            acc[q].x += a.rich[l] * uu.x;
            acc[q].y += a.rich[l] * uu.y;
          }
          const double s = Vs * scale;
          W[q] = double2{s * uu.x, s * uu.y};
        }
        if (k == nsub - 1) break;
        fwd(W);
        const double dphi = fpost[9 + 8];   // the next sub-step's phase increment
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          double2 E = Sl[t + TL * q];
          if (PH) E = cmul(E, incr(dphi, q));
          Bs[q] = cmul(E, double2{Bs[q].x + 2.0 * hd * W[q].y, Bs[q].y - 2.0 * hd * W[q].x});
        }
      }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) u[q] = acc[q];
    history(u, tab + a.oH + 8 * m, m % nh);
  }
  if (a.m1 <= ns) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) a.u_out[t + TL * q] = u[q];
    return;
  }
  // ------------------------------------------------ implicit Adams steps
  // shift register of phase increments: dh[i] = exp(i k (phi(t_{m+1-i}) - phi(t_{m-i}))) for the step m
  // about to form B_{m+1}, i = 0..n-2
  double2 dh[PH ? H : 1][EPT];
  auto dphi_at = [&](int i) -> double { return i >= 1 ? tab[a.oD + i - 1] : 0.0; };
  if constexpr (PH) {
    // the first B formed below is B_{mm0+1} (mm0 = ns at the Adams start,
    // else the step m): slots 1..n-2 hold the increments of the intervals
    // ending at t_{mm0}, t_{mm0-1}, ..
    const int mm0 = (m == ns + 1) ? ns : m;
#pragma unroll
    for (int i = 1; i < H; ++i)
#pragma unroll
      for (int q = 0; q < EPT; ++q) dh[i][q] = (i < nh) ? incr(dphi_at(mm0 + 1 - i), q) : double2{1.0, 0.0};
  }
  // history What_{mm+1-j}, j >= 2, of the B formed at step mm: loaded at the
  // start of the step, so that the transforms before its use hide the wait
  double2 Wh[H - 1][EPT];
  auto load_hist = [&](int mm) {
#pragma unroll
    for (int j = 2; j <= H; ++j) {
      if (j <= nh) {
        const int s = ((mm + 1 - j) % nh + nh) % nh;
#pragma unroll
        for (int q = 0; q < EPT; ++q) Wh[j - 2][q] = a.ring[(int64_t)s * N + t + TL * q];
      }
    }
  };
  // B_{mm+1} from uhat, What_mm = W and the history in Wh
  auto form_B = [&](const double2* uh, const double2* W, int mm) {
    // increments: the new interval [t_mm, t_{mm+1}] into slot 0
    if constexpr (PH) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) dh[0][q] = incr(dphi_at(mm + 1), q);
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      double2 D = PH ? dh[0][q] : double2{1.0, 0.0};
      const double2 E1 = PH ? cmul(stab[t + TL * q], D) : stab[t + TL * q];
      double2 accq = cmul(E1, cadd(uh[q], mi(a.ch[1], W[q])));
      double2 hist = double2{0.0, 0.0};
#pragma unroll
      for (int j = 2; j <= H; ++j) {
        if (j <= nh) {
          double2 Ej = stab[(j - 1) * N + t + TL * q];
          if constexpr (PH) {
            D = cmul(D, dh[j - 1][q]);
            Ej = cmul(Ej, D);
          }
          hist = cadd(hist, mi(a.ch[j], cmul(Ej, Wh[j - 2][q])));
        }
      }
      B[q] = cadd(accq, hist);
    }
    // the shift register moves on by one step
    if constexpr (PH) {
#pragma unroll
      for (int i = H - 1; i >= 1; --i)
#pragma unroll
        for (int q = 0; q < EPT; ++q) dh[i][q] = dh[i - 1][q];
    }
  };
  if (m == ns + 1) {
    // the Adams start: uhat_ns = F u_ns, What_ns in the ring
    if (ns == 0) history(u, tab + a.oH, 0);
    double2 uh[EPT], W[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      uh[q] = double2{u[q].x * scale, u[q].y * scale};
      W[q] = a.ring[(int64_t)(ns % nh) * N + t + TL * q];
    }
    load_hist(ns);
    fwd(uh);
    form_B(uh, W, ns);
  } else {
#pragma unroll
    for (int q = 0; q < EPT; ++q) B[q] = a.B[t + TL * q];
  }
  for (; m <= a.m1; ++m) {
    const double* fV = tab + a.oA + 8 * (m - ns - 1);
    if (m < a.nsteps) load_hist(m);
    double2 v[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) v[q] = B[q];
    inv(v);
    double2 W[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const double Vs = Vat(fV, q);
      const double qq = a.c0 * Vs;
      const double iv = 1.0 / (1.0 + qq * qq);
      u[q] = double2{(v[q].x + qq * v[q].y) * iv, (v[q].y - qq * v[q].x) * iv};
      const double s = Vs * scale;
      W[q] = double2{s * u[q].x, s * u[q].y};
    }
    if (m == a.nsteps) break;
    fwd(W);
    double2 uh[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) uh[q] = cadd(B[q], mi(a.c0, W[q]));
    form_B(uh, W, m);
    // What_m into the ring after the history reads of form_B
#pragma unroll
    for (int q = 0; q < EPT; ++q) a.ring[(int64_t)(m % nh) * N + t + TL * q] = W[q];
  }
  if (a.write_u) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) a.u_out[t + TL * q] = u[q];
  }
  if (a.m1 < a.nsteps) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) a.B[t + TL * q] = B[q];
  }
}

#define TDSE_RUN1D_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512)

bool run1d_supported(int N) {
  switch (N) {
#define X(n) case n:
    TDSE_RUN1D_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

constexpr int run1d_tl(int N) { return N / 4; }

size_t run1d_lds_bytes(int N, int stab_rows, int nV) {
  return sizeof(double2) * ((size_t)lds_line_len(N) + N + (size_t)stab_rows * N) + sizeof(double) * (size_t)nV * N;
}

template <bool PH>
hipError_t run1d_dispatch(const Run1DArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const size_t lds = run1d_lds_bytes(a.M, a.stab_rows, a.nV);
  switch (a.M) {
#define X(n)                                                                                               \
  case n:                                                                                                  \
    if (e0)                                                                                                \
      hipExtLaunchKernelGGL((k_run1d<n, run1d_tl(n), PH>), dim3(1), dim3(run1d_tl(n)), lds, s, e0, e1, 0, a); \
    else                                                                                                   \
      hipLaunchKernelGGL((k_run1d<n, run1d_tl(n), PH>), dim3(1), dim3(run1d_tl(n)), lds, s, a);          \
    break;
    TDSE_RUN1D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_run1d(const Run1DArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return a.has_phase ? run1d_dispatch<true>(a, s, e0, e1) : run1d_dispatch<false>(a, s, e0, e1);
}

}  // namespace tdse
