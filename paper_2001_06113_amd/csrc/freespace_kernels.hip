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
// Two thread layouts: nu/8 threads that carry both rays (the row pass at
// nu >= 1024 in 2D and 3D, with many rows and two workgroups per CU), and
// nu/4 threads with a ray per half (the column and middle-axis passes, the
// single row of a 1D problem, where one workgroup's latency is the pass's,
// and the short rows of nu <= 512).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

__device__ __forceinline__ double2 fs_mul_mi(double c, double2 z) { return double2{c * z.y, -c * z.x}; }

// Per-axis phase factors exp(i(-zeta^2 tau_j + zeta dphi_j)) for complex
// nodes zeta (|.| != 1 off the real axis), table ph[(j-1)(N1+N2) + k]; in
// 3D the first N1 = N0 Nm entries are the products of the axis-0 and
// middle-axis factors of the row (k0, k1).
__device__ __forceinline__ void build_phase_table_fs(const FSArgs& a, int nthreads) {
  const int per = a.N1 + a.N2;
  const int total = a.req.nj * per;
  for (int idx = blockIdx.x * nthreads + threadIdx.x; idx < total; idx += gridDim.x * nthreads) {
    const int j = idx / per;
    const int kk = idx - j * per;
    // theta = -(z . z) tau + z . dphi (complex); exp(i theta)
    double tr, ti;
    auto add = [&](double2 z, double dphi) {
      const double2 z2 = cmul(z, z);
      tr += -z2.x * a.req.tau[j] + z.x * dphi;
      ti += -z2.y * a.req.tau[j] + z.y * dphi;
    };
    tr = 0.0;
    ti = 0.0;
    if (kk >= a.N1) {
      add(a.ax2.zeta[kk - a.N1], a.req.dphi2[j]);
    } else if (a.Nm == 0) {
      add(a.ax1.zeta ? a.ax1.zeta[kk] : double2{0.0, 0.0}, a.req.dphi1[j]);
    } else {   // 3D row (k0, k1): axis 0 and the middle axis
      const int k0 = kk / a.Nm;
      add(a.ax1.zeta[k0], a.req.dphi0[j]);
      add(a.axm.zeta[kk - k0 * a.Nm], a.req.dphi1[j]);
    }
    const double mag = exp(-ti);
    double s, c;
    sincos(tr, &s, &c);
    a.ph[idx] = double2{mag * c, mag * s};
  }
}

// Line transforms with the ray modes in registers.  Thread t holds, for
// e = t + TL m: v3[m] = mode N - N_E + e (E3 ray) and v1[m] = mode N_E - 1 - e
// (E1 ray), zero for e >= N_E, which is the layout the nu-point FFT leaves
// them in.  N_E = nu/2 - 13 < nu/2 = 4 TL, so only m < RAY = 4 can hold a
// ray mode: the rays are carried as four values per thread, and the other
// four FFT slots are compile-time zeros going into the inverse FFTs.  The
// two rays' nu-point FFTs run together (fft_regs_dual), each line with its
// own LDS exchange buffer, so they share every exchange barrier.  The N_D
// dense modes N_E + q live in LDS (dm).  The dense block's forward sums are
// split over (mode, chunk) pairs and reduced through LDS (part, N_D *
// max(1, TL / N_D) entries, in the second exchange line once its FFT is done).
constexpr int RAY = 4;

// nu-point twiddles from two small tables in LDS (TwPair): 2^LF fine and
// nu / 2^LF coarse entries, staged from the full table at kernel start
template <int NU>
struct fs_tw {
  static constexpr int LF = NU >= 2048 ? 6 : (NU >= 512 ? 5 : 4);
  static constexpr int NF = 1 << LF, NC = NU >> LF;
  using type = TwPair<double2, LF>;
};
template <int NU>
__device__ __forceinline__ typename fs_tw<NU>::type stage_twiddles(const CFAxis& ax, double2* tws, int t) {
  constexpr int NC = fs_tw<NU>::NC, NF = fs_tw<NU>::NF, LF = fs_tw<NU>::LF;
  for (int i = t; i < NC + NF; i += NU / 8) tws[i] = i < NC ? ax.tw[i << LF] : ax.tw[i - NC];
  return typename fs_tw<NU>::type{tws, tws + NC};
}

// forward transform of f[0..M) (LDS); ends with dm complete (a barrier).
// dm may share f's LDS: it is written only after the last read of f.
// CH: the C-type block through the interpolant (ax.NT > 0).
template <int NU, bool CH>
__device__ __forceinline__ void cf_forward(const double2* f, double2 (&v3)[RAY], double2 (&v1)[RAY], double2* dm,
                                           double2* part, double2* fline, double2* fline2, const CFAxis& ax,
                                           const typename fs_tw<NU>::type& tw, int t) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND;
  // Table reads use an in-range twin index (min(e, n - 1)) and the result is
  // selected afterwards, so they carry no branch and issue together.
  double2 w[EPT], w1[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m, ec = min(e, M - 1);
    const double2 x = cmul(ax.pre3[ec], f[ec]), y = cmul(ax.pre1[ec], f[ec]);
    w[m] = e < M ? x : double2{0.0, 0.0};
    w1[m] = e < M ? y : double2{0.0, 0.0};
  }
  fft_regs_dual<NU, TL, false, true>(w, w1, t, fline, fline2, tw);
#pragma unroll
  for (int m = 0; m < RAY; ++m) {
    const int e = t + TL * m;
    const double2 x = cmul(ax.post3[min(e, NE - 1)], w[m]);
    v3[m] = e < NE ? x : double2{0.0, 0.0};
    const double2 y = cmul(ax.post1[min(e, NE - 1)], w1[m]);
    v1[m] = e < NE ? y : double2{0.0, 0.0};
  }
  // dense rows: thread (q, c) sums the contiguous chunk j0 <= j < j0 + L of
  // the row q of Dfwd.  Entries along a row form a geometric sequence
  // (equispaced x_j), so the chunk is Dfwd[q][j0] times a Horner sum in the
  // ratio rfwd[q]: two table reads per chunk, L LDS reads.
  const int NR = CH ? ax.NR : ND;
  const int C = TL / NR > 1 ? TL / NR : 1;
  // the rows' sums: the modes themselves without the interpolant, else the
  // node values, kept in the second exchange line behind the partials
  double2* dr = CH ? part + NR * C : dm;
  const int L = (M + C - 1) / C;
  for (int i = t; i < NR * C; i += TL) {   // more dense rows than threads: several pairs per thread
    const int q = i / C, c = i - q * C;
    const int j0 = c * L, j1 = min(j0 + L, M);
    double2 acc = {0.0, 0.0};
    if (j0 < M) {
      const double2 r = ax.rfwd[q];
      const double2 d0 = ax.Dfwd[(int64_t)q * M + j0];
      for (int j = j1 - 1; j >= j0; --j) acc = cadd(cmul(acc, r), f[j]);
      acc = cmul(d0, acc);
    }
    part[i] = acc;
  }
  __syncthreads();
  for (int q = t; q < NR; q += TL) {
    double2 acc = {0.0, 0.0};
    for (int c = 0; c < C; ++c) acc = cadd(acc, part[q * C + c]);
    dr[q] = acc;
  }
  __syncthreads();
  if (CH) {
    // C-modes from the transform's values at the interpolation nodes
    // (Section 4.1, eq. (expintrpm) in the form of its values): the Alpert
    // rows are modes already
    const int P = ax.NP, NT = ax.NT, NC = ND - 2 * P;
    for (int q = t; q < ND; q += TL) {
      double2 v;
      if (q < P) {
        v = dr[q];
      } else if (q >= P + NC) {
        v = dr[q - NC + NT];
      } else {
        const double* __restrict__ pr = ax.Pf + (int64_t)(q - P) * NT;
        v = double2{0.0, 0.0};
        for (int m = 0; m < NT; ++m) {
          const double w = pr[m];
          const double2 x = dr[P + m];
          v.x += w * x.x;
          v.y += w * x.y;
        }
      }
      dm[q] = v;
    }
    __syncthreads();
  }
}

// inverse transform of the modes (v3, v1 registers, dm LDS) into u[0..M)
// (LDS); thread t writes u[t + TL m] only, so it may read those entries back
// without a barrier.  With the interpolant (CH) dm shares u's LDS: u is
// written only after every read of dm.
template <int NU, bool CH>
__device__ __forceinline__ void cf_inverse(const double2 (&v3)[RAY], const double2 (&v1)[RAY], const double2* dm,
                                           double2* fline, double2* fline2, const CFAxis& ax,
                                           const typename fs_tw<NU>::type& tw, int t, double2* u) {
  constexpr int TL = NU / 8;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND, NR = CH ? ax.NR : ND;
  double2 w[EPT], w1[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (m < RAY) {
      const double2 x = cmul(ax.ipre3[min(e, NE - 1)], v3[m < RAY ? m : 0]);
      w[m] = e < NE ? x : double2{0.0, 0.0};
      const double2 y = cmul(ax.ipre1[min(e, NE - 1)], v1[m < RAY ? m : 0]);
      w1[m] = e < NE ? y : double2{0.0, 0.0};
    } else {
      w[m] = double2{0.0, 0.0};
      w1[m] = double2{0.0, 0.0};
    }
  }
  fft_regs_dual<NU, TL, true, false>(w, w1, t, fline, fline2, tw);   // ends with a barrier: both lines free
  constexpr int DB = 18;   // dense rows per batch of matrix entries
  if constexpr (!CH) {
    // dm has LDS of its own: E3 part into u, then E1 and the dense modes
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < M) u[e] = cmul(ax.ipost3[e], w[m]);
    }
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < M) {
        double2 s = cadd(u[e], cmul(ax.ipost1[e], w1[m]));
        for (int q0 = 0; q0 < ND; q0 += DB) {
          double2 d[DB];
#pragma unroll
          for (int u8 = 0; u8 < DB; ++u8) d[u8] = ax.Dinv[(int64_t)min(q0 + u8, ND - 1) * M + e];
#pragma unroll
          for (int u8 = 0; u8 < DB; ++u8) {
            if (q0 + u8 < ND) s = cadd(s, cmul(d[u8], dm[q0 + u8]));
          }
        }
        u[e] = s;
      }
    }
  } else {
    // dm shares u's LDS.  Contract the C-modes onto the interpolation nodes
    // (eq. (expintrpp) in the form of its values), split over (node, chunk)
    // pairs and reduced through the second exchange line, which then holds
    // the node values dv.
    const int P = ax.NP, NT = ax.NT, NC = ND - 2 * P;
    const int C = TL / NR > 1 ? TL / NR : 1;
    const int L = (NC + C - 1) / C;
    double2* dv = fline2 + NR * C;
    for (int i = t; i < NR * C; i += TL) {
      const int r = i / C, c = i - r * C;
      double2 acc = {0.0, 0.0};
      if (r < P || r >= P + NT) {
        if (c == 0) acc = dm[r < P ? r : r - NT + NC];
      } else {
        const double2* __restrict__ pr = ax.Pi + (int64_t)(r - P) * NC;
        const int k1 = min(c * L + L, NC);
        for (int k = c * L; k < k1; ++k) acc = cadd(acc, cmul(pr[k], dm[P + k]));
      }
      fline2[i] = acc;
    }
    __syncthreads();
    for (int r = t; r < NR; r += TL) {
      double2 acc = {0.0, 0.0};
      for (int c = 0; c < C; ++c) acc = cadd(acc, fline2[r * C + c]);
      dv[r] = acc;
    }
    __syncthreads();   // dv complete, and every read of dm done: u may be written
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < M) {
        double2 s = cadd(cmul(ax.ipost3[e], w[m]), cmul(ax.ipost1[e], w1[m]));
        for (int q0 = 0; q0 < NR; q0 += DB) {
          double2 d[DB];
#pragma unroll
          for (int u8 = 0; u8 < DB; ++u8) d[u8] = ax.Dinv[(int64_t)min(q0 + u8, NR - 1) * M + e];
#pragma unroll
          for (int u8 = 0; u8 < DB; ++u8) {
            if (q0 + u8 < NR) s = cadd(s, cmul(d[u8], dv[q0 + u8]));
          }
        }
        u[e] = s;
      }
    }
  }
}

// Ray-split line transforms: 2 TL threads per line.  Threads [0, TL) carry
// the E3 ray and threads [TL, 2 TL) the E1 ray, each thread one FFT line of
// its own ray (v[m] = that ray's mode at e = t + TL m, as above).  Both
// halves run the same forward FFT (the ray whose transform is an inverse FFT
// conjugates before and after it), so every barrier is reached from the same
// code; the two lines' exchanges share them.
template <int NU>
__device__ __forceinline__ typename fs_tw<NU>::type stage_twiddles_n(const CFAxis& ax, double2* tws, int tid,
                                                                     int nth) {
  constexpr int NC = fs_tw<NU>::NC, NF = fs_tw<NU>::NF, LF = fs_tw<NU>::LF;
  for (int i = tid; i < NC + NF; i += nth) tws[i] = i < NC ? ax.tw[i << LF] : ax.tw[i - NC];
  return typename fs_tw<NU>::type{tws, tws + NC};
}

__device__ __forceinline__ double2 conj_if(bool c, double2 z) { return c ? double2{z.x, -z.y} : z; }

// forward transform of f[0..M) (LDS) on the thread's ray; ends with dm
// complete (a barrier).  dm may share f's LDS (CH), as in cf_forward.
template <int NU, bool CH>
__device__ __forceinline__ void rs_forward(const double2* f, double2 (&v)[RAY], double2* dm, double2* part,
                                           double2* fline, double2* fline2, const CFAxis& ax,
                                           const typename fs_tw<NU>::type& tw, int tid) {
  constexpr int TL = NU / 8, NTH = 2 * TL;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND;
  const bool ray = tid >= TL;   // false: E3 (forward FFT), true: E1 (inverse FFT)
  const int t = ray ? tid - TL : tid;
  const double2* __restrict__ pre = ray ? ax.pre1 : ax.pre3;
  const double2* __restrict__ post = ray ? ax.post1 : ax.post3;
  double2 w[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m, ec = min(e, M - 1);
    const double2 x = conj_if(ray, cmul(pre[ec], f[ec]));
    w[m] = e < M ? x : double2{0.0, 0.0};
  }
  fft_regs<NU, TL, false>(w, t, ray ? fline2 : fline, tw);
#pragma unroll
  for (int m = 0; m < RAY; ++m) {
    const int e = t + TL * m;
    const double2 x = cmul(post[min(e, NE - 1)], conj_if(ray, w[m]));
    v[m] = e < NE ? x : double2{0.0, 0.0};
  }
  // dense rows as in cf_forward, over all 2 TL threads
  const int NR = CH ? ax.NR : ND;
  const int C = NTH / NR > 1 ? NTH / NR : 1;
  double2* dr = CH ? part + NR * C : dm;
  const int L = (M + C - 1) / C;
  for (int i = tid; i < NR * C; i += NTH) {
    const int q = i / C, c = i - q * C;
    const int j0 = c * L, j1 = min(j0 + L, M);
    double2 acc = {0.0, 0.0};
    if (j0 < M) {
      const double2 r = ax.rfwd[q];
      const double2 d0 = ax.Dfwd[(int64_t)q * M + j0];
      for (int j = j1 - 1; j >= j0; --j) acc = cadd(cmul(acc, r), f[j]);
      acc = cmul(d0, acc);
    }
    part[i] = acc;
  }
  __syncthreads();
  for (int q = tid; q < NR; q += NTH) {
    double2 acc = {0.0, 0.0};
    for (int c = 0; c < C; ++c) acc = cadd(acc, part[q * C + c]);
    dr[q] = acc;
  }
  __syncthreads();
  if (CH) {
    const int P = ax.NP, NT = ax.NT, NC = ND - 2 * P;
    for (int q = tid; q < ND; q += NTH) {
      double2 x;
      if (q < P) {
        x = dr[q];
      } else if (q >= P + NC) {
        x = dr[q - NC + NT];
      } else {
        const double* __restrict__ pr = ax.Pf + (int64_t)(q - P) * NT;
        x = double2{0.0, 0.0};
        for (int m = 0; m < NT; ++m) {
          const double wt = pr[m];
          const double2 y = dr[P + m];
          x.x += wt * y.x;
          x.y += wt * y.y;
        }
      }
      dm[q] = x;
    }
    __syncthreads();
  }
}

// inverse transform of the modes (v: the thread's ray, dm: LDS) into
// u[0..M) (LDS).  The E3 half writes u[t + TL m] last (after a barrier that
// follows the E1 half's writes of the same entries), so an E3 thread may read
// its own entries back without a barrier.  The dense rows are split between
// the halves.  With the interpolant (CH) dm shares u's LDS: u is written only
// after every read of dm.
template <int NU, bool CH>
__device__ __forceinline__ void rs_inverse(const double2 (&v)[RAY], const double2* dm, double2* fline,
                                           double2* fline2, const CFAxis& ax, const typename fs_tw<NU>::type& tw,
                                           int tid, double2* u) {
  constexpr int TL = NU / 8, NTH = 2 * TL;
  constexpr int EPT = 8;
  const int M = ax.M, NE = ax.NE, ND = ax.ND, NR = CH ? ax.NR : ND;
  const bool ray = tid >= TL;   // false: E3 (inverse FFT), true: E1 (forward FFT)
  const int t = ray ? tid - TL : tid;
  const double2* __restrict__ ipre = ray ? ax.ipre1 : ax.ipre3;
  const double2* __restrict__ ipost = ray ? ax.ipost1 : ax.ipost3;
  double2 w[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (m < RAY) {
      const double2 x = conj_if(!ray, cmul(ipre[min(e, NE - 1)], v[m < RAY ? m : 0]));
      w[m] = e < NE ? x : double2{0.0, 0.0};
    } else {
      w[m] = double2{0.0, 0.0};
    }
  }
  fft_regs<NU, TL, false>(w, t, ray ? fline2 : fline, tw);   // ends with a barrier: both lines free
  const double2* drow = dm;   // the rows' values: the dense modes, or (CH) the node values
  if constexpr (CH) {
    const int P = ax.NP, NT = ax.NT, NC = ND - 2 * P;
    const int C = NTH / NR > 1 ? NTH / NR : 1;
    const int L = (NC + C - 1) / C;
    double2* dv = fline2 + NR * C;
    for (int i = tid; i < NR * C; i += NTH) {
      const int r = i / C, c = i - r * C;
      double2 acc = {0.0, 0.0};
      if (r < P || r >= P + NT) {
        if (c == 0) acc = dm[r < P ? r : r - NT + NC];
      } else {
        const double2* __restrict__ pr = ax.Pi + (int64_t)(r - P) * NC;
        const int k1 = min(c * L + L, NC);
        for (int k = c * L; k < k1; ++k) acc = cadd(acc, cmul(pr[k], dm[P + k]));
      }
      fline2[i] = acc;
    }
    __syncthreads();
    for (int r = tid; r < NR; r += NTH) {
      double2 acc = {0.0, 0.0};
      for (int c = 0; c < C; ++c) acc = cadd(acc, fline2[r * C + c]);
      dv[r] = acc;
    }
    __syncthreads();   // dv complete, and every read of dm done: u may be written
    drow = dv;
  }
  // rows [0, h) summed by the E3 half, [h, NR) by the E1 half; the E1 half
  // writes its sums to u, the E3 half to the first exchange line (free once
  // the FFT is done; u shares no LDS with it or with drow, and with the
  // interpolant every read of dm is behind the barrier above), then the E3
  // half adds the two
  constexpr int DB = 8;
  const int h = NR / 2;
  const int q0 = ray ? h : 0, q1 = ray ? NR : h;
  double2* dst = ray ? u : fline;
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int e = t + TL * m;
    if (e < M) {
      double2 acc = cmul(ipost[e], conj_if(!ray, w[m]));
      for (int qb = q0; qb < q1; qb += DB) {
        double2 d[DB];
#pragma unroll
        for (int k = 0; k < DB; ++k) d[k] = ax.Dinv[(int64_t)min(qb + k, q1 - 1) * M + e];
#pragma unroll
        for (int k = 0; k < DB; ++k) {
          if (qb + k < q1) acc = cadd(acc, cmul(d[k], drow[qb + k]));
        }
      }
      dst[e] = acc;
    }
  }
  __syncthreads();
  if (!ray) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + TL * m;
      if (e < M) u[e] = cadd(u[e], fline[e]);
    }
  }
}

// LDS of a line kernel: dynamic f[M] | dm[ND] | first FFT exchange line |
// twiddles, and a static second exchange line that also holds the dense
// partials and, with the interpolant, the node values.  With the
// interpolant, f and dm share max(M, ND) entries.  At nu = 2048 with M = 256
// that is 79.9 KB with N_D = 36 direct rows and 79.4 KB with N_D <= 256
// through the interpolant: two workgroups per CU.
template <int NU>
size_t fs_lds_bytes(int M, int ND, bool ch) {
  const int line = ch ? (M > ND ? M : ND) : M + ND;
  return sizeof(double2) * (size_t)(line + lds_line_len(NU) + fs_tw<NU>::NC + fs_tw<NU>::NF);
}

// The per-mode step of the row pass for mode g = row_m + k; W is the mode of
// the forward transform (R_AM, R_UHACC).  T1[j-1] is the row's axis-0 factor
// of E^(j).  Returns the new B (R_UHACC: unused).  The history terms are
// unrolled, so a mode's loads are issued together.
__device__ __forceinline__ double2 fs_mode_update(const FSArgs& a, const double2 (&T1)[MAXH], int per, int k,
                                                  int64_t g, double2 W) {
  const int mode = a.mode;
  const double2* __restrict__ ph = a.ph;
  const double2* __restrict__ ring = a.ring;
  const int N1 = a.N1;
  const int nh = a.nh;
  const int64_t rs = a.ring_stride;
  // E^(j) = T1_j[k1] T2_j[k]
  auto E = [ph, per, N1, k, &T1](int j) { return cmul(T1[j - 1], ph[(j - 1) * per + N1 + k]); };
  double2 acc;
  if (mode == R_AM) {
    const double2 uh = cadd(a.Bm[g], fs_mul_mi(a.c0, W));
    acc = cmul(E(1), cadd(uh, fs_mul_mi(a.ch[1], W)));
#pragma unroll
    for (int j = 2; j < MAXH; ++j) {
      if (j <= nh) acc = cadd(acc, cmul(E(j), fs_mul_mi(a.ch[j], ring[a.slot_r[j] * rs + g])));
    }
    if (a.slot_w >= 0) a.ring[a.slot_w * rs + g] = W;
    a.Bm[g] = acc;
  } else if (mode == R_BINIT) {
    const double2 Wr = ring[a.slot_r[1] * rs + g];
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
#pragma unroll
    for (int j = 1; j < MAXH; ++j) {
      if (j <= nh) acc = cadd(acc, cmul(E(j), fs_mul_mi(a.ch[j], ring[a.slot_r[j] * rs + g])));
    }
    a.Bm[g] = acc;
  }
  return acc;
}

// ---------------------------------------------------------------- row pass

// Two workgroups per CU with the full register budget: with the history
// loads batched, spill traffic at a budget of 168 (three per CU) costs more
// than the latency a third wave per SIMD hides.
template <int NU, bool CH>
__global__ __launch_bounds__(NU / 8) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fs_row(FSArgs a) {
  constexpr int TL = NU / 8;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  __shared__ double2 fline2[lds_line_len(NU)];
  double2* part = fline2;
  const CFAxis& ax = a.ax2;
  const int M2 = ax.M, N2 = ax.N, NE = ax.NE, ND = ax.ND;
  double2* fin = fs_lds;                           // the row, then u (CH: the dense modes in between)
  double2* dm = CH ? fin : fin + M2;
  double2* fline = CH ? fin + (M2 > ND ? M2 : ND) : dm + ND;
  double2* tws = fline + lds_line_len(NU);
  const int t = threadIdx.x;
  const int k1 = blockIdx.x;
  const auto tw = stage_twiddles<NU>(ax, tws, t);   // read after the first barrier below
  const int mode = a.mode;
  const int per = a.N1 + a.N2;
  const int64_t row_m = (int64_t)k1 * N2;   // mode row
  const int64_t row_p = (int64_t)k1 * M2;   // tile row (physical axis 1)

  double2 v3[RAY], v1[RAY];
  const bool need_fwd = (mode == R_AM || mode == R_FWD || mode == R_UHACC);
  // Adams step with the full history: B of the thread's ray modes and the
  // first history batch (term j = 2 on the E3 ray) are loaded before the
  // forward transform, so their latency overlaps it
  const bool pre = mode == R_AM && a.nh == MAXH - 1;
  const bool pw = pre && a.pf_pow;
  double2 Bp3[RAY], Bp1[RAY], w0[RAY], pf0[RAY];
  if (pre) {
    const double2* __restrict__ r2 = a.ring + a.slot_r[2] * a.ring_stride + row_m;
    const double2* __restrict__ p2 = a.ph + (a.N1 + a.N2) + a.N1;
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int ec = min(t + TL * m, NE - 1);
      Bp3[m] = a.Bm[row_m + N2 - NE + ec];
      Bp1[m] = a.Bm[row_m + NE - 1 - ec];
      w0[m] = r2[N2 - NE + ec];
      if (!pw) pf0[m] = p2[N2 - NE + ec];
    }
  }
  if (need_fwd) {
    for (int j = t; j < M2; j += TL) fin[j] = a.src[row_p + j];
    __syncthreads();
    cf_forward<NU, CH>(fin, v3, v1, dm, part, fline, fline2, ax, tw, t);
  } else {
#pragma unroll
    for (int m = 0; m < RAY; ++m) v3[m] = v1[m] = double2{0.0, 0.0};
  }
  if (mode == R_FWD) {
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int e = t + TL * m;
      if (e < NE) {
        a.fdst[row_m + N2 - NE + e] = v3[m];
        a.fdst[row_m + NE - 1 - e] = v1[m];
      }
    }
    for (int q = t; q < ND; q += TL) a.fdst[row_m + NE + q] = dm[q];
    return;
  }
  // the row's axis-0 factors of E^(j) (uniform over the workgroup)
  double2 T1[MAXH];
  const int nj = (mode == R_AM || mode == R_FORM) ? a.nh : (mode == R_BINIT ? 1 : 0);
#pragma unroll
  for (int j = 1; j <= MAXH; ++j) T1[j - 1] = j <= nj ? a.ph[(j - 1) * per + k1] : double2{0.0, 0.0};
  if (mode == R_AM) {
    // The ray modes' Adams step, history term by history term over all of
    // the thread's modes.  The new history entry What_n goes to its ring slot
    // first (no history term reads that slot); B is stored after the last
    // load.  Lanes past the end of a ray load their ray's last mode and store
    // nothing.
    const double2* __restrict__ ph = a.ph;
    const double2* __restrict__ ring = a.ring;
    const int64_t rs = a.ring_stride;
    const int nh = a.nh;
    const int N1 = a.N1;
    int k3[RAY], k1r[RAY];
    double2 acc3[RAY], acc1[RAY];
    double2 P3[RAY], P1[RAY];   // the last axis' factors of E^(1)
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int ec = min(t + TL * m, NE - 1);
      k3[m] = N2 - NE + ec;
      k1r[m] = NE - 1 - ec;
      const double2 B3 = pre ? Bp3[m] : a.Bm[row_m + k3[m]], B1 = pre ? Bp1[m] : a.Bm[row_m + k1r[m]];
      P3[m] = ph[N1 + k3[m]];
      P1[m] = ph[N1 + k1r[m]];
      const double2 E3 = cmul(T1[0], P3[m]), E1 = cmul(T1[0], P1[m]);
      // E^(1) (uhat - i dt mu_1 W),  uhat = B - i dt mu_0 W
      acc3[m] = cmul(E3, cadd(cadd(B3, fs_mul_mi(a.c0, v3[m])), fs_mul_mi(a.ch[1], v3[m])));
      acc1[m] = cmul(E1, cadd(cadd(B1, fs_mul_mi(a.c0, v1[m])), fs_mul_mi(a.ch[1], v1[m])));
      if (a.slot_w >= 0 && t + TL * m < NE) {
        a.ring[a.slot_w * rs + row_m + k3[m]] = v3[m];
        a.ring[a.slot_w * rs + row_m + k1r[m]] = v1[m];
      }
    }
    // history terms j >= 2 in batches b = (j, ray): the history modes and
    // phase factors of batch b+1 are loaded while batch b is summed
    double2 w[2][RAY], pf[2][RAY];
    auto load = [&](int b) {
      const int j = 2 + (b >> 1);
      const double2* __restrict__ rj = ring + a.slot_r[j] * rs + row_m;
      const double2* __restrict__ pj = ph + (j - 1) * per + N1;
#pragma unroll
      for (int m = 0; m < RAY; ++m) {
        const int kk = (b & 1) ? k1r[m] : k3[m];
        w[b & 1][m] = rj[kk];
        pf[b & 1][m] = pj[kk];
      }
    };
    auto use = [&](int b) {
      const int j = 2 + (b >> 1);
#pragma unroll
      for (int m = 0; m < RAY; ++m) {
        const double2 x = fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], pf[b & 1][m]), w[b & 1][m]));
        if (b & 1) acc1[m] = cadd(acc1[m], x);
        else acc3[m] = cadd(acc3[m], x);
      }
    };
    if (pw) {
      // the full history with the last axis' factors as powers of E^(1)'s
      // (exp(-i zeta^2 j tau) = exp(-i zeta^2 tau)^j): only the history
      // modes are loaded, batch b + 1 while batch b is summed
      constexpr int NB = 2 * (MAXH - 2);
      double2 R3[RAY], R1[RAY];
#pragma unroll
      for (int m = 0; m < RAY; ++m) {
        w[0][m] = w0[m];
        R3[m] = P3[m];
        R1[m] = P1[m];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) {
          const int jn = 2 + ((b + 1) >> 1);
          const double2* __restrict__ rj = ring + a.slot_r[jn] * rs + row_m;
#pragma unroll
          for (int m = 0; m < RAY; ++m) w[(b + 1) & 1][m] = rj[((b + 1) & 1) ? k1r[m] : k3[m]];
        }
        __builtin_amdgcn_sched_barrier(0);
        const int j = 2 + (b >> 1);
#pragma unroll
        for (int m = 0; m < RAY; ++m) {
          if (b & 1) {
            R1[m] = cmul(R1[m], P1[m]);
            acc1[m] = cadd(acc1[m], fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], R1[m]), w[1][m])));
          } else {
            R3[m] = cmul(R3[m], P3[m]);
            acc3[m] = cadd(acc3[m], fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], R3[m]), w[0][m])));
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else if (nh == MAXH - 1) {   // the full order-8 history: straight-line, software-pipelined
      constexpr int NB = 2 * (MAXH - 2);
#pragma unroll
      for (int m = 0; m < RAY; ++m) {   // batch 0, loaded before the forward transform
        w[0][m] = w0[m];
        pf[0][m] = pf0[m];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) load(b + 1);
        __builtin_amdgcn_sched_barrier(0);
        use(b);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int b = 0; b < 2 * (MAXH - 2); ++b) {
        if (2 + (b >> 1) <= nh) {
          load(b);
          __builtin_amdgcn_sched_barrier(0);
          use(b);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const bool live = t + TL * m < NE;
      if (live) {
        a.Bm[row_m + k3[m]] = acc3[m];
        a.Bm[row_m + k1r[m]] = acc1[m];
      }
      v3[m] = live ? acc3[m] : double2{0.0, 0.0};
      v1[m] = live ? acc1[m] : double2{0.0, 0.0};
    }
  } else {
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int e = t + TL * m;
      if (e < NE) {
        v3[m] = fs_mode_update(a, T1, per, N2 - NE + e, row_m + N2 - NE + e, v3[m]);
        v1[m] = fs_mode_update(a, T1, per, NE - 1 - e, row_m + NE - 1 - e, v1[m]);
      }
    }
  }
  if (mode == R_AM && a.nh == MAXH - 1) {
    // dense modes, one per thread: every load of the mode issued together
    const double2* __restrict__ ph = a.ph;
    const double2* __restrict__ ring = a.ring;
    const int64_t rs = a.ring_stride;
    const int N1 = a.N1;
    for (int q = t; q < ND; q += TL) {
      const int k = NE + q;
      const int64_t g = row_m + k;
      const double2 W = dm[q];
      double2 pf[MAXH - 1], wh[MAXH - 2];
      const double2 B = a.Bm[g];
#pragma unroll
      for (int j = 1; j < MAXH; ++j) pf[j - 1] = ph[(j - 1) * per + N1 + k];
#pragma unroll
      for (int j = 2; j < MAXH; ++j) wh[j - 2] = ring[a.slot_r[j] * rs + g];
      __builtin_amdgcn_sched_barrier(0);
      double2 acc = cmul(cmul(T1[0], pf[0]), cadd(cadd(B, fs_mul_mi(a.c0, W)), fs_mul_mi(a.ch[1], W)));
#pragma unroll
      for (int j = 2; j < MAXH; ++j) acc = cadd(acc, fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], pf[j - 1]), wh[j - 2])));
      if (a.slot_w >= 0) a.ring[a.slot_w * rs + g] = W;
      a.Bm[g] = acc;
      dm[q] = acc;
    }
  } else {
    for (int q = t; q < ND; q += TL)
      dm[q] = fs_mode_update(a, T1, per, NE + q, row_m + NE + q, need_fwd ? dm[q] : double2{0.0, 0.0});
  }
  if (mode == R_UHACC) return;
  __syncthreads();
  cf_inverse<NU, CH>(v3, v1, dm, fline, fline2, ax, tw, t, fin);   // the forward input is no longer needed
  for (int e = t; e < M2; e += TL) a.dst[row_p + e] = fin[e];
}

// ------------------------------------------------------------- column pass

// Columns sharing a 128-byte line of the tile (8 complex128) are dealt to the
// same XCD (workgroups b, b + 8, ...), so their strided accesses meet in one L2.
__device__ __forceinline__ int fs_col_of(int b, int nb) {
  if (nb % 64) return b;
  const int x = b & 7, s = b >> 3;
  return 8 * ((s / 8) * 8 + x) + (s % 8);
}

// ------------------------------------------------ ray-split row and column passes

// The row pass with 2 TL threads per row: each thread carries RAY modes of
// one ray (E3 for threads [0, TL), E1 for [TL, 2 TL)) through the forward
// transform, the recurrence and the inverse transform.
template <int NU, bool CH>
__global__ __launch_bounds__(NU / 4) void k_fs_row_rs(FSArgs a) {
  constexpr int TL = NU / 8, NTH = 2 * TL;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  __shared__ double2 fline2[lds_line_len(NU)];
  double2* part = fline2;
  const CFAxis& ax = a.ax2;
  const int M2 = ax.M, N2 = ax.N, NE = ax.NE, ND = ax.ND;
  double2* fin = fs_lds;
  double2* dm = CH ? fin : fin + M2;
  double2* fline = CH ? fin + (M2 > ND ? M2 : ND) : dm + ND;
  double2* tws = fline + lds_line_len(NU);
  const int tid = threadIdx.x;
  const bool ray = tid >= TL;
  const int t = ray ? tid - TL : tid;
  const int k1 = blockIdx.x;
  const auto tw = stage_twiddles_n<NU>(ax, tws, tid, NTH);   // read after the first barrier below
  const int mode = a.mode;
  const int per = a.N1 + a.N2;
  const int64_t row_m = (int64_t)k1 * N2;
  const int64_t row_p = (int64_t)k1 * M2;
  // the thread's modes: E3 mode N2 - N_E + e, E1 mode N_E - 1 - e (lanes past
  // the end of the ray take its last mode and store nothing)
  int kk[RAY];
#pragma unroll
  for (int m = 0; m < RAY; ++m) {
    const int ec = min(t + TL * m, NE - 1);
    kk[m] = ray ? NE - 1 - ec : N2 - NE + ec;
  }

  double2 v[RAY];
  const bool need_fwd = (mode == R_AM || mode == R_FWD || mode == R_UHACC);
  if (need_fwd) {
    for (int j = tid; j < M2; j += NTH) fin[j] = a.src[row_p + j];
    __syncthreads();
    rs_forward<NU, CH>(fin, v, dm, part, fline, fline2, ax, tw, tid);
  } else {
#pragma unroll
    for (int m = 0; m < RAY; ++m) v[m] = double2{0.0, 0.0};
  }
  if (mode == R_FWD) {
#pragma unroll
    for (int m = 0; m < RAY; ++m)
      if (t + TL * m < NE) a.fdst[row_m + kk[m]] = v[m];
    for (int q = tid; q < ND; q += NTH) a.fdst[row_m + NE + q] = dm[q];
    return;
  }
  double2 T1[MAXH];
  const int nj = (mode == R_AM || mode == R_FORM) ? a.nh : (mode == R_BINIT ? 1 : 0);
#pragma unroll
  for (int j = 1; j <= MAXH; ++j) T1[j - 1] = j <= nj ? a.ph[(j - 1) * per + k1] : double2{0.0, 0.0};
  if (mode == R_AM) {
    const double2* __restrict__ ph = a.ph;
    const double2* __restrict__ ring = a.ring;
    const int64_t rs = a.ring_stride;
    const int nh = a.nh;
    const int N1 = a.N1;
    const bool pw = a.pf_pow != 0;   // the last axis' factors as powers of E^(1)'s
    double2 acc[RAY], P[RAY], R[RAY];
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const double2 B = a.Bm[row_m + kk[m]];
      P[m] = ph[N1 + kk[m]];
      R[m] = P[m];
      const double2 E = cmul(T1[0], P[m]);
      acc[m] = cmul(E, cadd(cadd(B, fs_mul_mi(a.c0, v[m])), fs_mul_mi(a.ch[1], v[m])));
      if (a.slot_w >= 0 && t + TL * m < NE) a.ring[a.slot_w * rs + row_m + kk[m]] = v[m];
    }
    // history terms j >= 2, one term at a time (the occupancy hides the
    // loads' latency)
#pragma unroll
    for (int j = 2; j < MAXH; ++j) {
      if (j <= nh) {
        const double2* __restrict__ rj = ring + a.slot_r[j] * rs + row_m;
        const double2* __restrict__ pj = ph + (j - 1) * per + N1;
        double2 w[RAY], pf[RAY];
#pragma unroll
        for (int m = 0; m < RAY; ++m) {
          w[m] = rj[kk[m]];
          if (pw) {
            R[m] = cmul(R[m], P[m]);
            pf[m] = R[m];
          } else {
            pf[m] = pj[kk[m]];
          }
        }
#pragma unroll
        for (int m = 0; m < RAY; ++m) acc[m] = cadd(acc[m], fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], pf[m]), w[m])));
      }
    }
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const bool live = t + TL * m < NE;
      if (live) a.Bm[row_m + kk[m]] = acc[m];
      v[m] = live ? acc[m] : double2{0.0, 0.0};
    }
  } else {
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      if (t + TL * m < NE) v[m] = fs_mode_update(a, T1, per, kk[m], row_m + kk[m], v[m]);
    }
  }
  if (mode == R_AM && a.nh == MAXH - 1) {
    const double2* __restrict__ ph = a.ph;
    const double2* __restrict__ ring = a.ring;
    const int64_t rs = a.ring_stride;
    const int N1 = a.N1;
    for (int q = tid; q < ND; q += NTH) {
      const int k = NE + q;
      const int64_t g = row_m + k;
      const double2 W = dm[q];
      double2 pfq[MAXH - 1], wh[MAXH - 2];
      const double2 B = a.Bm[g];
#pragma unroll
      for (int j = 1; j < MAXH; ++j) pfq[j - 1] = ph[(j - 1) * per + N1 + k];
#pragma unroll
      for (int j = 2; j < MAXH; ++j) wh[j - 2] = ring[a.slot_r[j] * rs + g];
      __builtin_amdgcn_sched_barrier(0);
      double2 acc = cmul(cmul(T1[0], pfq[0]), cadd(cadd(B, fs_mul_mi(a.c0, W)), fs_mul_mi(a.ch[1], W)));
#pragma unroll
      for (int j = 2; j < MAXH; ++j) acc = cadd(acc, fs_mul_mi(a.ch[j], cmul(cmul(T1[j - 1], pfq[j - 1]), wh[j - 2])));
      if (a.slot_w >= 0) a.ring[a.slot_w * rs + g] = W;
      a.Bm[g] = acc;
      dm[q] = acc;
    }
  } else {
    for (int q = tid; q < ND; q += NTH)
      dm[q] = fs_mode_update(a, T1, per, NE + q, row_m + NE + q, need_fwd ? dm[q] : double2{0.0, 0.0});
  }
  if (mode == R_UHACC) return;
  __syncthreads();
  rs_inverse<NU, CH>(v, dm, fline, fline2, ax, tw, tid, fin);
  if (!ray) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = t + TL * m;
      if (e < M2) a.dst[row_p + e] = fin[e];
    }
  }
}

// The column pass with 2 TL threads per column (ray halves as in the row pass);
// the columns are the ncol points of the other axes (x2, or (x1, x2) in 3D).
template <int NU, bool CH>
__global__ __launch_bounds__(NU / 4) void k_fs_col_rs(FSArgs a) {
  constexpr int TL = NU / 8, NTH = 2 * TL;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  __shared__ double2 fline2[lds_line_len(NU)];
  double2* part = fline2;
  const CFAxis& ax = a.ax1;
  const int M1 = ax.M, N1 = ax.N, NE = ax.NE, ND = ax.ND;
  const int64_t M2 = a.ncol;   // columns; the stride along axis 0
  double2* fin = fs_lds;
  double2* dm = CH ? fin : fin + M1;
  double2* fline = CH ? fin + (M1 > ND ? M1 : ND) : dm + ND;
  double2* tws = fline + lds_line_len(NU);
  const int tid = threadIdx.x;
  const bool ray = tid >= TL;
  const int t = ray ? tid - TL : tid;
  const int y = fs_col_of(blockIdx.x, gridDim.x);
  const auto tw = stage_twiddles_n<NU>(ax, tws, tid, NTH);
  const int mode = a.mode;

  if (a.req.nj > 0) build_phase_table_fs(a, NTH);
  double2 v[RAY];
  if (mode == C_SOLVE) {
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int e = t + TL * m;
      const int k = ray ? NE - 1 - e : N1 - NE + e;
      v[m] = e < NE ? a.src[(int64_t)k * M2 + y] : double2{0.0, 0.0};
    }
    for (int q = tid; q < ND; q += NTH) dm[q] = a.src[(int64_t)(NE + q) * M2 + y];
    __syncthreads();
    rs_inverse<NU, CH>(v, dm, fline, fline2, ax, tw, tid, fin);
    if (!ray) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = t + TL * m;
        if (e < M1) {
          const double2 wv = fin[e];
          const int64_t g = (int64_t)e * M2 + y;
          double Vs = 0.0;
          for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + g];
          const double q = a.csolve * Vs;
          const double inv = 1.0 / (1.0 + q * q);
          const double2 u = double2{(wv.x + q * wv.y) * inv, (wv.y - q * wv.x) * inv};
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
    }
  } else {  // C_FWD
    for (int e = tid; e < M1; e += NTH) {
      const int64_t g = (int64_t)e * M2 + y;
      double Vs = 0.0;
      for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + g];
      const double2 u = a.usrc[g];
      const double cr = a.alpha_re + a.beta_re * Vs, ci = a.alpha_im + a.beta_im * Vs;
      fin[e] = double2{cr * u.x - ci * u.y, cr * u.y + ci * u.x};
    }
  }
  __syncthreads();
  rs_forward<NU, CH>(fin, v, dm, part, fline, fline2, ax, tw, tid);
#pragma unroll
  for (int m = 0; m < RAY; ++m) {
    const int e = t + TL * m;
    if (e < NE) a.dst[(int64_t)(ray ? NE - 1 - e : N1 - NE + e) * M2 + y] = v[m];
  }
  for (int q = tid; q < ND; q += NTH) a.dst[(int64_t)(NE + q) * M2 + y] = dm[q];
}

// Middle-axis line transform of a 3D problem (ray halves as above): line
// (k0, x2) of the N0 x Nm x M2 mode array and of the N0 x Mm x M2 grid array,
// stride M2.  INV: modes to grid points (before the column pass), else grid
// points to modes (after it).
template <int NU, bool CH, bool INV>
__global__ __launch_bounds__(NU / 4) void k_fs_mid_rs(FSArgs a) {
  constexpr int TL = NU / 8, NTH = 2 * TL;
  HIP_DYNAMIC_SHARED(double2, fs_lds)
  __shared__ double2 fline2[lds_line_len(NU)];
  double2* part = fline2;
  const CFAxis& ax = a.axm;
  const int Mm = ax.M, Nm = ax.N, NE = ax.NE, ND = ax.ND;
  const int M2 = a.ax2.M;
  double2* fin = fs_lds;
  double2* dm = CH ? fin : fin + Mm;
  double2* fline = CH ? fin + (Mm > ND ? Mm : ND) : dm + ND;
  double2* tws = fline + lds_line_len(NU);
  const int tid = threadIdx.x;
  const bool ray = tid >= TL;
  const int t = ray ? tid - TL : tid;
  // lines sharing 128-byte lines of memory (consecutive x2) on one XCD
  const int line = fs_col_of(blockIdx.x, gridDim.x);
  const int k0 = line / M2, x2 = line - k0 * M2;
  const int64_t mbase = (int64_t)k0 * Nm * M2 + x2;   // mode k of the line at mbase + k M2
  const int64_t gbase = (int64_t)k0 * Mm * M2 + x2;   // point e of the line at gbase + e M2
  const auto tw = stage_twiddles_n<NU>(ax, tws, tid, NTH);
  double2 v[RAY];
  if constexpr (INV) {
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int e = t + TL * m;
      const int k = ray ? NE - 1 - e : Nm - NE + e;
      v[m] = e < NE ? a.src[mbase + (int64_t)k * M2] : double2{0.0, 0.0};
    }
    for (int q = tid; q < ND; q += NTH) dm[q] = a.src[mbase + (int64_t)(NE + q) * M2];
    __syncthreads();
    rs_inverse<NU, CH>(v, dm, fline, fline2, ax, tw, tid, fin);
    if (!ray) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int e = t + TL * m;
        if (e < Mm) a.dst[gbase + (int64_t)e * M2] = fin[e];
      }
    }
  } else {
    for (int e = tid; e < Mm; e += NTH) fin[e] = a.src[gbase + (int64_t)e * M2];
    __syncthreads();
    rs_forward<NU, CH>(fin, v, dm, part, fline, fline2, ax, tw, tid);
#pragma unroll
    for (int m = 0; m < RAY; ++m) {
      const int e = t + TL * m;
      if (e < NE) a.dst[mbase + (int64_t)(ray ? NE - 1 - e : Nm - NE + e) * M2] = v[m];
    }
    for (int q = tid; q < ND; q += NTH) a.dst[mbase + (int64_t)(NE + q) * M2] = dm[q];
  }
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

size_t fs_line_lds_bytes(int nu, int M, int ND, bool ch) {
  switch (nu) {
#define X(n) case n: return fs_lds_bytes<n>(M, ND, ch);
    TDSE_FS_NU(X)
#undef X
    default:
      return 0;
  }
}

// The row pass of a 1D problem is a single workgroup: it takes the ray-split
// kernel (twice the threads on the one line).  So do the many short rows of
// nu <= 512, whose workgroups are small enough that LDS does not cap the
// occupancy.  The rows of nu >= 1024 keep the two-ray kernel: at 80 KB of LDS
// per workgroup, two of them per CU keep more loads in flight.
hipError_t launch_fs_row(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.N1 == 1 || nu <= 512) {
    switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    if (a.ax2.NT)                                                                         \
      TDSE_FS_LAUNCH_SH((k_fs_row_rs<n, true>), dim3(a.N1), dim3(n / 4), fs_lds_bytes<n>(a.ax2.M, a.ax2.ND, a.ax2.NT != 0), s, e0, e1, a); \
    else                                                                                  \
      TDSE_FS_LAUNCH_SH((k_fs_row_rs<n, false>), dim3(a.N1), dim3(n / 4), fs_lds_bytes<n>(a.ax2.M, a.ax2.ND, a.ax2.NT != 0), s, e0, e1, a); \
    break;
      TDSE_FS_NU(X)
#undef X
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    if (a.ax2.NT)                                                                         \
      TDSE_FS_LAUNCH_SH((k_fs_row<n, true>), dim3(a.N1), dim3(n / 8), fs_lds_bytes<n>(a.ax2.M, a.ax2.ND, a.ax2.NT != 0), s, e0, e1, a); \
    else                                                                                  \
      TDSE_FS_LAUNCH_SH((k_fs_row<n, false>), dim3(a.N1), dim3(n / 8), fs_lds_bytes<n>(a.ax2.M, a.ax2.ND, a.ax2.NT != 0), s, e0, e1, a); \
    break;
    TDSE_FS_NU(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_col(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nu == 0) {   // 1D: pointwise, with enough workgroups for one phase entry per thread
    const int64_t entries = (int64_t)a.req.nj * (a.N1 + a.N2);
    const int64_t blocks = std::max<int64_t>((a.ax2.M + 255) / 256, std::min<int64_t>((entries + 255) / 256, 1024));
    TDSE_FS_LAUNCH(k_fs_point, dim3((unsigned)blocks), dim3(256), s, e0, e1, a);
    return hipGetLastError();
  }
  switch (nu) {
#define X(n)                                                                              \
  case n:                                                                                 \
    if (a.ax1.NT)                                                                         \
      TDSE_FS_LAUNCH_SH((k_fs_col_rs<n, true>), dim3((unsigned)a.ncol), dim3(n / 4), fs_lds_bytes<n>(a.ax1.M, a.ax1.ND, a.ax1.NT != 0), s, e0, e1, a); \
    else                                                                                  \
      TDSE_FS_LAUNCH_SH((k_fs_col_rs<n, false>), dim3((unsigned)a.ncol), dim3(n / 4), fs_lds_bytes<n>(a.ax1.M, a.ax1.ND, a.ax1.NT != 0), s, e0, e1, a); \
    break;
    TDSE_FS_NU(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_mid(int nu, bool inverse, const FSArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 g((unsigned)((int64_t)a.ax1.N * a.ax2.M));
  const size_t lds_b = fs_line_lds_bytes(nu, a.axm.M, a.axm.ND, a.axm.NT != 0);
  switch (nu) {
#define X(n)                                                                                                  \
  case n:                                                                                                     \
    if (a.axm.NT) {                                                                                           \
      if (inverse) TDSE_FS_LAUNCH_SH((k_fs_mid_rs<n, true, true>), g, dim3(n / 4), lds_b, s, e0, e1, a);       \
      else TDSE_FS_LAUNCH_SH((k_fs_mid_rs<n, true, false>), g, dim3(n / 4), lds_b, s, e0, e1, a);              \
    } else {                                                                                                  \
      if (inverse) TDSE_FS_LAUNCH_SH((k_fs_mid_rs<n, false, true>), g, dim3(n / 4), lds_b, s, e0, e1, a);      \
      else TDSE_FS_LAUNCH_SH((k_fs_mid_rs<n, false, false>), g, dim3(n / 4), lds_b, s, e0, e1, a);             \
    }                                                                                                         \
    break;
    TDSE_FS_NU(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fs_phase(const FSArgs& a, hipStream_t s) {
  const int64_t entries = (int64_t)a.req.nj * (a.N1 + a.N2);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((entries + 255) / 256, 1024));
  hipLaunchKernelGGL(k_fs_phase, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tdse
