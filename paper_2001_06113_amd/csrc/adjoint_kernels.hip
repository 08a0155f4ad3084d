// HIP kernels of the reverse-mode derivative (adjoint) of the periodic
// scheme, FP64, gfx950.
//
// For a fixed vector potential the scheme (eq. (uadamsk) with the
// Richardson start-up of eq. (utrapk)) is linear in the state, and A enters
// only through the phase factors of Lemma 1,
//   E = exp(-i |k|^2 tau + i k . dphi),  dphi = phi(t_b) - phi(t_a).
// The reverse sweep applies the conjugate transpose of each operation; the
// transforms and the conjugated implicit solve reuse the forward passes, and
// these kernels do the mode-wise parts:
//   k_adj_am     adjoint of one implicit Adams step in mode space: the
//                adjoint beta_n of B_n, the adjoint omega_{n-1} of What_{n-1},
//                and per-workgroup partial sums of dJ/d(dphi) of the phase
//                factors of step n+1;
//   k_adj_sub    the phase factor of an order-2 sub-step (forward, or adjoint
//                with its dJ/d(dphi) partial sums);
//   k_adj_point  diagonal factors (alpha + beta V) or 1/(alpha + beta V) on the grid;
//   k_adj_axpy, k_adj_copy2, k_adj_phase, k_adj_reduce, k_adj_to_A  (helpers).
#include <hip/hip_runtime.h>

#include "periodic_body.h"

namespace tdse {

__device__ __forceinline__ double2 conjd(double2 z) { return double2{z.x, -z.y}; }
// i z
__device__ __forceinline__ double2 mul_i(double2 z) { return double2{-z.y, z.x}; }

// E at (k1 index, k2 index) from entry e of the per-axis table
__device__ __forceinline__ double2 adj_phase(const double2* ph, int per, int M1, int e, int i1, int i2) {
  return cmul(ph[e * per + i1], ph[e * per + M1 + i2]);
}

// Per-axis factors exp(i(-k^2 tau + k dphi_a)) of up to ADJ_PH entries.
__global__ __launch_bounds__(256) void k_adj_phase(AdjPhase q) {
  const int per = q.M1 + q.M2;
  const int total = q.nj * per;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += gridDim.x * 256) {
    const int e = idx / per;
    const int kk = idx - e * per;
    double k, dphi;
    if (kk < q.M1) {
      k = (double)signed_mode(kk, q.M1);
      dphi = q.dphi1[e];
    } else {
      k = (double)signed_mode(kk - q.M1, q.M2);
      dphi = q.dphi2[e];
    }
    double s, c;
    sincos(-(k * k) * q.tau[e] + k * dphi, &s, &c);
    q.ph[idx] = double2{c, s};
  }
}

// Block sum of NV values per thread into part[v * nblk + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_partials(double (&val)[NV], double* part, int nblk) {
  __shared__ double buf[NV][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NV; ++v) buf[v][t] = val[v];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int v = 0; v < NV; ++v) buf[v][t] += buf[v][t + s];
    }
    __syncthreads();
  }
  if (t < NV) part[(int64_t)t * nblk + blockIdx.x] = buf[t][0];
}

__global__ __launch_bounds__(256) void k_adj_am(AdjAm a) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = g < a.P;
  const int per = a.M1 + a.M2;
  const int H = a.H;
  double val[2 * MAXH];
#pragma unroll
  for (int v = 0; v < 2 * MAXH; ++v) val[v] = 0.0;
  if (live) {
    const int i1 = (int)(g / a.M2), i2 = (int)(g - (int64_t)i1 * a.M2);
    const double k1 = (double)signed_mode(i1, a.M1), k2 = (double)signed_mode(i2, a.M2);
    const double2 b1 = a.slot_b1 >= 0 ? a.beta[a.slot_b1 * a.P + g] : double2{0.0, 0.0};
    double2 bn = double2{0.0, 0.0};
    if (a.beta_mode == 1) {
      // beta_n = conj(E^(1)_{n+1}) beta_{n+1} + G_n^H omega_n
      bn = cadd(cmul(conjd(adj_phase(a.ph, per, a.M1, 0, i1, i2)), b1), a.Z[g]);
      a.beta[a.slot_bn * a.P + g] = bn;
    } else if (a.beta_mode == 2) {
      bn = a.beta[a.slot_bn * a.P + g];
    }
    if (a.has_grad) {
      // step n+1: B_{n+1} = sum_j E^(j)_{n+1} x_j,
      //   x_1 = B_n - i c_1 What_n,  x_j = -i c_j What_{n+1-j};
      // dJ/dtheta = Re(conj(beta_{n+1}) i E x), weighted by k_a
      for (int j = 1; j <= H; ++j) {
        const double2 W = a.Wx[j][g];
        double2 x = double2{a.cx[j] * W.y, -a.cx[j] * W.x};   // -i c_j W
        if (j == 1) x = cadd(x, a.Bn[g]);
        const double2 Ex = cmul(adj_phase(a.ph, per, a.M1, j - 1, i1, i2), x);
        const double2 cb = conjd(b1);
        const double term = -(cb.x * Ex.y + cb.y * Ex.x);   // Re(conj(b) i E x)
        val[2 * (j - 1)] = k1 * term;
        val[2 * (j - 1) + 1] = k2 * term;
      }
    }
    if (a.omega) {
      // omega_{n-1} = sum_j i w_j conj(E^(j)_{n-1+j}) beta_{n-1+j}
      double2 om = double2{0.0, 0.0};
      for (int j = 1; j <= H; ++j) {
        if (a.wj[j] == 0.0) continue;
        double2 b;
        if (j == 1) b = bn;
        else if (a.slot_bj[j] >= 0) b = a.beta[a.slot_bj[j] * a.P + g];
        else continue;
        const double2 t = cmul(conjd(adj_phase(a.ph, per, a.M1, H + j - 1, i1, i2)), b);
        om = cadd(om, double2{-a.wj[j] * t.y, a.wj[j] * t.x});
      }
      a.omega[g] = om;
    }
  }
  if (a.has_grad) block_partials<2 * MAXH>(val, a.part, a.nblk);
}

// Order-2 sub-step phase, entry 0 of the table: mode 1: y = E g; mode 0:
// partial sums of Re(conj(y) i E g) k_a, then y = conj(E) y; mode 2:
// y = conj(E) y only.
__global__ __launch_bounds__(256) void k_adj_sub(AdjSub a) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int per = a.M1 + a.M2;
  double val[2] = {0.0, 0.0};
  if (g < a.P) {
    const int i1 = (int)(g / a.M2), i2 = (int)(g - (int64_t)i1 * a.M2);
    const double2 E = adj_phase(a.ph, per, a.M1, 0, i1, i2);
    if (a.mode == 1) {
      a.y[g] = cmul(E, a.g[g]);
    } else {
      const double2 y = a.y[g];
      if (a.mode == 0) {
        const double2 Ex = cmul(E, a.g[g]);
        const double term = -(y.x * Ex.y - y.y * Ex.x);    // Re(conj(y) i E g)
        val[0] = (double)signed_mode(i1, a.M1) * term;
        val[1] = (double)signed_mode(i2, a.M2) * term;
      }
      a.y[g] = cmul(conjd(E), y);
    }
  }
  if (a.mode == 0) block_partials<2>(val, a.part, a.nblk);
}

// out = s (alpha + beta V(t)) in   or   out = s in / (alpha + beta V(t));  optionally out +=
__global__ __launch_bounds__(256) void k_adj_point(AdjPoint a) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= a.P) return;
  double Vs = 0.0;
  for (int r = 0; r < a.nV; ++r) Vs += a.fV[r] * a.V[r * a.vstride + g];
  const double2 f = double2{a.ar + a.br * Vs, a.ai + a.bi * Vs};
  const double2 x = a.in[g];
  double2 y;
  if (a.divide) {
    const double den = f.x * f.x + f.y * f.y;
    y = double2{(x.x * f.x + x.y * f.y) / den, (x.y * f.x - x.x * f.y) / den};
  } else {
    y = cmul(f, x);
  }
  y.x *= a.s;
  y.y *= a.s;
  if (a.accumulate) y = cadd(y, a.out[g]);
  a.out[g] = y;
}

// out = x + c y (complex c)
__global__ __launch_bounds__(256) void k_adj_axpy(int64_t P, const double2* x, const double2* y, double cr, double ci,
                                                  double2* out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= P) return;
  out[g] = cadd(x[g], cmul(double2{cr, ci}, y[g]));
}

// two copies of P entries in one launch: workgroups [0, nb) copy src0 into
// dst0, the next nb copy src1 into dst1
__global__ __launch_bounds__(256) void k_adj_copy2(int64_t P, int nblk, double2* dst0, const double2* src0,
                                                   double2* dst1, const double2* src1) {
  const bool second = (int)blockIdx.x >= nblk;
  const int64_t g = (int64_t)(second ? blockIdx.x - nblk : blockIdx.x) * 256 + threadIdx.x;
  if (g >= P) return;
  if (second) dst1[g] = src1[g];
  else dst0[g] = src0[g];
}

// red[r] = sum_b part[r * nblk + b], one workgroup per row
__global__ __launch_bounds__(256) void k_adj_reduce(const double* part, double* red, int nblk) {
  __shared__ double buf[256];
  const int r = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nblk; b += 256) s += part[(int64_t)r * nblk + b];
  buf[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) buf[t] += buf[t + w];
    __syncthreads();
  }
  if (t == 0) red[r] = buf[0];
}

// out[o] = sum_{e in [rowptr[o], rowptr[o+1])} wt[e] red[src[e]]
__global__ __launch_bounds__(256) void k_adj_to_A(const double* red, const int* rowptr, const int* src, const double* wt,
                                                  double* out, int nout) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int e = rowptr[o]; e < rowptr[o + 1]; ++e) s += wt[e] * red[src[e]];
  out[o] = s;
}

static int nb(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_adj_phase(const AdjPhase& q, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_phase, dim3(std::max(1, nb((int64_t)q.nj * (q.M1 + q.M2)))), dim3(256), 0, s, q);
  return hipGetLastError();
}
hipError_t launch_adj_am(const AdjAm& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_am, dim3(a.nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_adj_sub(const AdjSub& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_sub, dim3(a.nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_adj_point(const AdjPoint& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_point, dim3(nb(a.P)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_adj_axpy(int64_t P, const double2* x, const double2* y, double cr, double ci, double2* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_adj_axpy, dim3(nb(P)), dim3(256), 0, s, P, x, y, cr, ci, out);
  return hipGetLastError();
}
hipError_t launch_adj_copy2(int64_t P, double2* dst0, const double2* src0, double2* dst1, const double2* src1,
                            hipStream_t s) {
  if (P <= 0) return hipSuccess;
  const int n = nb(P);
  hipLaunchKernelGGL(k_adj_copy2, dim3(2 * n), dim3(256), 0, s, P, n, dst0, src0, dst1, src1);
  return hipGetLastError();
}
hipError_t launch_adj_reduce(const double* part, double* red, int nrows, int nblk, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_reduce, dim3(nrows), dim3(256), 0, s, part, red, nblk);
  return hipGetLastError();
}
hipError_t launch_adj_to_A(const double* red, const int* rowptr, const int* src, const double* wt, double* out, int nout,
                           hipStream_t s) {
  if (nout <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_to_A, dim3(nb(nout)), dim3(256), 0, s, red, rowptr, src, wt, out, nout);
  return hipGetLastError();
}

}  // namespace tdse
