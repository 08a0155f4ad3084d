// Evaluation of a free-space solution at arbitrary points from its
// complex-frequency representation on Gamma_K (Section 3.2 and the Remark
// on evaluation outside [-1,1]), gfx950:
//   u(x_i, y_j) = sum_{k1,k2} E1[k1][i] E2[k2][j] uhat[k1][k2],
//   E_a[k][i]   = (w_k / 2 pi) exp(i zeta_k x_i)      (quadrature of axis a),
// as a table kernel per axis and two complex FP64 matrix-core products,
//   S = uhat E2 (N1 x ny), then u = E1^T S (nx x ny).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <mutex>

#include "tdse_internal.h"

namespace tdse {

// Device memory of the allocation-free evaluation (tdse_far_eval_noalloc):
// one array per GPU, part of the code object, so it needs no allocation call
// and lives until the process ends.  In host code its name is only a
// stand-in: its device address on the current GPU comes from
// hipGetSymbolAddress, looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[FAR_SCRATCH_BYTES];

hipError_t far_scratch(void** ptr) {
  constexpr int MAXDEV = 64;
  static std::mutex lock;
  static void* addr[MAXDEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> hold(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// E[k * n + i] = (w_k / 2 pi) exp(i zeta_k x_i), k < N, i < n
__global__ __launch_bounds__(256) void k_far_table(const double2* __restrict__ zeta, const double2* __restrict__ w,
                                                   int N, const double* __restrict__ x, int n,
                                                   double2* __restrict__ E) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)N * n) return;
  const int k = (int)(g / n), i = (int)(g % n);
  constexpr double INV_2PI = 0.159154943091895335768883763372514362;
  const double2 z = zeta[k], wk = w[k];
  const double xi = x[i];
  // exp(i zeta x) = exp(-Im(zeta) x) (cos(Re(zeta) x) + i sin(Re(zeta) x))
  double s, c;
  sincos(z.x * xi, &s, &c);
  const double m = exp(-z.y * xi) * INV_2PI;
  const double er = m * c, ei = m * s;
  E[g] = double2{wk.x * er - wk.y * ei, wk.x * ei + wk.y * er};
}

// C[m][n] = sum_k A[m sam + k sak] B[k sbk + n sbn] (complex128), C row-major
// with leading dimension ldc, on the FP64 matrix cores.  A workgroup of four
// waves computes a T x T tile of C (T = 32 WB), each wave a quarter of it as
// WB x WB blocks of the 16 x 16 x 4 FP64 MFMA.  K advances in chunks of 16
// staged through LDS (zeros beyond the operands' edges), four MFMA k-steps a
// chunk, and the next chunk's operands are loaded into registers while the
// MFMAs work on the current one.  Operand lanes: A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k; the result D[q + 4 r][j] sits in lane j + 16 q,
// element r.  A complex product takes four real ones: Re C += Re A Re B -
// Im A Im B, Im C += Re A Im B + Im A Re B.  Tiles are numbered along n first.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int FAR_K = 16;
template <int WB>
__global__ __launch_bounds__(256) void k_far_gemm(int M, int N, int K, const double2* __restrict__ A, int64_t sam,
                                                  int64_t sak, const double2* __restrict__ B, int64_t sbk,
                                                  int64_t sbn, double2* __restrict__ C, int64_t ldc) {
  constexpr int T = 32 * WB;           // output tile edge
  constexpr int LD = T * FAR_K / 256;  // operand elements per thread and chunk
  __shared__ double2 As[FAR_K][T + 1];
  __shared__ double2 Bs[FAR_K][T + 1];
  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  const int wm = 16 * WB * (wave / 2), wn = 16 * WB * (wave % 2);
  const int li = lane % 16, lk = lane / 16;
  const int ntn = (N + T - 1) / T;
  const int m0 = (blockIdx.x / ntn) * T, n0 = (blockIdx.x % ntn) * T;
  f64x4 cr[WB][WB], ci[WB][WB];
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[a][b][r] = 0.0;
        ci[a][b][r] = 0.0;
      }
  double2 ra[LD], rb[LD];
  // element e of a chunk: A along k when A is contiguous in k, else along m;
  // B along n
  auto a_at = [&](int e, int& ka, int& ma) {
    ka = sak == 1 ? e % FAR_K : e / T;
    ma = sak == 1 ? e / FAR_K : e % T;
  };
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LD; ++r) {
      const int e = tid + 256 * r;   // 0 .. T * FAR_K - 1
      int ka, ma;
      a_at(e, ka, ma);
      const int gm = m0 + ma, gka = k0 + ka;
      ra[r] = (gm < M && gka < K) ? A[(int64_t)gm * sam + (int64_t)gka * sak] : double2{0.0, 0.0};
      const int kb = e / T, nb = e % T;
      const int gn = n0 + nb, gkb = k0 + kb;
      rb[r] = (gn < N && gkb < K) ? B[(int64_t)gkb * sbk + (int64_t)gn * sbn] : double2{0.0, 0.0};
    }
  };
  if (K > 0) load_chunk(0);
  for (int k0 = 0; k0 < K; k0 += FAR_K) {
#pragma unroll
    for (int r = 0; r < LD; ++r) {
      const int e = tid + 256 * r;
      int ka, ma;
      a_at(e, ka, ma);
      As[ka][ma] = ra[r];
      Bs[e / T][e % T] = rb[r];
    }
    __syncthreads();
    if (k0 + FAR_K < K) load_chunk(k0 + FAR_K);
#pragma unroll
    for (int ks = 0; ks < FAR_K; ks += 4) {
      double2 av[WB], bv[WB];
#pragma unroll
      for (int a = 0; a < WB; ++a) av[a] = As[ks + lk][wm + 16 * a + li];
#pragma unroll
      for (int b = 0; b < WB; ++b) bv[b] = Bs[ks + lk][wn + 16 * b + li];
#pragma unroll
      for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[b].y, cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * a + lk + 4 * r, gn = n0 + wn + 16 * b + li;
        if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = double2{cr[a][b][r], ci[a][b][r]};
      }
}

hipError_t launch_far_table(const double2* zeta, const double2* w, int N, const double* x, int n, double2* E,
                            hipStream_t s) {
  const int64_t tot = (int64_t)N * n;
  if (tot <= 0) return hipSuccess;
  if ((tot + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_far_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, zeta, w, N, x, n, E);
  return hipGetLastError();
}

hipError_t launch_far_gemm(int M, int N, int K, const double2* A, int64_t sam, int64_t sak, const double2* B,
                           int64_t sbk, int64_t sbn, double2* C, int64_t ldc, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // 64 x 64 tiles when they give every compute unit two or more, else
  // 32 x 32 tiles (four times as many workgroups for small outputs)
  const int64_t tiles64 = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  const bool big = tiles64 >= 512;
  const int64_t tiles = big ? tiles64 : (int64_t)((M + 31) / 32) * ((N + 31) / 32);
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  // with events, recorded at the kernel's own start and end
#define FAR_LAUNCH(KER)                                                                                             \
  do {                                                                                                              \
    if (e0)                                                                                                         \
      hipExtLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(256), 0, s, e0, e1, 0, M, N, K, A, sam, sak, B, sbk,    \
                            sbn, C, ldc);                                                                           \
    else                                                                                                            \
      hipLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);   \
  } while (0)
  if (big)
    FAR_LAUNCH(k_far_gemm<2>);
  else
    FAR_LAUNCH(k_far_gemm<1>);
#undef FAR_LAUNCH
  return hipGetLastError();
}

}  // namespace tdse
