// Internal declarations shared by the host planner and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tdse {

constexpr int MAXV = 8;   // spatial potential fields V_r
constexpr int MAXH = 8;   // history terms of the implicit Adams rule (n - 1 <= 7)

// Pass kinds.  A "column" pass transforms along axis 0 (stride M2 in memory),
// a "row" pass along the last axis (contiguous).
enum PassMode : int {
  C_SOLVE = 0,  // inverse FFT, diagonal solve u = w/(1 + i c V), Vu, forward FFT
  C_FWD = 1,    // pre-multiply (alpha + beta V) u, forward FFT
  R_AM = 2,     // forward FFT, implicit Adams recurrence, inverse FFT
  R_INIT = 3,   // forward FFT, B = P G, inverse FFT
  R_FWD = 4,    // forward FFT, store modes
  R_FORM = 5,   // forward FFT = uhat, B from uhat and history, inverse FFT
  R_INV = 6,    // inverse FFT of the FP64 state B (rows) into the tile buffer
};

// Transform precision: FP64 everywhere, or complex64 transforms, tile
// buffer, history ring and history quadrature with FP64 carried state.
enum Precision : int { P_FP64 = 0, P_SPLIT = 1 };

// Phase entries a column pass precomputes for the next row pass:
// theta_a(k) = -k^2 tau_j + k dphi_a[j], table ph[(j-1)(M1+M2) + kidx].
struct PhaseReq {
  int nj;
  double tau[MAXH];
  double dphi1[MAXH];
  double dphi2[MAXH];
};

// Arguments of one line pass.  Buffers whose element type follows the
// transform precision (complex128 or complex64) are untyped here; the
// carried state B, the physical solution and the phase tables are always
// complex128; the potential is double (FP64) or float (split).
struct LineArgs {
  const void* src;     // tile source: transform-precision tile, or complex128 physical u (C_FWD)
  void* dst;           // tile destination (transform precision)
  int64_t line_stride, elem_stride;
  int nlines;
  int M1, M2;          // grid (M1 = 1 for a 1D problem)
  const void* tw;      // twiddles of this line length (transform precision)
  int mode;
  // potential V = sum_r fV[r] V_r
  const void* V;
  int nV;
  int64_t vstride;
  double fV[MAXV];
  // column pass
  double csolve;       // u = w / (1 + i csolve V)
  double scale;        // 1/(M1 M2) folded into the forward transform input
  double alpha_re, alpha_im, beta_re, beta_im;  // C_FWD pre-op (alpha + beta V) u
  double2* uout;       // optional copy of the physical solution
  double2* uacc;       // optional Richardson accumulator
  double wacc;
  int acc_first;
  // row pass
  double2* Bm;
  void* ring;          // history ring (transform precision)
  int64_t ring_stride;
  int nh;
  int slot_w;
  int slot_r[MAXH + 1];
  double c0;           // mu_0 dt  (uhat = B - i c0 W)
  double ch[MAXH + 1]; // dt mu_j
  void* fdst;          // R_FWD destination (transform precision)
  // phase table
  double2* ph;
  PhaseReq req;
};

// Launchers (periodic_kernels.hip).  Non-null events e0/e1 are recorded at
// the kernel's own start and end.  Return a hipError_t.
hipError_t launch_col_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_row_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
bool line_length_supported(int N);
// dst[i] = (complex64) src[i], i < n (FP64 start-up state to split precision)
hipError_t launch_narrow(const double2* src, float2* dst, int64_t n, hipStream_t s);

}  // namespace tdse
