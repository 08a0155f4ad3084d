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
};

// Phase entries a column pass precomputes for the next row pass:
// theta_a(k) = -k^2 tau_j + k dphi_a[j], table ph[(j-1)(M1+M2) + kidx].
struct PhaseReq {
  int nj;
  double tau[MAXH];
  double dphi1[MAXH];
  double dphi2[MAXH];
};

template <typename C>
struct LineArgsT {
  const C* src;        // tile source
  C* dst;              // tile destination
  int64_t line_stride, elem_stride;
  int nlines;
  int M1, M2;          // grid (M1 = 1 for a 1D problem)
  const C* tw;         // twiddles of this line length
  int mode;
  // potential V = sum_r fV[r] V_r
  const double* V;
  int nV;
  int64_t vstride;
  double fV[MAXV];
  // column pass
  double csolve;       // u = w / (1 + i csolve V)
  double scale;        // 1/(M1 M2) folded into the forward transform input
  double alpha_re, alpha_im, beta_re, beta_im;  // C_FWD pre-op (alpha + beta V) u
  C* uout;             // optional copy of the physical solution
  C* uacc;             // optional Richardson accumulator
  double wacc;
  int acc_first;
  // row pass
  C* Bm;
  C* ring;
  int64_t ring_stride;
  int nh;
  int slot_w;
  int slot_r[MAXH + 1];
  double c0;           // mu_0 dt  (uhat = B - i c0 W)
  double ch[MAXH + 1]; // dt mu_j
  C* fdst;             // R_FWD destination
  // phase table
  C* ph;
  PhaseReq req;
};

using LineArgs = LineArgsT<double2>;

// Launchers (periodic_kernels.hip).  Return a hipError_t.
hipError_t launch_col_pass(int N, const LineArgs& a, hipStream_t s);
hipError_t launch_row_pass(int N, const LineArgs& a, hipStream_t s);
// Column-pass tile width (lines per workgroup) and grid for a line length N.
int col_lines_per_block(int N);
int row_lines_per_block(int N);
bool line_length_supported(int N);

}  // namespace tdse
