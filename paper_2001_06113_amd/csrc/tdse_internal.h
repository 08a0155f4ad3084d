// Internal declarations shared by the host planner and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tdse {

constexpr int MAXV = 8;   // spatial potential fields V_r
constexpr int MAXH = 8;   // history terms of the implicit Adams rule (n - 1 <= 7)
constexpr int FS_CHEB_MAX = 64;   // terms of the C-type Chebyshev interpolant

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
  R_BINIT = 7,  // free space: B = P (uhat - i c What), inverse transform
  R_UHACC = 8,  // free space: forward transform, uhat^(l) = B - i c What accumulated
};

// Transform precision: FP64 everywhere, or complex64 transforms, tile
// buffer, history ring and history quadrature with FP64 carried state.
enum Precision : int { P_FP64 = 0, P_SPLIT = 1 };

// Phase entries a column pass precomputes for the next row pass:
// theta_a(k) = -k^2 tau_j + k dphi_a[j], table ph[(j-1)(M1+M2) + kidx].
// In 3D the row index combines axes 0 and 1 (k0, k1): its entry is
// -(k0^2 + k1^2) tau_j + k0 dphi0[j] + k1 dphi1[j].
struct PhaseReq {
  int nj;
  double tau[MAXH];
  double dphi0[MAXH];
  double dphi1[MAXH];
  double dphi2[MAXH];
};

// Arguments of one line pass.  Buffers whose element type follows the
// transform precision (complex128 or complex64) are untyped here; the
// carried state B, the physical solution and the phase tables are always
// complex128; the potential is double in both forms.
struct LineArgs {
  const void* src;     // tile source: transform-precision tile, or complex128 physical u (C_FWD)
  void* dst;           // tile destination (transform precision)
  int64_t line_stride, elem_stride;
  int nlines;
  int M1, M2;          // grid (M1 = 1 for a 1D problem); 3D: M1 = M0 Mmid rows of M2
  int M0, Mmid;        // 3D: the two leading axes (Mmid = 0 in 1D and 2D)
  // lines in slabs (the middle axis of a 3D grid): line l starts at
  // (l / slab_lines) slab_stride + (l % slab_lines) line_stride; 0: no slabs
  int slab_lines;
  int64_t slab_stride;
  const void* tw;      // twiddles of this line length (transform precision)
  int mode;
  // potential V = sum_r fV[r] V_r (vkind 0), or for vkind 1 the moving
  // periodic Gaussian well evaluated on the fly, with fV = {-V0, 1/(2 beta^2),
  // centre along axis 0 (2D), centre along the last axis, images per side}
  // at the pass's time
  const void* V;
  int nV;
  int64_t vstride;
  double fV[MAXV];
  int vkind;
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
  int pf_pow;          // R_AM: no field along the last axis, its factors of E^(j) are the
                       // j-th powers of E^(1)'s (formed by products, not loaded)
  // phase table
  double2* ph;
  float2* ph32;        // split form: the table rounded to complex64 (null in FP64 plans)
  PhaseReq req;
};

// One axis of the free-space complex-frequency transform (freespace_kernels.hip):
// modes ordered E1 | A1 C A3 | E3 with N = 2 NE + ND.  All tables complex128,
// device pointers into the plan's workspace.
// With the C-type block through the Chebyshev interpolant (NT > 0), the
// dense sums run over NR = 2p + NT rows: the A1 nodes, the NT interpolation
// nodes (1 - i) H s_m on Gamma_2 and the A3 nodes; the N_C C-modes are the
// interpolant's values, Pf (forward, [N_C][NT] real) expands the node values
// into them and Pi (inverse, [NT][N_C], weights w/2pi folded in) contracts
// them back onto the nodes.  NT = 0: NR = ND, every dense row is a mode.
struct CFAxis {
  int M, N, NE, ND;             // grid points, modes, E-nodes per side, dense modes
  int NR, NT, NP;               // dense rows, interpolation nodes (0: direct sums), Alpert nodes per side
  const double2 *pre3, *pre1;   // [M] forward pre-multipliers (E3, E1)
  const double2 *post3, *post1; // [NE] forward post-multipliers incl. 2/M
  const double2 *ipre3, *ipre1; // [NE] inverse pre-multipliers incl. w/(2 pi)
  const double2 *ipost3, *ipost1; // [M] inverse post-multipliers
  const double2* Dfwd;          // [NR][M] (2/M) exp(-i zeta_r x_j)
  const double2* Dinv;          // [NR][M] (w_r/2pi) exp(i zeta_r x_j) (interpolation rows: no weight)
  const double2* tw;            // nu-point twiddles
  const double2* zeta;          // [N] nodes (for the phase factors)
  const double2* rfwd;          // [NR] exp(-i zeta_r 2/M): Dfwd[r][j+1] = Dfwd[r][j] rfwd[r]
  const double2* wq;            // [N] quadrature weights of the nodes zeta
  const double* Pf;             // [N_C][NT] interpolation from the nodes to the C-modes
  const double2* Pi;            // [NT][N_C] its transpose times w_k / 2pi
};


struct FSArgs {
  int mode;
  int N1, N2;                   // modes per axis (N1 = 1 for a 1D problem)
  const double2* src;           // tile source
  double2* dst;                 // tile destination
  const double2* usrc;          // physical solution (C_FWD)
  double2* fdst;                // R_FWD destination (modes)
  double2* Bm;
  double2* ring;
  int64_t ring_stride;
  double2* UH;                  // carried uhat (start-up)
  double2* UHacc;               // Richardson accumulator of uhat
  double2* uout;
  double2* uacc;
  double wacc;
  int acc_first;
  const double* V;
  int nV;
  int64_t vstride;
  double fV[MAXV];
  double csolve;
  double alpha_re, alpha_im, beta_re, beta_im;
  int nh, slot_w;
  int slot_r[MAXH + 1];
  double c0;
  double ch[MAXH + 1];
  double2* ph;
  PhaseReq req;
  CFAxis ax1, ax2;
  // 3D: the row pass runs over N1 = N0 Nm rows (k0, k1), the column pass
  // over ncol = Mm M2 columns (x1, x2) of the (k0, x1, x2) array, and the
  // middle-axis passes transform along axis 1 (axm) between the two
  int pf_pow;                   // the last axis' phase factors of E^(j) are the j-th powers of E^(1)'s
                                // (no field component along it): the row pass forms them by products
  int Nm;                       // middle-axis modes (0: 1D or 2D)
  int64_t ncol;                 // columns of the column pass (M2 in 2D)
  CFAxis axm;
};

// Batched passes (batch_fp64.hip, batch_split.hip): one launch per schedule
// family over the tiles of many instances.  A tile is one workgroup's lines
// of one instance, transformed with the schedule sched = N * 64 + EPT (line
// length N, EPT elements per thread); blk/nblk number the tile among the
// instance's tiles of the pass.
constexpr int BATCH_THREADS = 256;
struct BatchTile {
  int32_t inst, line0, blk, nblk, sched, pad;
};
bool batch_schedule_ok(int N, int ept);
int batch_family(int N, int ept);                               // -1 if no such schedule
size_t batch_lds_bytes(int prec, bool col, int N, int ept);   // 0 if no such schedule
hipError_t launch_batch_pass(int prec, bool col, int family, const LineArgs* args, const BatchTile* tiles,
                             int ntiles, size_t lds_bytes, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);

// Adjoint of the periodic scheme (adjoint_kernels.hip), FP64.
constexpr int ADJ_PH = 2 * MAXH;   // phase entries of one adjoint Adams step
struct AdjPhase {                  // per-axis table ph[e (M1+M2) + k], e < nj
  int M1, M2, nj;
  double tau[ADJ_PH], dphi1[ADJ_PH], dphi2[ADJ_PH];
  double2* ph;
};
struct AdjAm {                     // one adjoint implicit Adams step (mode space, P modes)
  int M1, M2, H;
  int64_t P;
  const double2* ph;               // entries j-1: E^(j)_{n+1}; H+j-1: E^(j)_{n-1+j}
  double2* beta;                   // ring of adjoint states, slots of P modes
  int slot_b1;                     // beta_{n+1} (-1: zero)
  int slot_bn;                     // beta_n
  int beta_mode;                   // 0: beta_n = 0; 1: beta_n = conj(E^(1)_{n+1}) beta_{n+1} + Z; 2: read
  const double2* Z;                // G_n^H omega_n
  double2* omega;                  // out: omega_{n-1} (null: none)
  int slot_bj[MAXH + 1];           // beta_{n-1+j}, j >= 2 (-1: zero)
  double wj[MAXH + 1];             // omega weights dt c_{n-1,j}
  int has_grad;                    // dJ/d(dphi) partials of the phase factors of step n+1
  const double2* Bn;               // x_1 = B_n - i cx[1] What_n
  const double2* Wx[MAXH + 1];     // Wx[1] = What_n, Wx[j] = What_{n+1-j}
  double cx[MAXH + 1];             // x_j = -i cx[j] What_{n+1-j}, j >= 2
  double* part;                    // partial sums [2 (j-1) + axis][nblk]
  int nblk;
};
struct AdjSub {                    // phase factor of an order-2 sub-step (entry 0 of ph)
  int M1, M2, mode;                // 1: y = E g; 0: partials and y = conj(E) y; 2: y = conj(E) y
  int64_t P;
  const double2* ph;
  double2* y;
  const double2* g;
  double* part;                    // partial sums [axis][nblk]
  int nblk;
};
struct AdjPoint {                  // out (+)= s (alpha + beta V) in, or s in / (alpha + beta V)
  int64_t P;
  const double2* in;
  double2* out;
  const double* V;
  int nV;
  int64_t vstride;
  double fV[MAXV];
  double ar, ai, br, bi, s;
  int divide, accumulate;
};
hipError_t launch_adj_phase(const AdjPhase& q, hipStream_t s);
hipError_t launch_adj_am(const AdjAm& a, hipStream_t s);
hipError_t launch_adj_sub(const AdjSub& a, hipStream_t s);
hipError_t launch_adj_point(const AdjPoint& a, hipStream_t s);
hipError_t launch_adj_axpy(int64_t P, const double2* x, const double2* y, double cr, double ci, double2* out,
                           hipStream_t s);
hipError_t launch_adj_copy2(int64_t P, double2* dst0, const double2* src0, double2* dst1, const double2* src1,
                            hipStream_t s);
hipError_t launch_adj_reduce(const double* part, double* red, int nrows, int nblk, hipStream_t s);
hipError_t launch_adj_to_A(const double* red, const int* rowptr, const int* src, const double* wt, double* out,
                           int nout, hipStream_t s);

// Free-space launchers (freespace_kernels.hip); events as for the periodic passes.
hipError_t launch_fs_row(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// nu = 0: the pointwise pass of a 1D problem
hipError_t launch_fs_col(int nu, const FSArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_fs_phase(const FSArgs& a, hipStream_t s);
// 3D: the line transform along the middle axis (a.axm) of the N0 x Nm x M2
// mode array src into the N0 x Mm x M2 grid array dst (inverse), or back
// (forward); lines (k0, x2), one per workgroup
hipError_t launch_fs_mid(int nu, bool inverse, const FSArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
bool fs_nu_supported(int nu);
size_t fs_line_lds_bytes(int nu, int M, int ND, bool ch);   // dynamic LDS of a line workgroup (ch: interpolant on)

// Evaluation of a free-space representation at arbitrary points (far_kernels.hip).
// far_scratch: device address, on the current GPU, of the library-owned array
// of FAR_SCRATCH_BYTES that the allocation-free evaluation uses as workspace.
constexpr size_t FAR_SCRATCH_BYTES = (size_t)64 << 20;
hipError_t far_scratch(void** ptr);
// E[k n + i] = (w_k / 2 pi) exp(i zeta_k x_i), k < N, i < n
hipError_t launch_far_table(const double2* zeta, const double2* w, int N, const double* x, int n, double2* E,
                            hipStream_t s);
// C[m][n] = sum_k A[m sam + k sak] B[k sbk + n sbn], complex128, C row-major (ldc)
hipError_t launch_far_gemm(int M, int N, int K, const double2* A, int64_t sam, int64_t sak, const double2* B,
                           int64_t sbk, int64_t sbn, double2* C, int64_t ldc, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);

// One-workgroup run of a 1D periodic FP64 problem (run1d_kernels.hip): steps
// m0+1 .. m1 of the scheme in one launch.  Per-step scalars come from `tab`:
//   oH + 8 m                      f_r(t_m), m = 0..ns (history at the start-up times)
//   oR + 9 ((m-1)(2^L-1) + 2^l - 1 + k)
//                                 start-up step m, level l, sub-step k: f_r at its end
//                                 time [8], then the phase increment phi(end) - phi(start)
//   oA + 8 (m - ns - 1)           f_r(t_m), Adams step m
//   oD + i - 1                    phi(t_i) - phi(t_{i-1}), i = 1..nsteps
// (f_r: the eight potential time factors, or the moving well's parameters).
// stab holds exp(-i k^2 j dt), j = 1..n-1, then exp(-i k^2 dt / 2^l), l < L.
struct Run1DArgs {
  int M, order, ns, nsteps, L;
  int m0, m1;
  int nV, vkind;
  int write_u, has_phase, stab_rows;
  double dt, c0;
  double ch[MAXH + 1];
  double rich[4];
  const double* V;
  int64_t vstride;
  const double* tab;
  int64_t oH, oR, oA, oD;
  const double2* u_in;
  double2* u_out;
  double2* B;
  double2* ring;
  const double2* stab;
  const double2* tw;
};
bool run1d_supported(int N);
size_t run1d_lds_bytes(int N, int stab_rows, int nV);
hipError_t launch_run1d(const Run1DArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Persistent implicit Adams steps of a square 2D periodic FP64 problem
// (persist2d_kernels.hip): steps m0+1 .. m1 (all past the Adams start) by one
// co-resident grid of N/2 workgroups.  Per step m, tab + ostep (m - mbase)
// holds the eight potential time factors at t_m and phi_1(t_{m+1}) -
// phi_1(t_{m+1-j}), j = 1..7; tab[oD2 + i - 1] = phi_2(t_i) - phi_2(t_{i-1}).
// S2 holds exp(-i k2^2 j dt), j = 1..n-1.  tile: the row-major tile of the
// two-pass path (read by the first step, written by a launch that ends
// before T); xbuf: an N x N complex128 exchange buffer (blocked layout).
// bar: P2_BAR_WORDS words of barrier counters, flag: the timeout flag (both
// reset by the launch).
struct Persist2DArgs {
  int N, order, nsteps, m0, m1, mbase, ostep, nV, write_u, ph2, spin_limit;
  double dt, c0, scale;
  double ch[MAXH + 1];
  const double* V;
  int64_t vstride;
  const double* tab;
  int64_t oD2;
  double2* tile;
  double2* xbuf;
  double2* B;
  double2* ring;
  const double2* S2;
  const double2* tw;
  double2* uout;
  unsigned* bar;
  unsigned* flag;
};
constexpr int P2_BAR_WORDS = 32 * 9 + 32;   // grid counter, eight XCD counters (128 bytes apart), flag
bool persist2d_supported(int N);
size_t persist2d_lds_bytes(int N, int order);
int persist2d_capacity(int N, int order, bool ph2);   // co-resident workgroups the device holds
hipError_t launch_persist2d(const Persist2DArgs& a, hipStream_t s);

// Diagnostics (diag_kernels.hip).  acc: two doubles, flag: one word, both
// cleared by the launch (the guard: unless clear is false, to accumulate
// several arrays).  Guard: acc[0] += sum x_i^2 over n doubles, flag set if one
// is not finite.  Difference: acc[0] += sum |a - b|^2, acc[1] += sum |b|^2
// over n complex entries, a complex64 (a32) or complex128 (a64).
hipError_t launch_guard(const double* x, int64_t n, double* acc, unsigned* flag, bool clear, hipStream_t s);
hipError_t launch_diffnorm(const float2* a32, const double2* a64, const double2* b, int64_t n, double* acc,
                           unsigned* flag, hipStream_t s);

// Launchers (periodic_kernels.hip).  Non-null events e0/e1 are recorded at
// the kernel's own start and end.  Return a hipError_t.
hipError_t launch_col_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_mid_pass(int prec, int N, bool inverse, const LineArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);   // 3D middle axis, in place (a.src == a.dst)
hipError_t launch_row_pass(int prec, int N, const LineArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
bool line_length_supported(int N);
// dst[i] = (complex64) src[i], i < n (FP64 start-up state to split precision)
hipError_t launch_narrow(const double2* src, float2* dst, int64_t n, hipStream_t s);

}  // namespace tdse
