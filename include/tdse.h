/* tdse.h -- C ABI of the MI355X (gfx950) Volterra-integral TDSE marcher.
 *
 * Method: Kaye, Barnett, Greengard, "A high-order integral equation-based
 * solver for the time-dependent Schrodinger equation" (arXiv:2001.06113).
 *
 * The library solves, on one GPU,
 *     i u_t = -Lap u + V(x,t) u + i A(t).grad u,   u(x,0) = u0(x)      (Section 1, eq. (schrodfree))
 * on the periodic box [-pi,pi]^d (Section 2) or in free space with u0, V
 * supported in [-1,1]^d (Section 3, complex-frequency modes on the contour
 * Gamma with the FFT-based transforms of Section 4), for d = 1 or 2, with
 *     V(x,t) = sum_r f_r(t) V_r(x)    (real fields V_r on the grid),
 * by the Fourier-mode recurrence of Lemma 1 with the n-th order implicit
 * Adams rule of eq. (uadamsk) (Section 2.2, Table 1 for n = 8) and the
 * iterated-Richardson start-up of Section 2.2.  Each step is one inverse
 * FFT, a pointwise diagonal solve, one forward FFT and a per-mode
 * recurrence, all in HIP kernels.
 *
 * Conventions
 *   - complex values are interleaved (re, im) doubles (complex128), arrays in
 *     C order with the last axis fastest; a 1D problem has shape [M[0]].
 *   - periodic grid x_j = -pi + 2 pi j / M, j = 0..M-1 (Section 2.1);
 *     free-space grid x_j = -1 + 2 j / M (Section 3.3).
 *   - dt = T / nsteps.
 *
 * Errors: every call returns TDSE_OK (0) or a negative status; no C++
 * exception crosses this boundary.  tdse_status_string() names a status and
 * tdse_last_error() gives the text of the most recent failure on the calling
 * thread.
 *
 * Ownership: host inputs are copied during tdse_plan (callbacks are invoked
 * only inside tdse_plan).  The device workspace belongs to the caller and
 * must outlive every call that uses it; the plan owns only host metadata.
 * Device work is asynchronous on the stream given to tdse_bind; calls that
 * return data to host memory synchronize that stream.  A plan is not
 * thread-safe.
 */
#ifndef TDSE_H
#define TDSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define TDSE_OK            0
#define TDSE_EINVAL       -1   /* bad sizes, non-integer T/dt, bad order, NULL */
#define TDSE_EUNSUPPORTED -2   /* a valid request the library does not do    */
#define TDSE_ENOMEM       -3   /* workspace missing or too small              */
#define TDSE_EDEVICE      -4   /* a HIP runtime error                         */
#define TDSE_ENONFINITE   -5   /* the state became NaN/Inf                    */
#define TDSE_ESTATE       -6   /* calls made in the wrong order               */

/* ---- enumerations ------------------------------------------------------- */
#define TDSE_PERIODIC 0        /* D = [-pi,pi]^d, Section 2                    */
#define TDSE_FREE     1        /* D = R^d, supp u0, V in [-1,1]^d, Section 3   */

#define TDSE_FP64        0     /* every stage in double precision             */
#define TDSE_FP32_SPLIT  1     /* complex64 transforms and history, FP64 state */

#define TDSE_F_CONST     0     /* f_r(t) = 1                                   */
#define TDSE_F_SIN       1     /* f_r(t) = 1 + f_params[2r] sin(f_params[2r+1] t) */
#define TDSE_F_CALLBACK  2     /* f_r(t) = f_fn(r, t, f_ctx)                   */

/* potential kinds (V_kind) */
#define TDSE_V_FIELDS    0     /* V = sum_r f_r(t) V_r(x) from nV stored fields */
#define TDSE_V_MOVING_WELL 1   /* Example 1 of Section 6: periodic Gaussian well moving at constant velocity,
                                  V = -V0 sum_k exp(-|x - 2 pi k - c t|^2 / (2 beta^2)), evaluated on the fly;
                                  V_params = {V0, beta, c[0], c[1]} (c[a] along axis a; 0 < beta <= 1, so at most
                                  three images per axis lie within 9.2 beta of a point);
                                  periodic plans; no fields (nV = 0, V_fields NULL) */
#define TDSE_V_SAMPLED   2     /* a general V(x, t) given by its samples at the step times t_n = n dt:
                                  V_fields = [nsteps + 1][prod M] (nV ignored).  At a step time the sample;
                                  between step times (the Richardson start-up's sub-steps) the degree-7
                                  Lagrange interpolant through the eight nearest samples
                                  t_n0..t_n0+7, n0 = clamp(floor(t/dt) - 3, 0, nsteps - 7) (every sample
                                  when nsteps < 7), whose O(dt^8) error matches the scheme's order.
                                  Periodic and free-space single plans, 1D to 3D; at most 64 GiB of
                                  samples; no batch, no adjoint */

#define TDSE_A_NONE      0     /* A = 0                                        */
#define TDSE_A_PULSE_SIN2 1    /* A = E0 sin^2(pi t/Tp) sin(w t) dir; A_params = {E0, w, Tp, dir[0..d-1]} */
#define TDSE_A_CALLBACK  2     /* A(t) from A_fn; phi = int A by Gauss-Legendre per step */
#define TDSE_A_STEPWISE  3     /* A constant on each step: A_steps[nsteps][d]  */
#define TDSE_A_PULSE_COS2 4    /* eq. (apulse): A = E0 sin^2(pi t/Tp) cos(w t) dir; A_params as for PULSE_SIN2 */

typedef double (*tdse_scalar_fn)(int32_t r, double t, void* ctx);
typedef void (*tdse_vector_fn)(double t, double* A_out, void* ctx);

/* Problem statement (Section 1: domain, u0 via tdse_set_state, V(x,t), A(t),
 * T, step size, order).  Unused fields may be zero.
 * d = 3 (Section 4.3): the periodic scheme of Section 2 in three dimensions
 * (TDSE_FP64 or TDSE_FP32_SPLIT) or the free-space scheme with the line
 * transforms of Section 4.1 along each of the three axes (TDSE_FP64; the 125
 * node-type subsets of Section 4.3 in tensor order); stored or sampled
 * potentials (V_kind 0 or 2), at most 2^28 grid points; single plans (no
 * batch, no adjoint, no evaluation at arbitrary points).  Arrays are
 * row-major over
 * M[0] x M[1] x M[2] with the last axis fastest; A has d components. */
typedef struct {
  int32_t dim;             /* 1, 2 or 3                                      */
  int32_t domain;          /* TDSE_PERIODIC | TDSE_FREE (FP64 only)          */
  int32_t M[3];            /* grid points per axis: 2^a or 3*2^a, 8..3072    */
  double  T;               /* final time > 0                                 */
  int32_t nsteps;          /* number of steps, dt = T / nsteps               */
  int32_t order;           /* implicit Adams order n in {2,4,6,8}            */
  int32_t n_start;         /* Richardson start-up steps; < 0 means n - 2     */
  int32_t precision;       /* TDSE_FP64 | TDSE_FP32_SPLIT                    */
  int32_t nV;              /* number of spatial fields, 1..8 (0: V_kind well; ignored: sampled) */
  const double* V_fields;  /* host [nV][prod M] real, last axis fastest      */
  int32_t f_kind;          /* TDSE_F_*                                       */
  const double* f_params;  /* TDSE_F_SIN: [nV][2] = (amp, omega)             */
  tdse_scalar_fn f_fn; void* f_ctx;
  int32_t A_kind;          /* TDSE_A_*                                       */
  const double* A_params;  /* TDSE_A_PULSE_SIN2/COS2: {E0, omega, Tp, dir[d]} */
  const double* A_steps;   /* TDSE_A_STEPWISE: host [nsteps][d]              */
  tdse_vector_fn A_fn; void* A_ctx;
  /* free space (Sections 3.4 and 4): tolerance eps for the choice of H
   * (Remark on H, applied per axis with that axis' quiver radius),
   * Alpert order p (8: 16th order, kappa = 7 omitted nodes),
   * q Gauss nodes per panel and `panels` dyadic panels per side of Gamma_2,
   * FFT size nu per axis (N_E = nu/2 - 2 kappa + 1 equispaced nodes per ray,
   * h = pi M / nu); H > 0 overrides the rule for H. */
  double  eps;
  int32_t p, q, panels;
  int32_t nu[3];
  double  H;
  /* potential kind (TDSE_V_*; 0 = stored fields) and its parameters */
  int32_t V_kind;
  double  V_params[4];
  /* free space: the C-type transforms on Gamma_2 (Section 4.1).  Either
   * direct sums over the N_C = 2 q panels Gauss nodes, or the Chebyshev
   * interpolant of eqs. (expintrpm)/(expintrpp) on [-H, H] with NT terms,
   * which costs O(M NT + NT N_C) per line instead of O(M N_C).  The library
   * evaluates the interpolant through its values at the NT Chebyshev points of
   * the first kind (the same polynomial as the paper's coefficient form).
   * 0: automatic: the interpolant when its NT < N_C, NT the smallest count
   *    with 4 sum_{l >= NT} I_l(sqrt(2) H) <= 2^-52 (exact to rounding);
   * -1: direct sums; 2..64: the interpolant with that many terms.
   * In 2D the axes' transforms compose, which gives the (C,E) and (C,C)
   * subsets of Section 4.2 with the sums in tensor order. */
  int32_t cheb;
} tdse_problem_t;

typedef struct tdse_plan_s* tdse_plan_t;   /* opaque, owned by the library  */

/* Build a plan: validate the problem and precompute every time-dependent
 * scalar (phi(t) = int_0^t A, eq. (phi); f_r(t)) at all step and sub-step
 * times, the implicit Adams weights (Table 1 for n = 8) and the Richardson
 * weights (Section 2.2).  Host only.  On success *out owns a new plan. */
int tdse_plan(const tdse_problem_t* prob, tdse_plan_t* out);

/* Bytes of device workspace the plan needs (alignment 256). */
int tdse_workspace_size(tdse_plan_t plan, size_t* bytes);

/* Attach a device workspace of `bytes` bytes (caller-owned, 256-aligned) and
 * a HIP stream (NULL = default stream); uploads the static tables.  May be
 * called again to move the plan to another buffer or stream. */
int tdse_bind(tdse_plan_t plan, void* device_workspace, size_t bytes, void* hip_stream);

/* Set u(.,0) = u0 (complex128, shape M) and reset the clock to t = 0.
 * on_device != 0: u0 is a device pointer (copied asynchronously); otherwise
 * host memory (copied before return). */
int tdse_set_state(tdse_plan_t plan, const void* u0, int32_t on_device);

/* Advance `nsteps` time steps (asynchronous on the bound stream).  The first
 * n_start steps use Richardson extrapolation of the order-2 scheme of
 * eq. (utrapk); later steps use eq. (uadamsk).  ESTATE past t = T. */
int tdse_step(tdse_plan_t plan, int32_t nsteps);

/* Copy u(., t_current) into `u` (complex128, shape M).  on_device != 0:
 * device pointer, asynchronous; otherwise host memory, synchronizes. */
int tdse_get_state(tdse_plan_t plan, void* u, int32_t on_device);

/* set_state(u0) + step(all remaining) + get_state(uT). */
int tdse_run(tdse_plan_t plan, const void* u0, void* uT, int32_t on_device);

/* ---- evaluation of a free-space solution at arbitrary points -----------
 *
 * Once uhat(zeta, t) is resolved on Gamma_K, the complex-frequency
 * representation u(x, t) = (1/2pi) int_{Gamma_K} exp(i zeta . x) uhat d zeta
 * (Section 3.2) holds at every real x, inside [-1,1]^d or outside it (Remark
 * on evaluation outside [-1,1]).  tdse_far_eval evaluates its discretization
 * on the plan's own nodes and weights (eq. (uciftdisc)),
 *   u(x_i, y_j) = sum_{k1,k2} (w_k1 w_k2 / 4 pi^2) exp(i (zeta_k1 x_i + zeta_k2 y_j)) uhat_k1k2,
 * on the tensor grid of the axis-0 points xs[0..nx) and the last-axis points
 * ys[0..ny) (a 1D plan: nx = 1, xs ignored, may be NULL).  The nodes are not
 * refined, so accuracy falls off with |x| - 1 as exp(H (|x| - 1)) amplifies
 * rounding and truncation (about 1e-12 at |x| = 2 for the wave packet of
 * Section 6, Example 2 with eps = 1e-12).
 *
 * The mode state exists at t = 0 (uhat = F u0), after each start-up step, and
 * at t = T (uhat_N = B_N - i mu_0 dt F(V u_N)); at other times ESTATE.
 * xs, ys, out (complex128, nx x ny row-major: out[i ny + j] = u(xs[i], ys[j]))
 * and work (caller-owned, 256-byte aligned, size from tdse_far_workspace_size)
 * are device pointers; the call is asynchronous on the bound stream.  Free-space
 * plans only (EUNSUPPORTED otherwise); 1 <= nx, ny <= 2^24.  With profiling on
 * (tdse_profile), the first product (the contraction over the last axis) is
 * timed into TDSE_Q_PROF_MS_FAR. */
int tdse_far_workspace_size(tdse_plan_t plan, int32_t nx, int32_t ny, size_t* bytes);
int tdse_far_eval(tdse_plan_t plan, const double* xs, int32_t nx, const double* ys, int32_t ny, void* out,
                  void* work, size_t bytes);

/* Allocation-free evaluation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results as tdse_far_eval, with the workspace taken
 * from a library-owned device array of TDSE_FAR_SCRATCH_BYTES per GPU
 * (part of the library's code object, held until the process ends) instead
 * of a caller buffer.  Calls no allocation routine.  TDSE_ENOMEM when
 * tdse_far_workspace_size for (nx, ny) exceeds TDSE_FAR_SCRATCH_BYTES.
 * Every call on one GPU shares that array: calls ordered on one stream are
 * safe, calls that overlap on one GPU (several streams or host threads) race.
 * Arguments and errors otherwise as for tdse_far_eval (no profiling). */
#define TDSE_FAR_SCRATCH_BYTES ((size_t)64 << 20)
int tdse_far_eval_noalloc(tdse_plan_t plan, const double* xs, int32_t nx, const double* ys, int32_t ny, void* out);

/* Scalar queries (keys below). */
#define TDSE_Q_MODES          0   /* modes per instance (prod M)               */
#define TDSE_Q_STEPS_DONE     1   /* steps taken since set_state               */
#define TDSE_Q_DT             2
#define TDSE_Q_BYTES_PER_STEP 3   /* algorithmic HBM bytes of one Adams step   */
#define TDSE_Q_PROF_MS_MID    5   /* profiling (3D): summed ms of the middle-axis FFT passes */
#define TDSE_Q_PROF_N_MID     6   /* profiling (3D): number of timed middle-axis passes      */
#define TDSE_Q_BYTES_MID      7   /* 3D: algorithmic HBM bytes of one middle-axis pass        */
#define TDSE_Q_PROF_MS_COL    8   /* profiling: summed ms of Adams column passes */
#define TDSE_Q_PROF_MS_ROW    9   /* profiling: summed ms of Adams row passes  */
#define TDSE_Q_PROF_N_COL    10   /* profiling: number of timed column passes  */
#define TDSE_Q_PROF_N_ROW    11   /* profiling: number of timed row passes     */
#define TDSE_Q_BYTES_COL     12   /* algorithmic HBM bytes of one Adams column pass */
#define TDSE_Q_BYTES_ROW     13   /* algorithmic HBM bytes of one Adams row pass    */
#define TDSE_Q_PROF_MS_FAR   14   /* profiling: summed ms of tdse_far_eval's first product */
#define TDSE_Q_PROF_N_FAR    15   /* profiling: number of timed tdse_far_eval calls        */
#define TDSE_Q_MU             16  /* + j: Adams weight mu_j                    */
#define TDSE_Q_PROF_MS_RUN1D  24  /* profiling: summed ms of one-workgroup 1D runs (1D periodic FP64 plans, M <= 512) */
#define TDSE_Q_PROF_N_RUN1D   25  /* profiling: number of timed one-workgroup 1D runs */
#define TDSE_Q_PROF_MS_PERSIST 26 /* profiling: summed ms of persistent 2D launches */
#define TDSE_Q_PROF_N_PERSIST 27  /* profiling: number of timed persistent 2D launches */
#define TDSE_Q_PATH           28  /* how tdse_step marches: 0 kernel passes per step, 1 one-workgroup 1D run,
                                     2 persistent 2D launch for the Adams steps (eligible and enabled) */
#define TDSE_Q_RESIDUAL       29  /* single periodic plans, at an Adams step before T: relative L2 difference of the
                                     history entry What_n = F(V(t_n) u_n) as the plan stores it (complex64 in the
                                     split form) from its FP64 recomputation out of u_n; measures the transform
                                     precision's error injected per step (about 1e-7 split, 1e-16 FP64; the implicit
                                     solve itself is a diagonal division, Section 2.1).  Synchronizes the stream;
                                     ESTATE before the Adams start or at T, EUNSUPPORTED for batches and free space */
#define TDSE_Q_STATE_NORM     30  /* 2-norm of the state at the last guard check (TDSE_CFG_GUARD); ESTATE if none ran */
#define TDSE_Q_RICHARDSON     32  /* + l: weight of the 2^l-sub-step result    */
#define TDSE_Q_PHI            64  /* + axis: phi_axis(T)                       */
#define TDSE_Q_FS_H           80  /* free space: contour parameter H of axis 0 */
#define TDSE_Q_FS_MODES       81  /* + axis: complex-frequency modes N_axis     */
#define TDSE_Q_FS_NE          83  /* + axis: equispaced nodes per ray N_E      */
#define TDSE_Q_FS_H_AXIS      86  /* + axis: contour parameter H of that axis   */
#define TDSE_Q_FS_HSTEP      128  /* + axis: node spacing h = pi M / nu           */
#define TDSE_Q_FS_NU         130  /* + axis: FFT size nu                          */
#define TDSE_Q_FS_K          132  /* + axis: truncation K of Gamma_K (the last equispaced node is K - kappa h) */
#define TDSE_Q_FS_CHEB       134  /* + axis: terms NT of the C-type Chebyshev interpolant (0: direct sums) */
#define TDSE_Q_FS_AXIS2      136  /* + f: axis 2 of a 3D free-space plan (the keys above take axes 0 and 1):
                                     f = 0 modes, 1 N_E, 2 H, 3 h, 4 nu, 5 K, 6 NT */
#define TDSE_Q_ALPERT_X       96  /* + k: Alpert node x_k (units of h), k < p   */
#define TDSE_Q_ALPERT_W      112  /* + k: Alpert weight w_k, k < p              */
#define TDSE_Q_INSTANCES       4  /* batch: number of instances                 */
#define TDSE_Q_INST_OFFSET  4096  /* batch, + i: element offset of instance i in packed states */
#define TDSE_Q_INST_EPT_COL 8192  /* batch, + i: elements per thread of i's Adams column pass */
#define TDSE_Q_INST_EPT_ROW 12288 /* batch, + i: elements per thread of i's Adams row pass    */
int tdse_query(tdse_plan_t plan, int32_t key, double* value);

/* Plan options.  TDSE_CFG_PERSISTENT (default 1): a square 2D periodic FP64
 * plan (M = 32..512, a power of two, stored potential fields) marches its
 * implicit Adams steps in one launch of a co-resident grid (one workgroup per
 * two lines; the multistep state stays in registers and LDS, the grid
 * synchronizes between the two transform directions of each step), falling
 * back to two kernel passes per step when the device cannot hold the grid;
 * 0 always takes the passes.  Not while a run is under way (ESTATE).  The
 * persistent launch synchronizes the stream once, to check that no grid
 * barrier timed out (TDSE_EDEVICE if one did). */
#define TDSE_CFG_PERSISTENT 0
/* TDSE_CFG_GUARD (default 0, off): with value K >= 1, tdse_step marches in
 * pieces of at most K steps and after each piece, and tdse_run after the
 * run, scans the physical solution u(t) (every instance of a batch) on the
 * device for entries that are not finite and sums its squared norm
 * (TDSE_Q_STATE_NORM); a non-finite state stops the call with
 * TDSE_ENONFINITE.  Each check synchronizes the stream. */
#define TDSE_CFG_GUARD 1
int tdse_configure(tdse_plan_t plan, int32_t key, int32_t value);

/* Per-kernel timing: with enable != 0 every implicit Adams column and row
 * pass is bracketed by HIP events on the bound stream; the TDSE_Q_PROF_*
 * queries synchronize that stream and return the sums since the last call
 * with enable != 0.  enable = 0 stops recording. */
int tdse_profile(tdse_plan_t plan, int32_t enable);

/* Whole-run graph replay: with enable != 0, tdse_run captures the complete
 * step sequence of [0, T] into a hipGraph on its first call and replays it on
 * later calls (the u0 and uT copies stay outside the graph).  Needs a
 * non-default stream at tdse_bind; EINVAL otherwise.  Profiling
 * (tdse_profile) runs eagerly.  tdse_bind drops a captured graph. */
int tdse_graph(tdse_plan_t plan, int32_t enable);

/* ---- batches of independent instances ----------------------------------
 *
 * A batch plan marches `count` independent periodic problems together: at
 * every pass of the scheme (the column and row passes of Section 2.2's steps
 * and of the start-up) one launch per transform-schedule family covers the
 * lines of every instance, so a time step of the whole batch is two or a few
 * launches however many instances it holds.  The instances may differ in
 * dimension, grid, potential, field and T, but share order, nsteps,
 * n_start and precision (EINVAL otherwise); line lengths must be 2^a in
 * 64..2048 or 3 * 2^a in 192..1536 (EUNSUPPORTED otherwise).
 *
 * The batch handle takes every call above: tdse_workspace_size / tdse_bind
 * (one workspace for all instances; bind records the launch arguments of the
 * whole run into it), tdse_set_state / tdse_get_state / tdse_run with packed
 * states (instance i at element offset TDSE_Q_INST_OFFSET + i, in instance
 * order), tdse_step, tdse_graph (tdse_run replays the whole batched run),
 * tdse_profile and tdse_query (TDSE_Q_MODES: all instances' modes; keys
 * that describe one problem answer for instance 0). */
int tdse_plan_batch(const tdse_problem_t* probs, int32_t count, tdse_plan_t* out);

/* Schedule search of a bound batch plan: for each pass kind and line length,
 * every compiled schedule (elements per thread, hence lines per workgroup)
 * is timed over `reps` launches of a recorded Adams step and the fastest is
 * kept for the Adams passes.  The timing launches overwrite the state: call
 * tdse_set_state (or tdse_run) afterwards.  EUNSUPPORTED for a single plan. */
int tdse_autotune(tdse_plan_t plan, int32_t reps);

/* Set or read one instance's state (complex128, that instance's shape); a
 * batch steps once every instance has been set since its last step.  For a
 * single plan instance 0 is the plan itself. */
int tdse_set_instance_state(tdse_plan_t plan, int32_t instance, const void* u0, int32_t on_device);
int tdse_get_instance_state(tdse_plan_t plan, int32_t instance, void* u, int32_t on_device);

/* ---- field updates and the adjoint -------------------------------------
 *
 * Replace the stepwise field samples of a TDSE_A_STEPWISE plan: A_steps is
 * [nsteps][dim] (batch: every instance's block in instance order).  EINVAL
 * for other field kinds.  A captured graph is dropped; a batch re-records its
 * launch arguments. */
int tdse_set_field(tdse_plan_t plan, const double* A_steps);

/* Concurrency of a batch plan's adjoint: the instances' adjoints run from
 * `streams` host threads (1..16, default 8), each on a stream of its own with
 * a workspace slice of its own, since one instance's adjoint is a long chain
 * of small launches.  1 runs them one after another on the bound stream.
 * Call before tdse_adjoint_workspace_size (the size scales with it).  Single
 * plans accept and ignore it. */
int tdse_adjoint_streams(tdse_plan_t plan, int32_t streams);

/* Device bytes the adjoint needs with checkpoints every `checkpoint_every`
 * Adams steps (<= 0: about the square root of the step count). */
int tdse_adjoint_workspace_size(tdse_plan_t plan, int32_t checkpoint_every, size_t* bytes);

/* Reverse-mode derivative of a real objective J(u(T)) of the periodic scheme
 * with a stepwise field, for the FP64 form of the scheme (a split plan's
 * Adams passes are recomputed in FP64).  lambda_T is the adjoint seed:
 * dJ = Re sum_j conj(lambda_T,j) du_j(T) (for <x_a> = w sum x_a |u|^2 with
 * cell volume w, lambda_T = 2 w x_a u(T)).  The forward run from u0 is
 * recomputed with checkpoints every `checkpoint_every` Adams steps and the
 * scheme is then reversed step by step: every phase factor of Lemma 1
 * contributes sum_k k_a Re(conj(adjoint of its output) i E x) to
 * dJ/d(phi_a(t_b) - phi_a(t_a)), which the interval's overlap with step m
 * carries to dJ/dA_m.  Outputs: dF_dA (host, [nsteps][dim]; batch: instance
 * blocks in order) and, unless NULL, dF_du0 (dJ = Re <dF_du0, du0>; same
 * memory kind as u0).  u0, lambda_T and dF_du0 are device pointers when
 * on_device != 0, else host.  Synchronizes the bound stream; overwrites the
 * plan's state (call tdse_set_state again before stepping).  EUNSUPPORTED for
 * free-space plans or other field kinds. */
int tdse_adjoint(tdse_plan_t plan, void* adj_workspace, size_t bytes, int32_t checkpoint_every, const void* u0,
                 const void* lambda_T, int32_t on_device, double* dF_dA, void* dF_du0);

/* Release the plan (not the caller's workspace). */
void tdse_destroy(tdse_plan_t plan);

const char* tdse_status_string(int status);
const char* tdse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TDSE_H */
