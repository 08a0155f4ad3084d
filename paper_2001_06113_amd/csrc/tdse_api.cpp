// C ABI and host planner of the periodic marching scheme.
//
// The planner precomputes, in double precision on the host, every scalar the
// step kernels need: the implicit Adams weights mu_j (Section 2.2, Table 1 for
// n = 8), the iterated-Richardson weights (Section 2.2), phi(t) = int_0^t A
// (eq. (phi)) and f_r(t) at each step and sub-step time.  The step sequence
// itself is a flat list of kernel launches on the bound stream; per-step
// scalars travel as kernel arguments, so the host does no arithmetic on
// device data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tdse.h"
#include "tdse_internal.h"

using namespace tdse;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return fail(TDSE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));        \
  } while (0)

// ------------------------------------------------------------ exact weights

int64_t gcd64(int64_t a, int64_t b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Rat {
  int64_t p = 0, q = 1;
  Rat() = default;
  Rat(int64_t a, int64_t b = 1) : p(a), q(b) { norm(); }
  void norm() {
    if (q < 0) { p = -p; q = -q; }
    int64_t g = gcd64(p, q);
    if (g > 1) { p /= g; q /= g; }
  }
  Rat operator+(const Rat& o) const { return Rat(p * (o.q / gcd64(q, o.q)) + o.p * (q / gcd64(q, o.q)), q / gcd64(q, o.q) * o.q); }
  Rat operator-(const Rat& o) const { return *this + Rat(-o.p, o.q); }
  Rat operator*(const Rat& o) const { return Rat(p * o.p, q * o.q); }
  Rat operator/(const Rat& o) const { return Rat(p * o.q, q * o.p); }
  double val() const { return (double)p / (double)q; }
};

// mu_j = int_{-1}^{0} l_j(s) ds, l_j the Lagrange basis on nodes s = 0,-1,..,-(n-1)
// (the interpolant of Section 2.2 integrated exactly, in units of dt).
std::vector<double> adams_weights(int n) {
  std::vector<double> mu(n);
  for (int j = 0; j < n; ++j) {
    // numerator polynomial prod_{m != j} (s + m), coefficients c[d] of s^d
    std::vector<int64_t> c(1, 1);
    int64_t den = 1;
    for (int m = 0; m < n; ++m) {
      if (m == j) continue;
      std::vector<int64_t> nc(c.size() + 1, 0);
      for (size_t d = 0; d < c.size(); ++d) {
        nc[d] += c[d] * m;
        nc[d + 1] += c[d];
      }
      c.swap(nc);
      den *= (m - j);  // l_j(s) = prod (s + m) / prod (m - j)  with node s_j = -j
    }
    Rat acc(0);
    for (size_t d = 0; d < c.size(); ++d) {
      // int_{-1}^{0} s^d ds = (-1)^d / (d + 1)
      acc = acc + Rat(c[d] * ((d % 2) ? -1 : 1), (int64_t)d + 1);
    }
    acc = acc / Rat(den);
    mu[j] = acc.val();
  }
  return mu;
}

// Richardson: U_m^(l) = (4^m U_{m-1}^(l+1) - U_{m-1}^(l)) / (4^m - 1), folded
// into one weight per trapezoid result U_0^(l).
std::vector<double> richardson_weights(int L) {
  std::vector<std::vector<Rat>> col(L, std::vector<Rat>(L, Rat(0)));
  for (int l = 0; l < L; ++l) col[l][l] = Rat(1);
  for (int m = 1; m < L; ++m) {
    const int64_t f = (int64_t)1 << (2 * m);
    std::vector<std::vector<Rat>> nxt(L - m, std::vector<Rat>(L, Rat(0)));
    for (int l = 0; l < L - m; ++l)
      for (int b = 0; b < L; ++b) nxt[l][b] = (Rat(f) * col[l + 1][b] - col[l][b]) / Rat(f - 1);
    col.swap(nxt);
  }
  std::vector<double> w(L);
  for (int b = 0; b < L; ++b) w[b] = col[0][b].val();
  return w;
}

// ------------------------------------------------------------ Gauss-Legendre

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      long double dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    long double dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = (double)z;
    w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
  }
}

// ------------------------------------------------------------ time functions

struct TimeFns {
  int dim = 1, nV = 1, nsteps = 1;
  double dt = 1.0;
  int f_kind = TDSE_F_CONST;
  std::vector<double> f_params;
  tdse_scalar_fn f_fn = nullptr;
  void* f_ctx = nullptr;
  int A_kind = TDSE_A_NONE;
  std::vector<double> A_params;
  std::vector<double> A_steps;   // [nsteps][dim]
  std::vector<double> cum;       // phi at step boundaries [nsteps+1][dim] (stepwise, callback)
  tdse_vector_fn A_fn = nullptr;
  void* A_ctx = nullptr;
  std::vector<double> glx, glw;

  double f(int r, double t) const {
    switch (f_kind) {
      case TDSE_F_SIN: return 1.0 + f_params[2 * r] * std::sin(f_params[2 * r + 1] * t);
      case TDSE_F_CALLBACK: return f_fn(r, t, f_ctx);
      default: return 1.0;
    }
  }

  // int_0^t E0 sin^2(pi s/Tp) sin(w s) ds, with sin^2 = (1 - cos)/2 and the
  // product-to-sum identity; (1 - cos(c t))/c = 2 sin^2(c t / 2) / c.
  static double pulse_integral(double t, double E0, double w, double Tp) {
    const double Om = 2.0 * M_PI / Tp;
    auto g = [t](double c) {
      if (c == 0.0) return 0.0;
      const double s = std::sin(0.5 * c * t);
      return 2.0 * s * s / c;
    };
    return 0.5 * E0 * (g(w) - 0.5 * (g(w + Om) + g(w - Om)));
  }

  // int_0^t E0 sin^2(pi s/Tp) cos(w s) ds (the pulse of eq. (apulse)) by the
  // same identities, with int_0^t cos(c s) ds = sin(c t)/c (t at c = 0).
  static double pulse_cos_integral(double t, double E0, double w, double Tp) {
    const double Om = 2.0 * M_PI / Tp;
    auto g = [t](double c) { return c == 0.0 ? t : std::sin(c * t) / c; };
    return 0.5 * E0 * (g(w) - 0.5 * (g(w + Om) + g(w - Om)));
  }

  void A_at(double t, double* out) const {
    if (A_kind == TDSE_A_CALLBACK) {
      A_fn(t, out, A_ctx);
    } else {
      for (int a = 0; a < dim; ++a) out[a] = 0.0;
    }
  }

  void gl_piece(double a, double b, double* out) const {
    double tmp[3];
    for (int c = 0; c < dim; ++c) out[c] = 0.0;
    for (size_t i = 0; i < glx.size(); ++i) {
      const double s = 0.5 * (a + b) + 0.5 * (b - a) * glx[i];
      A_at(s, tmp);
      for (int c = 0; c < dim; ++c) out[c] += 0.5 * (b - a) * glw[i] * tmp[c];
    }
  }

  void prepare() {
    if (A_kind == TDSE_A_STEPWISE || A_kind == TDSE_A_CALLBACK) {
      if (A_kind == TDSE_A_CALLBACK) gauss_legendre(24, glx, glw);
      cum.assign((size_t)(nsteps + 1) * dim, 0.0);
      double piece[3];
      for (int m = 0; m < nsteps; ++m) {
        if (A_kind == TDSE_A_STEPWISE) {
          for (int c = 0; c < dim; ++c) piece[c] = A_steps[(size_t)m * dim + c] * dt;
        } else {
          gl_piece(m * dt, (m + 1) * dt, piece);
        }
        for (int c = 0; c < dim; ++c) cum[(size_t)(m + 1) * dim + c] = cum[(size_t)m * dim + c] + piece[c];
      }
    }
  }

  void phi(double t, double* out) const {
    for (int a = 0; a < 3; ++a) out[a] = 0.0;
    switch (A_kind) {
      case TDSE_A_PULSE_SIN2:
      case TDSE_A_PULSE_COS2: {
        const double s = A_kind == TDSE_A_PULSE_SIN2 ? pulse_integral(t, A_params[0], A_params[1], A_params[2])
                                                     : pulse_cos_integral(t, A_params[0], A_params[1], A_params[2]);
        for (int a = 0; a < dim; ++a) out[a] = s * A_params[3 + a];
        return;
      }
      case TDSE_A_STEPWISE:
      case TDSE_A_CALLBACK: {
        int m = (int)std::floor(t / dt + 1e-9);
        m = std::min(std::max(m, 0), nsteps);
        if (A_kind == TDSE_A_STEPWISE) {
          const int ms = std::min(m, nsteps - 1);
          for (int a = 0; a < dim; ++a)
            out[a] = cum[(size_t)ms * dim + a] + A_steps[(size_t)ms * dim + a] * (t - ms * dt);
        } else {
          double piece[3] = {0, 0, 0};
          if (std::fabs(t - m * dt) > 1e-15 * std::max(1.0, std::fabs(t))) gl_piece(m * dt, t, piece);
          for (int a = 0; a < dim; ++a) out[a] = cum[(size_t)m * dim + a] + piece[a];
        }
        return;
      }
      default:
        return;
    }
  }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------ plan object

// A launch recorded instead of issued (batched execution, see tdse_plan_batch).
struct RecLaunch {
  int kind;          // 0 column pass, 1 row pass, 2 complex128 -> complex64 narrowing
  int g;             // buffer stage
  bool timed;        // an implicit Adams pass (profiled)
  LineArgs a;        // passes
  const void* nsrc;  // narrowing
  void* ndst;
  int64_t nn;
};

constexpr int NFAM = 6;   // batched pass families (schedule families 0..2, phase-power rows 3..5)

struct tdse_plan_s {
  // grid: M1 x M2 (1D: M1 = 1).  A 3D grid M0 x Mmid x M2 is held as M1 =
  // M0 Mmid rows of M2: the row pass runs over the last axis, the column pass
  // over axis 0 (lines of stride Mmid M2), and the middle axis has FFT-only
  // passes of its own around every column pass.
  int dim = 1, M1 = 1, M2 = 1;
  int M0 = 1, Mmid = 0;
  int64_t P = 1;
  int order = 8, ns = 6, L = 4, nsteps = 1, nV = 1, precision = TDSE_FP64;
  double T = 1.0, dt = 1.0;
  std::vector<double> mu, rich;
  TimeFns tf;
  // Buffer sets of a "stage": the start-up always runs in FP64 (stage 0);
  // the implicit Adams steps run in the plan's precision (stage 1, the same
  // buffers as stage 0 for FP64 plans).
  struct Stage {
    int prec = P_FP64;
    size_t cplx = 16, real = 8;          // bytes of a complex / real element
    size_t o_ring = 0, o_tmp = 0, o_V = 0, o_tw1 = 0, o_tw2 = 0, o_tw3 = 0;
    std::vector<char> Vhost, tw1, tw2, tw3;   // host copies uploaded at bind (tw3: 3D middle axis)
  } st[2];
  // workspace layout
  size_t o_B = 0, o_u[2] = {0, 0}, o_ph = 0, o_ph32 = 0, total = 0;

  // ---- free space (Sections 3.4 and 4)
  bool free_space = false;
  double H = 0.0;              // contour parameter of physical axis 0
  double Hfx[3] = {0.0, 0.0, 0.0};  // per transform axis fx[a] (see fx_of)
  std::vector<double> alp_x, alp_w;   // Alpert end correction, units of h
  struct FAxis {
    int M = 1, N = 1, NE = 0, ND = 0, nu = 0;
    int NT = 0, NR = 0, NP = 0;        // interpolation nodes (0: direct C sums), dense rows, Alpert nodes per side
    double h = 0.0;
    std::vector<double2> zeta, w;      // nodes and weights, order E1 A1 C A3 E3
    std::vector<char> tables;          // pre3 pre1 ipost3 ipost1 [M], post3 post1 ipre3 ipre1 [NE],
                                       // Dfwd [NR][M], Dinv [NR][M], tw [nu], zeta [N], rfwd [NR],
                                       // w [N], Pf [N_C][NT], Pi [NT][N_C]
    size_t o_tab = 0;                  // workspace offset of the tables
  } fx[3];                            // fx[0]: axis 0 (column pass), fx[1]: the last axis (row
                                       // pass), fx[2]: the middle axis of a 3D problem
  int64_t NM = 1;                      // modes N1 N2 (3D: N0 N2 Nm)
  std::vector<double> Vsrc;            // potential fields (host copy, FP64)
  size_t o_UH[2] = {0, 0}, o_tmpf = 0, o_ringf = 0, o_Vf = 0, o_midf = 0;
  int uh_cur = 0;
  // binding and clock
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = -1;   // steps taken since set_state; -1: no state
  int ucur = 0;   // which physical buffer holds u(t_cur)
  // per-kernel event timing (tdse_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<size_t, int>> prof_marks;  // (first event index, 0 col / 1 row)

  // when set, passes are appended here instead of launched
  std::vector<RecLaunch>* rec = nullptr;

  // ---- batch of independent periodic instances (tdse_plan_batch)
  std::vector<tdse_plan_s*> sub;                // owned
  int adj_streams = 8;                          // batch adjoint: host threads / streams
  std::vector<size_t> sub_off;                  // workspace offset of each instance
  std::vector<int64_t> sub_elem;                // element offset of each instance in packed states
  struct GLaunch {
    int kind, g;
    bool timed;
    int64_t arg0;    // first of count entries in the args table (kind 0/1) or the narrowing list (kind 2)
  };
  std::vector<std::vector<GLaunch>> seg;        // [m]: step m without output (m = 1..nsteps)
  std::vector<GLaunch> seg_last;                // step nsteps with output
  std::vector<int> ucur_after;                  // [m]: physical buffer of u after step m
  std::vector<LineArgs> bargs;                  // host copy of the args table
  struct Narrow {
    const void* src;
    void* dst;
    int64_t n;
  };
  std::vector<Narrow> narrows;
  size_t o_args = 0, cap_args = 0, o_targs = 0, cap_targs = 0, o_tiles = 0;
  int64_t cap_tiles[2] = {0, 0};                // tile capacity per pass kind
  struct TileSet {
    int64_t off = 0;                            // element offset in the tile region
    // schedule families 0..2, and for row passes 3..5: the same schedules
    // for instances whose last axis carries no field (phase powers)
    int first[NFAM] = {}, cnt[NFAM] = {};
    size_t lds[NFAM] = {};
  };
  TileSet tiles[2][2];                          // [column/row][stage]
  std::vector<int> ept[2];                      // [column/row][instance]: schedule of the Adams stage
  bool batch_ready = false;                     // program recorded for the bound workspace
  size_t lds_max = 65536;                       // device limit of LDS per workgroup
  bool is_batch() const { return !sub.empty(); }

  // one-workgroup run of a 1D periodic FP64 plan (run1d_kernels.hip): the
  // per-step scalar table and the static phase factors, at the end of the
  // workspace (total_core: the workspace without them)
  bool run1d = false;
  std::vector<double> r1tab;
  std::vector<double2> r1stab;
  size_t o_r1tab = 0, o_r1stab = 0, total_core = 0;
  int64_t r1_oH = 0, r1_oR = 0, r1_oA = 0, r1_oD = 0;

  // persistent Adams steps of a square 2D periodic FP64 plan
  // (persist2d_kernels.hip): per-step scalars, static column factors and the
  // barrier words, at the end of the workspace
  bool persist = false;       // the plan qualifies
  bool persist_on = true;     // tdse_configure(TDSE_CFG_PERSISTENT)
  int persist_cap = -1;       // co-resident workgroups of the device (-1: not asked yet)
  std::vector<double> p2tab;
  std::vector<double2> p2S2;
  size_t o_p2tab = 0, o_p2S2 = 0, o_p2bar = 0;
  int64_t p2_oD2 = 0;
  bool p2_ph2 = false;
  static constexpr int P2_OSTEP = 16;

  // failure guard (tdse_configure TDSE_CFG_GUARD): check every guard_every
  // steps; diagnostics words at o_diag (two doubles and a flag); o_dbuf: an
  // FP64 mode array for the residual of periodic FP64 plans
  int guard_every = 0;
  size_t o_diag = 0, o_dbuf = 0;
  double state_norm = -1.0;

  // whole-run graph (tdse_graph): captured on the first tdse_run, replayed after
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_ucur = 0;

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
  // batch: the schedule families of one pass run concurrently, families 1
  // and 2 on side streams forked from and joined back to the bound stream
  hipStream_t fam_st[NFAM - 1] = {};
  hipEvent_t fam_fork = nullptr, fam_join[NFAM - 1] = {};

  ~tdse_plan_s() {
    drop_graph();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (int i = 0; i < NFAM - 1; ++i) {
      if (fam_join[i]) (void)hipEventDestroy(fam_join[i]);
      if (fam_st[i]) (void)hipStreamDestroy(fam_st[i]);
    }
    if (fam_fork) (void)hipEventDestroy(fam_fork);
    for (tdse_plan_s* q : sub) delete q;
  }

  double2* B() const { return (double2*)(ws + o_B); }
  double2* UH(int i) const { return (double2*)(ws + o_UH[i]); }
  void* ring(int g) const { return ws + st[g].o_ring; }
  void* ring_slot(int g, int s) const { return ws + st[g].o_ring + (size_t)s * P * st[g].cplx; }
  void* tmp(int g) const { return ws + st[g].o_tmp; }
  double2* u(int i) const { return (double2*)(ws + o_u[i]); }
  const void* V(int g) const { return ws + st[g].o_V; }
  double2* ph() const { return (double2*)(ws + o_ph); }
  float2* ph32() const { return o_ph32 ? (float2*)(ws + o_ph32) : nullptr; }
  const void* tw(int g, int axis) const {
    return ws + (axis == 0 ? st[g].o_tw1 : axis == 1 ? st[g].o_tw2 : st[g].o_tw3);
  }
  int col_len() const { return Mmid ? M0 : M1; }   // line length of the column pass
  bool force_fp64 = false;   // run the Adams passes of a split plan in FP64 (adjoint recomputation)
  bool split() const { return precision == TDSE_FP32_SPLIT && !force_fp64; }

  double t_at(int m) const { return m * dt; }
  // moving well (TDSE_V_MOVING_WELL): V0, 1/(2 beta^2), velocity per axis
  int vkind = TDSE_V_FIELDS;
  double well[4] = {0.0, 0.0, 0.0, 0.0};
  double well_k = 0.0;
  int64_t nsamp = 0;   // TDSE_V_SAMPLED: samples V(., t_n), n = 0..nsteps
  // V(., t) as a weighted sum of stored fields: weights f[0..k) (k returned)
  // of the fields starting at field *first.  Sampled V: the sample at a step
  // time; elsewhere the degree-7 Lagrange interpolant through the eight
  // samples n0..n0+7, n0 = clamp(floor(t/dt) - 3, 0, nsteps - 7) (every
  // sample when nsteps < 7); a time within 1e-9 dt of a step time is that
  // step time.
  int V_window(double t, double* f, int64_t* first) const {
    if (vkind != TDSE_V_SAMPLED) {
      fV_at(t, f);
      *first = 0;
      return nV;
    }
    for (int r = 0; r < MAXV; ++r) f[r] = 0.0;
    const double sv = t / dt;
    const double nr = std::nearbyint(sv);
    if (std::fabs(sv - nr) < 1e-9 && nr >= 0.0 && nr <= (double)nsteps) {
      f[0] = 1.0;
      *first = (int64_t)nr;
      return 1;
    }
    const int count = std::min(MAXV, nsteps + 1);
    int64_t n0 = (int64_t)std::floor(sv) - (count / 2 - 1);
    n0 = std::min<int64_t>(std::max<int64_t>(n0, 0), (int64_t)nsteps + 1 - count);
    for (int i = 0; i < count; ++i) {
      double w = 1.0;
      for (int j = 0; j < count; ++j)
        if (j != i) w *= (sv - (double)(n0 + j)) / (double)(i - j);
      f[i] = w;
    }
    *first = n0;
    return count;
  }
  void fV_at(double t, double* f) const {
    for (int r = 0; r < MAXV; ++r) f[r] = r < nV ? tf.f(r, t) : 0.0;
    if (vkind == TDSE_V_MOVING_WELL) {
      // the centre c t, wrapped into [-pi, pi) (V is 2 pi periodic in it)
      auto wrap = [](double x) { return x - 2.0 * M_PI * std::floor((x + M_PI) / (2.0 * M_PI)); };
      f[0] = -well[0];
      f[1] = well[1];
      f[2] = dim == 2 ? wrap(well[2] * t) : 0.0;
      f[3] = wrap((dim == 2 ? well[3] : well[2]) * t);
      f[4] = well_k;   // periodic images per side that can lie within 9.2 beta of a point
    }
  }
};

namespace {

// tw[m] = exp(-2 pi i m / N) from extended precision, rounded once to the
// transform precision
std::vector<char> twiddles(int N, bool split) {
  const int n = std::max(N, 1);
  std::vector<char> tw(n * (split ? sizeof(float2) : sizeof(double2)));
  for (int m = 0; m < N; ++m) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
    if (split) ((float2*)tw.data())[m] = float2{(float)cosl(a), (float)sinl(a)};
    else ((double2*)tw.data())[m] = double2{(double)cosl(a), (double)sinl(a)};
  }
  return tw;
}

LineArgs base_args(const tdse_plan_s* p, int g) {
  LineArgs a;
  std::memset(&a, 0, sizeof(a));
  a.M1 = p->M1;
  a.M2 = p->M2;
  a.M0 = p->M0;
  a.Mmid = p->Mmid;
  a.V = p->V(g);
  a.nV = p->nV;
  a.vkind = p->vkind;
  a.vstride = p->P;
  a.scale = 1.0 / (double)p->P;
  a.ring = p->ring(g);
  a.ring_stride = p->P;
  a.Bm = p->B();
  a.ph = p->ph();
  a.ph32 = p->ph32();
  a.slot_w = -1;
  return a;
}

// the potential of a pass at time t: weights, and for a sampled V the window
// of samples (a.V moved to its first sample, a.nV its length)
void set_V(const tdse_plan_s* p, int g, LineArgs& a, double t) {
  int64_t first = 0;
  const int k = p->V_window(t, a.fV, &first);
  if (p->vkind == TDSE_V_SAMPLED) {
    a.V = (const char*)p->V(g) + first * p->P * (int64_t)sizeof(double);
    a.nV = k;
  }
}

// column-pass geometry: lines are the M2 columns, elements step by M2 (3D:
// the Mmid M2 lines along axis 0)
void col_geom(const tdse_plan_s* p, int g, LineArgs& a) {
  const int64_t w = p->Mmid ? (int64_t)p->Mmid * p->M2 : p->M2;
  a.line_stride = 1;
  a.elem_stride = w;
  a.nlines = (int)w;
  a.tw = p->tw(g, 0);
}
void row_geom(const tdse_plan_s* p, int g, LineArgs& a) {
  a.line_stride = p->M2;
  a.elem_stride = 1;
  a.nlines = p->M1;
  a.tw = p->tw(g, 1);
}

// phase request for E^(j) at t_b, j = 1..nj, over intervals of length j*tau
void phase_req(const tdse_plan_s* p, LineArgs& a, int nj, double t_b, double tau, bool stepgrid, int m_b) {
  a.req.nj = nj;
  double pb[3], pa[3];
  if (stepgrid) p->tf.phi(p->t_at(m_b), pb);
  else p->tf.phi(t_b, pb);
  for (int j = 1; j <= nj; ++j) {
    if (stepgrid) p->tf.phi(p->t_at(m_b - j), pa);
    else p->tf.phi(t_b - j * tau, pa);
    a.req.tau[j - 1] = j * tau;
    if (p->dim == 3) {
      a.req.dphi0[j - 1] = pb[0] - pa[0];
      a.req.dphi1[j - 1] = pb[1] - pa[1];
      a.req.dphi2[j - 1] = pb[2] - pa[2];
    } else if (p->dim == 2) {
      a.req.dphi1[j - 1] = pb[0] - pa[0];
      a.req.dphi2[j - 1] = pb[1] - pa[1];
    } else {
      a.req.dphi1[j - 1] = 0.0;
      a.req.dphi2[j - 1] = pb[0] - pa[0];
    }
  }
}

// FFT-only pass along the middle axis of a 3D grid, in place on buf: lines
// (i0, i2) of Mmid elements at stride M2, slabs of M2 lines per i0
int launch_mid(const tdse_plan_s* p, int g, void* buf, bool inverse, hipEvent_t e0, hipEvent_t e1) {
  LineArgs m;
  std::memset(&m, 0, sizeof(m));
  m.M1 = p->M1;
  m.M2 = p->M2;
  m.M0 = p->M0;
  m.Mmid = p->Mmid;
  m.src = buf;
  m.dst = buf;
  m.line_stride = 1;
  m.elem_stride = p->M2;
  m.nlines = p->M0 * p->M2;
  m.slab_lines = p->M2;
  m.slab_stride = (int64_t)p->Mmid * p->M2;
  m.tw = p->tw(g, 2);
  const hipError_t e = launch_mid_pass(p->st[g].prec, p->Mmid, inverse, m, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return TDSE_OK;
}

hipEvent_t next_event(tdse_plan_s* p);

// 3D: the middle-axis pass, timed (kind 5) when profiling
int launch_mid_timed(const tdse_plan_s* p, int g, void* buf, bool inverse) {
  tdse_plan_s* q = const_cast<tdse_plan_s*>(p);
  if (!q->prof) return launch_mid(p, g, buf, inverse, nullptr, nullptr);
  const size_t first = q->ev_used;
  hipEvent_t e0 = next_event(q), e1 = next_event(q);
  if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  const int s = launch_mid(p, g, buf, inverse, e0, e1);
  if (s) return s;
  q->prof_marks.push_back({first, 5});
  return TDSE_OK;
}

int launch(const tdse_plan_s* p, int g, bool col, const LineArgs& a, hipEvent_t e0 = nullptr,
           hipEvent_t e1 = nullptr) {
  if (p->rec) {
    p->rec->push_back(RecLaunch{col ? 0 : 1, g, e0 != nullptr, a, nullptr, nullptr, 0});
    return TDSE_OK;
  }
  const int prec = p->st[g].prec;
  // 3D: the column pass sees the tile transformed along axis 0 only, so the
  // middle axis is inverted before a solve and transformed forward after it
  if (col && p->Mmid && a.mode == C_SOLVE) {
    const int s = launch_mid_timed(p, g, const_cast<void*>(a.src), true);
    if (s) return s;
  }
  hipError_t e = col ? launch_col_pass(prec, p->col_len(), a, p->stream, e0, e1)
                     : launch_row_pass(prec, p->M2, a, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  if (col && p->Mmid) return launch_mid_timed(p, g, a.dst, false);
  return TDSE_OK;
}

hipEvent_t next_event(tdse_plan_s* p) {
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->ev_pool.push_back(e);
  }
  return p->ev_pool[p->ev_used++];
}

// launch an implicit Adams pass; when profiling, the dispatch itself records
// events at the kernel's start and end
int launch_timed(tdse_plan_s* p, int g, bool col, const LineArgs& a) {
  if (p->rec) {
    p->rec->push_back(RecLaunch{col ? 0 : 1, g, true, a, nullptr, nullptr, 0});
    return TDSE_OK;
  }
  if (!p->prof) return launch(p, g, col, a);
  const size_t first = p->ev_used;
  hipEvent_t e0 = next_event(p), e1 = next_event(p);
  if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  int s = launch(p, g, col, a, e0, e1);
  if (s) return s;
  p->prof_marks.push_back({first, col ? 0 : 1});
  return TDSE_OK;
}

// What_m = F(V(t_m) u_m) into ring slot m mod (n-1) (start-up stage, FP64)
int op_history(tdse_plan_s* p, int m) {
  const int g = 0;
  LineArgs a = base_args(p, g);
  col_geom(p, g, a);
  a.mode = C_FWD;
  a.src = p->u(p->ucur);
  a.dst = p->tmp(g);
  set_V(p, g, a, p->t_at(m));
  a.alpha_re = 0.0; a.alpha_im = 0.0; a.beta_re = 1.0; a.beta_im = 0.0;
  int s = launch(p, g, true, a);
  if (s) return s;
  LineArgs r = base_args(p, g);
  row_geom(p, g, r);
  r.mode = R_FWD;
  r.src = p->tmp(g);
  r.fdst = p->ring_slot(g, m % (p->order - 1));
  return launch(p, g, false, r);
}

// One iterated-Richardson start-up step from t_{m-1} to t_m (FP64).
int op_richardson(tdse_plan_s* p, int m) {
  const int g = 0;
  const double t = p->t_at(m - 1);
  const int src = p->ucur, acc = 1 - p->ucur;
  for (int l = 0; l < p->L; ++l) {
    const int nsub = 1 << l;
    const double delta = p->dt / nsub;
    // B = P F((1 - i delta/2 V(t)) u)
    LineArgs a = base_args(p, g);
    col_geom(p, g, a);
    a.mode = C_FWD;
    a.src = p->u(src);
    a.dst = p->tmp(g);
    set_V(p, g, a, t);
    a.alpha_re = 1.0; a.alpha_im = 0.0; a.beta_re = 0.0; a.beta_im = -0.5 * delta;
    phase_req(p, a, 1, t + delta, delta, false, 0);
    int s = launch(p, g, true, a);
    if (s) return s;
    LineArgs r = base_args(p, g);
    row_geom(p, g, r);
    r.mode = R_INIT;
    r.src = p->tmp(g);
    r.dst = p->tmp(g);
    s = launch(p, g, false, r);
    if (s) return s;
    for (int k = 0; k < nsub; ++k) {
      const double ts = t + k * delta;
      const double ts1 = ts + delta;
      const bool last = (k == nsub - 1);
      LineArgs c = base_args(p, g);
      col_geom(p, g, c);
      c.mode = C_SOLVE;
      c.src = p->tmp(g);
      c.dst = p->tmp(g);
      set_V(p, g, c, ts1);
      c.csolve = 0.5 * delta;
      if (last) {
        c.uacc = p->u(acc);
        c.wacc = p->rich[l];
        c.acc_first = (l == 0);
      } else {
        phase_req(p, c, 1, ts1 + delta, delta, false, 0);
      }
      s = launch(p, g, true, c);
      if (s) return s;
      if (!last) {
        LineArgs rr = base_args(p, g);
        row_geom(p, g, rr);
        rr.mode = R_AM;
        rr.src = p->tmp(g);
        rr.dst = p->tmp(g);
        rr.nh = 1;
        rr.c0 = 0.5 * delta;
        rr.ch[1] = 0.5 * delta;
        rr.slot_w = -1;
        s = launch(p, g, false, rr);
        if (s) return s;
      }
    }
  }
  p->ucur = acc;
  return TDSE_OK;
}

// B_{ns+1} from uhat_ns = F u_ns and the history What_0..What_ns (FP64); a
// split plan then narrows the history ring and the tile buffer to complex64.
int op_am_init(tdse_plan_s* p) {
  const int n = p->order, m = p->ns, g = 0;
  LineArgs a = base_args(p, g);
  col_geom(p, g, a);
  a.mode = C_FWD;
  a.src = p->u(p->ucur);
  a.dst = p->tmp(g);
  a.alpha_re = 1.0; a.alpha_im = 0.0; a.beta_re = 0.0; a.beta_im = 0.0;
  phase_req(p, a, n - 1, 0.0, p->dt, true, m + 1);
  int s = launch(p, g, true, a);
  if (s) return s;
  LineArgs r = base_args(p, g);
  row_geom(p, g, r);
  r.mode = R_FORM;
  r.src = p->tmp(g);
  r.dst = p->tmp(g);
  r.nh = n - 1;
  for (int j = 1; j <= n - 1; ++j) {
    r.slot_r[j] = (m + 1 - j) % (n - 1);
    r.ch[j] = p->dt * p->mu[j];
  }
  s = launch(p, g, false, r);
  if (s) return s;
  if (p->split() && p->rec) {
    p->rec->push_back(RecLaunch{2, 0, false, LineArgs{}, p->ring(0), p->ring(1), (int64_t)(n - 1) * p->P});
    p->rec->push_back(RecLaunch{2, 0, false, LineArgs{}, p->tmp(0), p->tmp(1), p->P});
  } else if (p->split()) {
    hipError_t e = launch_narrow((const double2*)p->ring(0), (float2*)p->ring(1), (int64_t)(n - 1) * p->P, p->stream);
    if (e == hipSuccess) e = launch_narrow((const double2*)p->tmp(0), (float2*)p->tmp(1), p->P, p->stream);
    if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("narrow: ") + hipGetErrorString(e));
  }
  return TDSE_OK;
}

// u_m = F^-1 B_m / (1 + i mu_0 dt V(t_m)) in FP64 from the FP64 state B
// (output of a split plan).
int op_fp64_output(tdse_plan_s* p, int m) {
  const int g = 0;
  LineArgs r = base_args(p, g);
  row_geom(p, g, r);
  r.mode = R_INV;
  r.dst = p->tmp(g);
  int s = launch(p, g, false, r);
  if (s) return s;
  LineArgs c = base_args(p, g);
  col_geom(p, g, c);
  c.mode = C_SOLVE;
  c.src = p->tmp(g);
  c.dst = p->tmp(g);
  set_V(p, g, c, p->t_at(m));
  c.csolve = p->mu[0] * p->dt;
  c.uout = p->u(p->ucur);
  return launch(p, g, true, c);
}

// Implicit Adams step m (eq. (uadamsk)), stage 1.
int op_am_step(tdse_plan_s* p, int m, bool write_u) {
  const int n = p->order, g = p->split() ? 1 : 0;
  if (write_u && p->split()) {
    int s = op_fp64_output(p, m);
    if (s) return s;
    write_u = false;
  }
  if (m == p->nsteps && !write_u && p->split()) return TDSE_OK;
  LineArgs c = base_args(p, g);
  col_geom(p, g, c);
  c.mode = C_SOLVE;
  c.src = p->tmp(g);
  c.dst = p->tmp(g);
  set_V(p, g, c, p->t_at(m));
  c.csolve = p->mu[0] * p->dt;
  if (write_u) c.uout = p->u(p->ucur);
  if (m < p->nsteps) phase_req(p, c, n - 1, 0.0, p->dt, true, m + 1);
  int s = launch_timed(p, g, true, c);
  if (s) return s;
  if (m == p->nsteps) return TDSE_OK;
  LineArgs r = base_args(p, g);
  row_geom(p, g, r);
  r.mode = R_AM;
  r.src = p->tmp(g);
  r.dst = p->tmp(g);
  r.nh = n - 1;
  r.c0 = p->mu[0] * p->dt;
  r.slot_w = m % (n - 1);
  for (int j = 1; j <= n - 1; ++j) {
    r.ch[j] = p->dt * p->mu[j];
    r.slot_r[j] = ((m + 1 - j) % (n - 1) + (n - 1)) % (n - 1);
  }
  // no field component along the last axis: its factors of E^(j) are the
  // j-th powers of E^(1)'s
  r.pf_pow = 1;
  for (int j = 0; j < n - 1; ++j)
    if (c.req.dphi2[j] != 0.0) r.pf_pow = 0;
  return launch_timed(p, g, false, r);
}


// ============================================================== free space

// Alpert end correction (Section 3.4; the table itself is only cited there):
// the p-point Gauss rule of the functional
//   Lambda[f] = sum_{k<kappa} f(k) + sum_m (B_{m+1}/(m+1)) f^(m)(0)/m!,
// whose moments Lambda[x^m] = B_{m+1}(kappa)/(m+1) make the corrected
// trapezoid rule exact on x^m, m < 2p.  Recurrence coefficients by Gautschi's
// modified Chebyshev algorithm on monic Legendre polynomials of [0, kappa],
// nodes and weights from the Jacobi matrix (Golub-Welsch), all in long double.
void alpert_rule(int p, int kappa, std::vector<double>& xo, std::vector<double>& wo) {
  typedef long double LD;
  const int n2 = 2 * p;
  std::vector<LD> B(n2 + 2, 0.0L);
  B[0] = 1.0L;
  for (int m = 1; m <= n2 + 1; ++m) {
    LD sum = 0.0L, binom = 1.0L;   // C(m+1, k)
    for (int k = 0; k < m; ++k) {
      sum += binom * B[k];
      binom = binom * (LD)(m + 1 - k) / (LD)(k + 1);
    }
    B[m] = -sum / (LD)(m + 1);
  }
  const LD c = (LD)kappa;
  std::vector<LD> a(n2 + 1), b(n2 + 1);
  for (int l = 0; l <= n2; ++l) {
    a[l] = c / 2;
    b[l] = l == 0 ? 0.0L : (c / 2) * (c / 2) * (LD)l * l / (4.0L * l * l - 1.0L);
  }
  // pi_l: monomial coefficients d[l][m] and values at the integers k < kappa
  std::vector<std::vector<LD>> d(n2 + 1, std::vector<LD>(n2 + 1, 0.0L));
  std::vector<std::vector<LD>> val(n2 + 1, std::vector<LD>(kappa, 0.0L));
  d[0][0] = 1.0L;
  for (int k = 0; k < kappa; ++k) val[0][k] = 1.0L;
  for (int l = 0; l + 1 <= n2; ++l) {
    for (int m = 0; m <= l + 1; ++m) {
      LD v = (m >= 1 ? d[l][m - 1] : 0.0L) - a[l] * d[l][m];
      if (l >= 1) v -= b[l] * d[l - 1][m];
      d[l + 1][m] = v;
    }
    for (int k = 0; k < kappa; ++k)
      val[l + 1][k] = ((LD)k - a[l]) * val[l][k] - (l >= 1 ? b[l] * val[l - 1][k] : 0.0L);
  }
  std::vector<LD> nu(n2);
  for (int l = 0; l < n2; ++l) {
    LD s = 0.0L;
    for (int k = 0; k < kappa; ++k) s += val[l][k];
    for (int m = 0; m <= l; ++m) s += d[l][m] * B[m + 1] / (LD)(m + 1);
    nu[l] = s;
  }
  // modified Chebyshev algorithm
  std::vector<LD> alpha(p), beta(p);
  std::vector<LD> sm1(n2, 0.0L), s0(nu), s1(n2, 0.0L);
  alpha[0] = a[0] + nu[1] / nu[0];
  beta[0] = nu[0];
  for (int k = 1; k < p; ++k) {
    for (int l = k; l <= n2 - k - 1; ++l)
      s1[l] = s0[l + 1] - (alpha[k - 1] - a[l]) * s0[l] - beta[k - 1] * sm1[l] + b[l] * s0[l - 1];
    alpha[k] = a[k] + s1[k + 1] / s1[k] - s0[k] / s0[k - 1];
    beta[k] = s1[k] / s0[k - 1];
    sm1 = s0;
    s0 = s1;
  }
  // symmetric Jacobi matrix, cyclic Jacobi rotations with eigenvectors
  std::vector<std::vector<LD>> J(p, std::vector<LD>(p, 0.0L)), Vv(p, std::vector<LD>(p, 0.0L));
  for (int k = 0; k < p; ++k) {
    J[k][k] = alpha[k];
    if (k + 1 < p) J[k][k + 1] = J[k + 1][k] = std::sqrt(beta[k + 1]);
    Vv[k][k] = 1.0L;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    LD off = 0.0L;
    for (int i = 0; i < p; ++i)
      for (int j = i + 1; j < p; ++j) off += J[i][j] * J[i][j];
    if (off < 1e-36L) break;
    for (int i = 0; i < p; ++i)
      for (int j = i + 1; j < p; ++j) {
        if (std::fabs(J[i][j]) < 1e-40L) continue;
        const LD tau = (J[j][j] - J[i][i]) / (2.0L * J[i][j]);
        const LD t = (tau >= 0 ? 1.0L : -1.0L) / (std::fabs(tau) + std::sqrt(1.0L + tau * tau));
        const LD cs = 1.0L / std::sqrt(1.0L + t * t), sn = t * cs;
        for (int k = 0; k < p; ++k) {
          const LD jik = J[i][k], jjk = J[j][k];
          J[i][k] = cs * jik - sn * jjk;
          J[j][k] = sn * jik + cs * jjk;
        }
        for (int k = 0; k < p; ++k) {
          const LD jki = J[k][i], jkj = J[k][j];
          J[k][i] = cs * jki - sn * jkj;
          J[k][j] = sn * jki + cs * jkj;
        }
        for (int k = 0; k < p; ++k) {
          const LD vki = Vv[k][i], vkj = Vv[k][j];
          Vv[k][i] = cs * vki - sn * vkj;
          Vv[k][j] = sn * vki + cs * vkj;
        }
      }
  }
  std::vector<std::pair<LD, LD>> nw(p);
  for (int k = 0; k < p; ++k) nw[k] = {J[k][k], beta[0] * Vv[0][k] * Vv[0][k]};
  std::sort(nw.begin(), nw.end());
  xo.resize(p);
  wo.resize(p);
  for (int k = 0; k < p; ++k) {
    xo[k] = (double)nw[k].first;
    wo[k] = (double)nw[k].second;
  }
}

inline double2 cexp_ld(long double re, long double im) {
  const long double m = std::exp(re);
  return double2{(double)(m * std::cos(im)), (double)(m * std::sin(im))};
}

// Terms of the Chebyshev interpolant of tau -> exp(-/+ (1 + i) tau x) on
// [-H, H], |x| <= 1 (Section 4.1, eqs. (expintrpm), (expintrpp)).  Its
// Chebyshev coefficients are 2 I_l(z) with |z| <= sqrt(2) H and
// |I_l(z)| <= I_l(|z|); interpolation at most doubles the tail, so NT is the
// smallest count with 4 sum_{l >= NT} I_l(sqrt(2) H) <= 2^-52: the
// interpolant is exact to rounding.  I_l by its power series in long double.
int cheb_terms(double H) {
  typedef long double LD;
  const LD r = std::sqrt(2.0L) * (LD)H, h2 = r * r / 4.0L;
  auto bessel_i = [&](int l) {
    LD lead = 1.0L;   // (r/2)^l / l!
    for (int k = 1; k <= l; ++k) lead *= (r / 2.0L) / (LD)k;
    LD term = lead, sum = lead;
    for (int m = 1; m < 400 && term > 1e-40L * sum; ++m) {
      term *= h2 / ((LD)m * (LD)(l + m));
      sum += term;
    }
    return sum;
  };
  for (int n = 2; n <= FS_CHEB_MAX; ++n) {
    LD tail = 0.0L;
    for (int l = n; l < n + 60; ++l) tail += bessel_i(l);
    if (4.0L * tail <= std::ldexp(1.0L, -52)) return n;
  }
  return 0;   // more than FS_CHEB_MAX terms
}

// Nodes, weights and transform tables of one axis (Sections 3.4 and 4.1).
// cheb: 0 automatic (the interpolant when it has fewer terms than Gamma_2 has
// nodes), -1 direct C sums, n > 0 the interpolant with n terms.
// transform axis fx[] of physical axis a: 1D: the row axis fx[1]; 2D: fx[a];
// 3D: axis 0 -> fx[0], the middle axis -> fx[2], the last axis -> fx[1]
int fx_of(int dim, int a) {
  if (dim == 1) return 1;
  if (dim == 2) return a;
  return a == 0 ? 0 : (a == 1 ? 2 : 1);
}

void plan_free_axis(tdse_plan_s* p, int axis, int M, int nu, int q, int panels, int cheb) {
  typedef long double LD;
  tdse_plan_s::FAxis& F = p->fx[axis];
  const int kappa = 7, pp = (int)p->alp_x.size();
  const LD H = p->Hfx[axis];
  const LD PI = 3.14159265358979323846264338327950288L;
  F.M = M;
  F.nu = nu;
  F.NE = nu / 2 - 2 * kappa + 1;
  F.h = (double)(PI * M / nu);
  const LD h = PI * (LD)M / (LD)nu;
  // Gamma_2 panels: dyadic toward 0, `panels` per side
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  std::vector<LD> tc, wc;
  for (int k = 1; k <= panels; ++k) {
    const LD lo = k == 1 ? 0.0L : H / std::pow(2.0L, (LD)(panels - k + 1));
    const LD hi = H / std::pow(2.0L, (LD)(panels - k));
    for (int j = 0; j < q; ++j) {
      // Gauss-Legendre nodes come in descending order from gauss_legendre
      const int jj = q - 1 - j;
      tc.push_back(0.5L * (hi - lo) * gx[jj] + 0.5L * (hi + lo));
      wc.push_back(0.5L * (hi - lo) * gw[jj]);
    }
  }
  const int half = (int)tc.size();
  F.ND = 2 * pp + 2 * half;
  F.N = 2 * F.NE + F.ND;
  F.zeta.assign(F.N, double2{0, 0});
  F.w.assign(F.N, double2{0, 0});
  // E1 (mirror of E3), A1 (mirror of A3), C (-H..H), A3, E3
  for (int e = 0; e < F.NE; ++e) {
    const LD tau = H + kappa * h + e * h;
    F.zeta[F.N - F.NE + e] = double2{(double)tau, (double)-H};
    F.w[F.N - F.NE + e] = double2{(double)h, 0.0};
    F.zeta[F.NE - 1 - e] = double2{(double)-tau, (double)H};
    F.w[F.NE - 1 - e] = double2{(double)h, 0.0};
  }
  for (int k = 0; k < pp; ++k) {
    const LD tau = H + (LD)p->alp_x[k] * h;
    const int i3 = F.NE + pp + 2 * half + k, i1 = F.NE + pp - 1 - k;
    F.zeta[i3] = double2{(double)tau, (double)-H};
    F.w[i3] = double2{(double)(h * (LD)p->alp_w[k]), 0.0};
    F.zeta[i1] = double2{(double)-tau, (double)H};
    F.w[i1] = double2{(double)(h * (LD)p->alp_w[k]), 0.0};
  }
  for (int k = 0; k < half; ++k) {
    // zeta = (1 - i) tau, weight (1 - i) w
    const int ip = F.NE + pp + half + k, im = F.NE + pp + half - 1 - k;
    F.zeta[ip] = double2{(double)tc[k], (double)-tc[k]};
    F.w[ip] = double2{(double)wc[k], (double)-wc[k]};
    F.zeta[im] = double2{(double)-tc[k], (double)tc[k]};
    F.w[im] = double2{(double)wc[k], (double)-wc[k]};
  }
  // C-type block: direct sums, or the interpolant through NT nodes
  const int NC = 2 * half;
  F.NP = pp;
  F.NT = 0;
  if (cheb > 0) {
    F.NT = cheb;
  } else if (cheb == 0) {
    const int nt = cheb_terms((double)H);
    F.NT = (nt > 0 && nt < NC) ? nt : 0;
  }
  F.NR = F.NT ? 2 * pp + F.NT : F.ND;
  // dense rows r: A1 nodes, interpolation nodes (1 - i) H s_m (s_m the
  // Chebyshev points of the first kind), A3 nodes; without the interpolant
  // every dense mode is a row
  std::vector<double2> rz(F.NR), rw(F.NR);
  std::vector<LD> sm(F.NT);
  for (int r = 0; r < F.NR; ++r) {
    if (!F.NT || r < pp) {
      rz[r] = F.zeta[F.NE + r];
      rw[r] = F.w[F.NE + r];
    } else if (r >= pp + F.NT) {
      rz[r] = F.zeta[F.NE + r - F.NT + NC];
      rw[r] = F.w[F.NE + r - F.NT + NC];
    } else {
      const int m = r - pp;
      sm[m] = std::cos(PI * ((LD)m + 0.5L) / (LD)F.NT);
      rz[r] = double2{(double)(H * sm[m]), (double)(-H * sm[m])};
      rw[r] = double2{2.0 * PI, 0.0};   // no weight: 2 pi cancels the inverse's 1/(2 pi)
    }
  }
  // P[k][m] = (1/NT) sum_l c_l T_l(tau_k / H) T_l(s_m), c_0 = 1, c_l = 2: the
  // interpolant's value at the C-node tau_k from its values at the nodes
  std::vector<double2> Pf((size_t)(NC * F.NT + 1) / 2), Pi((size_t)F.NT * NC);
  for (int k = 0; k < NC && F.NT; ++k) {
    const LD sk = (LD)F.zeta[F.NE + pp + k].x / H;
    for (int m = 0; m < F.NT; ++m) {
      LD t0a = 1.0L, t1a = sk, t0b = 1.0L, t1b = sm[m];
      LD acc = 1.0L;
      for (int l = 1; l < F.NT; ++l) {
        acc += 2.0L * t1a * t1b;
        const LD t2a = 2.0L * sk * t1a - t0a, t2b = 2.0L * sm[m] * t1b - t0b;
        t0a = t1a; t1a = t2a; t0b = t1b; t1b = t2b;
      }
      const LD P = acc / (LD)F.NT;
      ((double*)Pf.data())[(size_t)k * F.NT + m] = (double)P;
      const double2 wk = F.w[F.NE + pp + k];
      Pi[(size_t)m * NC + k] = double2{(double)(P * (LD)wk.x / (2.0L * PI)), (double)(P * (LD)wk.y / (2.0L * PI))};
    }
  }
  // transform tables
  const int NE = F.NE, ND = F.NR;
  const LD alpha = H + kappa * h;
  const LD s2M = 2.0L / (LD)M;
  std::vector<double2> pre3(M), pre1(M), ipost3(M), ipost1(M), post3(NE), post1(NE), ipre3(NE), ipre1(NE);
  std::vector<double2> Dfwd((size_t)ND * M), Dinv((size_t)M * ND), twt(nu), z(F.zeta);
  for (int j = 0; j < M; ++j) {
    const LD x = -1.0L + 2.0L * j / (LD)M;
    const LD ph = 2.0L * alpha * j / (LD)M;
    pre3[j] = cexp_ld(-H * x, -ph);
    pre1[j] = cexp_ld(H * x, ph);
    ipost3[j] = cexp_ld(H * x, -alpha + ph);
    ipost1[j] = cexp_ld(-H * x, alpha - ph);
  }
  for (int e = 0; e < NE; ++e) {
    const LD eh = e * h;
    const double2 a3 = cexp_ld(0.0L, alpha + eh), a1 = cexp_ld(0.0L, -alpha - eh);
    post3[e] = double2{(double)(s2M * a3.x), (double)(s2M * a3.y)};
    post1[e] = double2{(double)(s2M * a1.x), (double)(s2M * a1.y)};
    const LD wf = h / (2.0L * PI);
    const double2 b3 = cexp_ld(0.0L, -eh), b1 = cexp_ld(0.0L, eh);
    ipre3[e] = double2{(double)(wf * b3.x), (double)(wf * b3.y)};
    ipre1[e] = double2{(double)(wf * b1.x), (double)(wf * b1.y)};
  }
  for (int q2 = 0; q2 < ND; ++q2) {
    const double2 zz = rz[q2], ww = rw[q2];
    for (int j = 0; j < M; ++j) {
      const LD x = -1.0L + 2.0L * j / (LD)M;
      // exp(-i zeta x) = exp(Im(zeta) x) exp(-i Re(zeta) x)
      const double2 ef = cexp_ld((LD)zz.y * x, -(LD)zz.x * x);
      Dfwd[(size_t)q2 * M + j] = double2{(double)(s2M * ef.x), (double)(s2M * ef.y)};
      const double2 eb = cexp_ld(-(LD)zz.y * x, (LD)zz.x * x);
      const LD wr = (LD)ww.x / (2.0L * PI), wi = (LD)ww.y / (2.0L * PI);
      Dinv[(size_t)q2 * M + j] = double2{(double)(wr * eb.x - wi * eb.y), (double)(wr * eb.y + wi * eb.x)};
    }
  }
  for (int m = 0; m < nu; ++m) {
    const LD a = -2.0L * PI * (LD)m / (LD)nu;
    twt[m] = double2{(double)std::cos(a), (double)std::sin(a)};
  }
  // ratio of consecutive forward dense entries: Dfwd[q][j+1] = Dfwd[q][j] exp(-i zeta_q 2/M)
  std::vector<double2> rfwd(ND);
  for (int q2 = 0; q2 < ND; ++q2) {
    const double2 zz = rz[q2];
    rfwd[q2] = cexp_ld((LD)zz.y * 2.0L / (LD)M, -(LD)zz.x * 2.0L / (LD)M);
  }
  std::vector<double2> wv(F.w);
  std::vector<std::vector<double2>*> parts = {&pre3, &pre1, &ipost3, &ipost1, &post3, &post1, &ipre3, &ipre1,
                                              &Dfwd, &Dinv, &twt, &z, &rfwd, &wv, &Pf, &Pi};
  size_t bytes = 0;
  for (auto* v : parts) bytes = align256(bytes + v->size() * sizeof(double2));
  F.tables.assign(bytes, 0);
  size_t off = 0;
  for (auto* v : parts) {
    if (!v->empty()) std::memcpy(F.tables.data() + off, v->data(), v->size() * sizeof(double2));
    off = align256(off + v->size() * sizeof(double2));
  }
}

// device view of axis a's tables
CFAxis cf_axis(const tdse_plan_s* p, int axis) {
  const tdse_plan_s::FAxis& F = p->fx[axis];
  CFAxis c;
  std::memset(&c, 0, sizeof(c));
  c.M = F.M;
  c.N = F.N;
  c.NE = F.NE;
  c.ND = F.ND;
  c.NR = F.NR;
  c.NT = F.NT;
  c.NP = F.NP;
  if (F.nu == 0) {   // axis without transform (1D problem): one mode at zeta = 0
    c.zeta = (const double2*)(p->ws + F.o_tab);
    return c;
  }
  const double2* base = (const double2*)(p->ws + F.o_tab);
  size_t off = 0;
  auto take = [&](size_t n) {
    const double2* q = (const double2*)((const char*)base + off);
    off = align256(off + n * sizeof(double2));
    return q;
  };
  c.pre3 = take(F.M);
  c.pre1 = take(F.M);
  c.ipost3 = take(F.M);
  c.ipost1 = take(F.M);
  c.post3 = take(F.NE);
  c.post1 = take(F.NE);
  c.ipre3 = take(F.NE);
  c.ipre1 = take(F.NE);
  c.Dfwd = take((size_t)F.NR * F.M);
  c.Dinv = take((size_t)F.M * F.NR);
  c.tw = take(F.nu);
  c.zeta = take(F.N);
  c.rfwd = take(F.NR);
  c.wq = take(F.N);
  const int NC = F.ND - 2 * F.NP;
  c.Pf = (const double*)take(((size_t)NC * F.NT + 1) / 2);
  c.Pi = take((size_t)F.NT * NC);
  return c;
}

FSArgs fs_args(const tdse_plan_s* p) {
  FSArgs a;
  std::memset(&a, 0, sizeof(a));
  const bool d3 = p->dim == 3;
  a.N1 = p->fx[0].N * (d3 ? p->fx[2].N : 1);
  a.N2 = p->fx[1].N;
  a.ax1 = cf_axis(p, 0);
  a.ax2 = cf_axis(p, 1);
  a.Nm = d3 ? p->fx[2].N : 0;
  a.ncol = (int64_t)p->fx[1].M * (d3 ? p->fx[2].M : 1);
  if (d3) a.axm = cf_axis(p, 2);
  a.Bm = p->B();
  a.ring = (double2*)(p->ws + p->o_ringf);
  a.ring_stride = p->NM;
  a.V = (const double*)(p->ws + p->o_Vf);
  a.nV = p->nV;
  a.vstride = p->P;
  a.ph = p->ph();
  a.slot_w = -1;
  a.src = (const double2*)(p->ws + p->o_tmpf);
  a.dst = (double2*)(p->ws + p->o_tmpf);
  a.UH = p->UH(p->uh_cur);
  a.UHacc = p->UH(1 - p->uh_cur);
  return a;
}

// the potential of a free-space pass at time t (see the periodic set_V)
void set_V(const tdse_plan_s* p, int, FSArgs& a, double t) {
  int64_t first = 0;
  const int k = p->V_window(t, a.fV, &first);
  if (p->vkind == TDSE_V_SAMPLED) {
    a.V = (const double*)(p->ws + p->o_Vf) + first * p->P;
    a.nV = k;
  }
}

// 3D: a middle-axis transform between the (k0, k1, x2) mode tile and the
// (k0, x1, x2) grid array, timed (kind 5) like the other passes
int fs_mid(tdse_plan_s* p, const FSArgs& a, bool inverse, bool timed) {
  FSArgs m = a;
  m.src = inverse ? (const double2*)(p->ws + p->o_tmpf) : (const double2*)(p->ws + p->o_midf);
  m.dst = inverse ? (double2*)(p->ws + p->o_midf) : (double2*)(p->ws + p->o_tmpf);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t first = p->ev_used;
  if (timed && p->prof) {
    e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  }
  const hipError_t e = launch_fs_mid(p->fx[2].nu, inverse, m, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  if (e0) p->prof_marks.push_back({first, 5});
  return TDSE_OK;
}

int fs_launch(tdse_plan_s* p, bool col, const FSArgs& a, bool timed = false) {
  const bool d3 = p->dim == 3;
  FSArgs c = a;
  if (col && d3) {
    // the column pass works on the (k0, x1, x2) array: the modes' middle axis
    // is inverted first for a solve, and transformed back after the pass
    if (a.mode == C_SOLVE) {
      const int s = fs_mid(p, a, true, timed);
      if (s) return s;
    }
    c.src = (const double2*)(p->ws + p->o_midf);
    c.dst = (double2*)(p->ws + p->o_midf);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t first = p->ev_used;
  if (timed && p->prof) {
    e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  }
  hipError_t e = col ? launch_fs_col(p->dim >= 2 ? p->fx[0].nu : 0, c, p->stream, e0, e1)
                     : launch_fs_row(p->fx[1].nu, c, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  if (e0) p->prof_marks.push_back({first, col ? 0 : 1});
  if (col && d3) return fs_mid(p, a, false, timed);
  return TDSE_OK;
}

void fs_phase_req(const tdse_plan_s* p, FSArgs& a, int nj, double t_b, double tau, bool stepgrid, int m_b) {
  LineArgs tmp;
  std::memset(&tmp, 0, sizeof(tmp));
  phase_req(p, tmp, nj, t_b, tau, stepgrid, m_b);
  a.req = tmp.req;
}

int fs_phase_only(const tdse_plan_s* p, const FSArgs& a) {
  hipError_t e = launch_fs_phase(a, p->stream);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("phase kernel: ") + hipGetErrorString(e));
  return TDSE_OK;
}

// modes dst = F((alpha + beta V(t)) u)
int fs_forward(tdse_plan_s* p, double t, double ar, double ai, double br, double bi, double2* dst) {
  FSArgs a = fs_args(p);
  a.mode = C_FWD;
  a.usrc = p->u(p->ucur);
  set_V(p, 0, a, t);
  a.alpha_re = ar; a.alpha_im = ai; a.beta_re = br; a.beta_im = bi;
  int s = fs_launch(p, true, a);
  if (s) return s;
  FSArgs r = fs_args(p);
  r.mode = R_FWD;
  r.fdst = dst;
  return fs_launch(p, false, r);
}

double2* fs_ring_slot(const tdse_plan_s* p, int s) { return (double2*)(p->ws + p->o_ringf) + (int64_t)s * p->NM; }

int fs_history(tdse_plan_s* p, int m) {
  return fs_forward(p, p->t_at(m), 0.0, 0.0, 1.0, 0.0, fs_ring_slot(p, m % (p->order - 1)));
}

// Iterated Richardson step from t_{m-1} on both u and uhat (Remark on
// high-order free-space schemes).
int fs_richardson(tdse_plan_s* p, int m) {
  const int n = p->order;
  const double t = p->t_at(m - 1);
  const int acc = 1 - p->ucur;
  for (int l = 0; l < p->L; ++l) {
    const int nsub = 1 << l;
    const double delta = p->dt / nsub;
    FSArgs ph = fs_args(p);
    fs_phase_req(p, ph, 1, t + delta, delta, false, 0);
    int s = fs_phase_only(p, ph);
    if (s) return s;
    FSArgs r = fs_args(p);
    r.mode = R_BINIT;
    r.slot_r[1] = (m - 1) % (n - 1);
    r.c0 = 0.5 * delta;
    s = fs_launch(p, false, r);
    if (s) return s;
    for (int k = 0; k < nsub; ++k) {
      const double ts1 = t + k * delta + delta;
      const bool last = (k == nsub - 1);
      FSArgs c = fs_args(p);
      c.mode = C_SOLVE;
      set_V(p, 0, c, ts1);
      c.csolve = 0.5 * delta;
      if (last) {
        c.uacc = p->u(acc);
        c.wacc = p->rich[l];
        c.acc_first = (l == 0);
      } else {
        fs_phase_req(p, c, 1, ts1 + delta, delta, false, 0);
      }
      s = fs_launch(p, true, c);
      if (s) return s;
      FSArgs rr = fs_args(p);
      if (!last) {
        rr.mode = R_AM;
        rr.nh = 1;
        rr.c0 = 0.5 * delta;
        rr.ch[1] = 0.5 * delta;
      } else {
        rr.mode = R_UHACC;
        rr.c0 = 0.5 * delta;
        rr.wacc = p->rich[l];
        rr.acc_first = (l == 0);
      }
      s = fs_launch(p, false, rr);
      if (s) return s;
    }
  }
  p->ucur = acc;
  p->uh_cur = 1 - p->uh_cur;
  return TDSE_OK;
}

int fs_am_init(tdse_plan_s* p) {
  const int n = p->order, m = p->ns;
  FSArgs ph = fs_args(p);
  fs_phase_req(p, ph, n - 1, 0.0, p->dt, true, m + 1);
  int s = fs_phase_only(p, ph);
  if (s) return s;
  FSArgs r = fs_args(p);
  r.mode = R_FORM;
  r.nh = n - 1;
  for (int j = 1; j <= n - 1; ++j) {
    r.slot_r[j] = (m + 1 - j) % (n - 1);
    r.ch[j] = p->dt * p->mu[j];
  }
  return fs_launch(p, false, r);
}

int fs_am_step(tdse_plan_s* p, int m, bool write_u) {
  const int n = p->order;
  FSArgs c = fs_args(p);
  c.mode = C_SOLVE;
  set_V(p, 0, c, p->t_at(m));
  c.csolve = p->mu[0] * p->dt;
  if (write_u) c.uout = p->u(p->ucur);
  if (m < p->nsteps) fs_phase_req(p, c, n - 1, 0.0, p->dt, true, m + 1);
  int s = fs_launch(p, true, c, true);
  if (s) return s;
  if (m == p->nsteps) return TDSE_OK;
  FSArgs r = fs_args(p);
  r.mode = R_AM;
  r.nh = n - 1;
  r.c0 = p->mu[0] * p->dt;
  r.slot_w = m % (n - 1);
  // no field component along the last axis: its factors of E^(j) are the
  // j-th powers of E^(1)'s, formed in the row pass instead of loaded
  r.pf_pow = 1;
  for (int j = 0; j < n - 1; ++j)
    if (c.req.dphi2[j] != 0.0) r.pf_pow = 0;
  for (int j = 1; j <= n - 1; ++j) {
    r.ch[j] = p->dt * p->mu[j];
    r.slot_r[j] = ((m + 1 - j) % (n - 1) + (n - 1)) % (n - 1);
  }
  return fs_launch(p, false, r, true);
}

int fs_step(tdse_plan_s* p, int m, bool write_u) {
  int s = TDSE_OK;
  if (m == 1) {
    // uhat_0 = F u0 and What_0 = F(V(0) u0) (Section 3.3)
    s = fs_forward(p, 0.0, 1.0, 0.0, 0.0, 0.0, p->UH(p->uh_cur));
    if (!s) s = fs_history(p, 0);
  }
  if (s) return s;
  if (m <= p->ns) {
    s = fs_richardson(p, m);
    if (!s) s = fs_history(p, m);
    return s;
  }
  if (m == p->ns + 1) s = fs_am_init(p);
  if (!s) s = fs_am_step(p, m, write_u);
  return s;
}

// Plan the free-space tables and workspace (after the common planning).
int plan_free(tdse_plan_s* p, const tdse_problem_t* prob) {
  if (prob->p != 8) return fail(TDSE_EUNSUPPORTED, "free space supports the order-16 Alpert rule only (p = 8)");
  if (prob->q < 2 || prob->q > 32 || prob->panels < 1 || prob->panels > 8) return fail(TDSE_EINVAL, "need 2 <= q <= 32, 1 <= panels <= 8");
  if (prob->cheb < -1 || prob->cheb == 1 || prob->cheb > FS_CHEB_MAX)
    return fail(TDSE_EINVAL, "cheb must be -1 (direct), 0 (automatic) or 2..64 interpolation terms");
  if (!(prob->eps > 0.0 && prob->eps < 1.0) && !(prob->H > 0.0)) return fail(TDSE_EINVAL, "need 0 < eps < 1 or H > 0");
  p->free_space = true;
  alpert_rule(8, 7, p->alp_x, p->alp_w);
  // H from the Remark on its choice, log(eps / ((1 + ||V||_{2,inf}) eps_m)) / (2 d (1 + phi_max)),
  // taken in each dimension, as the analysis of the complex-frequency
  // representation bounds it, with that axis' quiver radius max_t |phi_a(t)|;
  // maxima over the step times
  if (prob->H > 0.0) {
    p->Hfx[0] = p->Hfx[1] = p->Hfx[2] = prob->H;
  } else {
    const double cell = std::ldexp(1.0, p->dim) / (double)p->P;
    double normV = 0.0, phimax[3] = {0.0, 0.0, 0.0};
    std::vector<double> f(MAXV);
    for (int n = 0; n <= p->nsteps; ++n) {
      const double t = p->t_at(n);
      int64_t first = 0;
      const int k = p->V_window(t, f.data(), &first);
      double s2 = 0.0;
      for (int64_t g = 0; g < p->P; ++g) {
        double v = 0.0;
        for (int r = 0; r < k; ++r) v += f[r] * p->Vsrc[(size_t)(first + r) * p->P + g];
        s2 += v * v;
      }
      normV = std::max(normV, std::sqrt(s2 * cell));
      double ph[3];
      p->tf.phi(t, ph);
      for (int a = 0; a < p->dim; ++a) phimax[a] = std::max(phimax[a], std::fabs(ph[a]));
    }
    const double num = std::log(prob->eps / ((1.0 + normV) * std::ldexp(1.0, -52)));
    for (int a = 0; a < p->dim; ++a) p->Hfx[fx_of(p->dim, a)] = num / (2.0 * p->dim * (1.0 + phimax[a]));
  }
  p->H = p->Hfx[fx_of(p->dim, 0)];
  for (int a = 0; a < p->dim; ++a)
    if (!(p->Hfx[fx_of(p->dim, a)] > 0.0)) return fail(TDSE_EINVAL, "the rule for H gives H <= 0 (eps too small)");
  int axes[3] = {1, 1, 1}, nus[3] = {0, 0, 0};
  for (int a = 0; a < p->dim; ++a) {
    axes[fx_of(p->dim, a)] = prob->M[a];
    nus[fx_of(p->dim, a)] = prob->nu[a];
  }
  for (int a = 0; a < (p->dim == 3 ? 3 : 2); ++a) {
    if (a == 0 && p->dim == 1) {
      tdse_plan_s::FAxis& F = p->fx[0];
      F = tdse_plan_s::FAxis();
      F.tables.assign(256, 0);   // zeta = {0}
      continue;
    }
    const int M = axes[a], nu = nus[a];
    if (!fs_nu_supported(nu)) return fail(TDSE_EINVAL, "nu must be 256, 512, 1024 or 2048");
    const int NE = nu / 2 - 13;
    if (M < 8 || M % 2 || M > nu || NE <= M / 2) return fail(TDSE_EINVAL, "free space needs even M, M <= nu and N_E > M/2");
    plan_free_axis(p, a, M, nu, prob->q, prob->panels, prob->cheb);
    // the line kernels carry each ray in the first half of the nu-point FFT
    if (p->fx[a].NE >= nu / 2) return fail(TDSE_EINVAL, "ray modes must number fewer than nu/2");
    // the dense rows' partial sums share the second FFT exchange line
    if (p->fx[a].NR > nu / 2)
      return fail(TDSE_EINVAL, "more than nu/2 dense rows (2p + 2 q panels direct sums, or 2p + NT); use the interpolant or a larger nu");
    if (fs_line_lds_bytes(nu, M, p->fx[a].ND, p->fx[a].NT != 0) > 65536)
      return fail(TDSE_EINVAL, "free-space line needs more than 64 KiB of LDS (M too large for this nu)");
  }
  const bool d3 = p->dim == 3;
  const int64_t Nm = d3 ? p->fx[2].N : 1, Mm = d3 ? p->fx[2].M : 1;
  p->NM = (int64_t)p->fx[0].N * Nm * p->fx[1].N;
  if ((double)p->NM * sizeof(double2) * (p->order + 3) > (double)((int64_t)200 << 30))
    return fail(TDSE_EINVAL, "free space: the mode arrays would pass 200 GiB");
  size_t off = 0;
  const size_t mb = (size_t)p->NM * sizeof(double2);
  p->o_B = off; off = align256(off + mb);
  p->o_ringf = off; off = align256(off + (size_t)(p->order - 1) * mb);
  p->o_UH[0] = off; off = align256(off + mb);
  p->o_UH[1] = off; off = align256(off + mb);
  p->o_tmpf = off; off = align256(off + (size_t)p->fx[0].N * Nm * p->fx[1].M * sizeof(double2));
  if (d3) {   // the (k0, x1, x2) array between the middle-axis passes and the column pass
    p->o_midf = off;
    off = align256(off + (size_t)p->fx[0].N * Mm * p->fx[1].M * sizeof(double2));
  }
  p->o_u[0] = off; off = align256(off + (size_t)p->P * sizeof(double2));
  p->o_u[1] = off; off = align256(off + (size_t)p->P * sizeof(double2));
  p->o_Vf = off; off = align256(off + p->Vsrc.size() * sizeof(double));
  p->o_ph = off; off = align256(off + (size_t)(p->order - 1) * (p->fx[0].N * Nm + p->fx[1].N) * sizeof(double2));
  for (int a = 0; a < (d3 ? 3 : 2); ++a) {
    p->fx[a].o_tab = off;
    off = align256(off + p->fx[a].tables.size());
  }
  p->total = off;
  return TDSE_OK;
}


// ============================================================ 1D, one workgroup
//
// Tables of the one-workgroup 1D run (layout in tdse_internal.h): the time
// factors and phase increments of every step and start-up sub-step, in the
// order the kernel consumes them, and the static phase factors
// exp(-i k^2 tau) of the Adams intervals tau = j dt and of the sub-steps
// tau = dt / 2^l, from extended precision.
void build_run1d(tdse_plan_s* p) {
  const int N = p->nsteps, ns = p->ns, L = p->L, M = p->M2, nh = p->order - 1;
  std::vector<double>& T = p->r1tab;
  T.clear();
  double f[MAXV];
  p->r1_oH = 0;
  for (int m = 0; m <= ns; ++m) {
    p->fV_at(p->t_at(m), f);
    T.insert(T.end(), f, f + MAXV);
  }
  p->r1_oR = (int64_t)T.size();
  double pb[3], pa[3];
  for (int m = 1; m <= ns; ++m) {
    const double t = p->t_at(m - 1);
    for (int l = 0; l < L; ++l) {
      const int nsub = 1 << l;
      const double delta = p->dt / nsub;
      for (int k = 0; k < nsub; ++k) {
        const double ts1 = (t + k * delta) + delta;   // end of sub-step k
        p->fV_at(ts1, f);
        T.insert(T.end(), f, f + MAXV);
        p->tf.phi(ts1, pb);
        p->tf.phi(ts1 - delta, pa);
        T.push_back(pb[0] - pa[0]);
      }
    }
  }
  p->r1_oA = (int64_t)T.size();
  for (int m = ns + 1; m <= N; ++m) {
    p->fV_at(p->t_at(m), f);
    T.insert(T.end(), f, f + MAXV);
  }
  p->r1_oD = (int64_t)T.size();
  for (int i = 1; i <= N; ++i) {
    p->tf.phi(p->t_at(i), pb);
    p->tf.phi(p->t_at(i - 1), pa);
    T.push_back(pb[0] - pa[0]);
  }
  p->r1stab.assign((size_t)(nh + L) * M, double2{0.0, 0.0});
  for (int r = 0; r < nh + L; ++r) {
    const long double tau = r < nh ? (long double)(r + 1) * (long double)p->dt
                                   : (long double)p->dt / (long double)(1 << (r - nh));
    for (int idx = 0; idx < M; ++idx) {
      const long double k = (long double)(idx < M / 2 ? idx : idx - M);
      const long double th = -k * k * tau;
      p->r1stab[(size_t)r * M + idx] = double2{(double)cosl(th), (double)sinl(th)};
    }
  }
}

int upload_run1d(tdse_plan_s* p) {
  HIP_TRY(hipMemcpyAsync(p->ws + p->o_r1tab, p->r1tab.data(), p->r1tab.size() * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  HIP_TRY(hipMemcpyAsync(p->ws + p->o_r1stab, p->r1stab.data(), p->r1stab.size() * sizeof(double2),
                         hipMemcpyHostToDevice, p->stream));
  return TDSE_OK;
}

// Steps cur+1 .. end of a 1D plan in one launch; u(t_end) is left where the
// multi-launch path leaves it (the physical buffer flips once per start-up step).
int run1d_step(tdse_plan_s* p, int end) {
  Run1DArgs a;
  std::memset(&a, 0, sizeof(a));
  a.M = p->M2;
  a.order = p->order;
  a.ns = p->ns;
  a.nsteps = p->nsteps;
  a.L = p->L;
  a.m0 = p->cur;
  a.m1 = end;
  a.nV = p->nV;
  a.vkind = p->vkind;
  a.write_u = 1;
  a.has_phase = p->tf.A_kind != TDSE_A_NONE;
  a.stab_rows = p->order - 1 + p->L;
  a.dt = p->dt;
  a.c0 = p->mu[0] * p->dt;
  for (int j = 1; j < p->order; ++j) a.ch[j] = p->dt * p->mu[j];
  for (int l = 0; l < p->L; ++l) a.rich[l] = p->rich[l];
  a.V = (const double*)p->V(0);
  a.vstride = p->P;
  a.tab = (const double*)(p->ws + p->o_r1tab);
  a.oH = p->r1_oH;
  a.oR = p->r1_oR;
  a.oA = p->r1_oA;
  a.oD = p->r1_oD;
  const int uo = std::min(end, p->ns) % 2;
  a.u_in = p->u(p->ucur);
  a.u_out = p->u(uo);
  a.B = p->B();
  a.ring = (double2*)p->ring(0);
  a.stab = (const double2*)(p->ws + p->o_r1stab);
  a.tw = (const double2*)p->tw(0, 1);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t first = p->ev_used;
  if (p->prof) {
    e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  }
  const hipError_t e = launch_run1d(a, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("1D run kernel: ") + hipGetErrorString(e));
  if (e0) p->prof_marks.push_back({first, 3});
  p->cur = end;
  p->ucur = uo;
  return TDSE_OK;
}

// ============================================================ 2D, persistent
//
// Tables of the persistent 2D Adams steps (layout in tdse_internal.h): per
// Adams step m = ns+1..N the potential time factors at t_m and the axis-0
// phase differences of the n-1 intervals ending at t_{m+1}; the axis-1 phase
// increments of every step; the static axis-1 factors exp(-i k2^2 j dt) from
// extended precision.
void build_persist2d(tdse_plan_s* p) {
  const int N = p->nsteps, ns = p->ns, M = p->M2, nh = p->order - 1;
  std::vector<double>& T = p->p2tab;
  T.clear();
  double f[MAXV], pb[3], pa[3];
  for (int m = ns + 1; m <= N; ++m) {
    p->fV_at(p->t_at(m), f);
    T.insert(T.end(), f, f + MAXV);
    p->tf.phi(p->t_at(m + 1), pb);
    for (int j = 1; j <= MAXH - 1; ++j) {
      if (j <= nh) {
        p->tf.phi(p->t_at(m + 1 - j), pa);
        T.push_back(pb[0] - pa[0]);
      } else {
        T.push_back(0.0);
      }
    }
    T.push_back(0.0);
  }
  p->p2_oD2 = (int64_t)T.size();
  p->p2_ph2 = false;
  for (int i = 1; i <= N; ++i) {
    p->tf.phi(p->t_at(i), pb);
    p->tf.phi(p->t_at(i - 1), pa);
    T.push_back(pb[1] - pa[1]);
    if (pb[1] - pa[1] != 0.0) p->p2_ph2 = true;
  }
  p->p2S2.assign((size_t)nh * M, double2{0.0, 0.0});
  for (int j = 1; j <= nh; ++j)
    for (int idx = 0; idx < M; ++idx) {
      const long double k = (long double)(idx < M / 2 ? idx : idx - M);
      const long double th = -k * k * (long double)j * (long double)p->dt;
      p->p2S2[(size_t)(j - 1) * M + idx] = double2{(double)cosl(th), (double)sinl(th)};
    }
}

int upload_persist2d(tdse_plan_s* p) {
  HIP_TRY(hipMemcpyAsync(p->ws + p->o_p2tab, p->p2tab.data(), p->p2tab.size() * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  HIP_TRY(hipMemcpyAsync(p->ws + p->o_p2S2, p->p2S2.data(), p->p2S2.size() * sizeof(double2), hipMemcpyHostToDevice,
                         p->stream));
  return TDSE_OK;
}

// Adams steps cur+1 .. end (cur > ns, after the Adams start) in one persistent
// launch.  Returns 1 (and clears p->persist) when the device cannot hold the
// co-resident grid, so the caller takes the two-pass path.
int persist2d_step(tdse_plan_s* p, int end, bool write_u) {
  const int grid = p->M2 / 2;
  if (p->persist_cap < 0) p->persist_cap = persist2d_capacity(p->M2, p->order, p->p2_ph2);
  if (p->persist_cap < grid) {
    p->persist = false;
    return 1;
  }
  Persist2DArgs a;
  std::memset(&a, 0, sizeof(a));
  a.N = p->M2;
  a.order = p->order;
  a.nsteps = p->nsteps;
  a.m0 = p->cur;
  a.m1 = end;
  a.mbase = p->ns + 1;
  a.ostep = tdse_plan_s::P2_OSTEP;
  a.nV = p->nV;
  a.write_u = write_u ? 1 : 0;
  a.ph2 = p->p2_ph2 ? 1 : 0;
  a.spin_limit = 1000000;
  a.dt = p->dt;
  a.c0 = p->mu[0] * p->dt;
  a.scale = 1.0 / (double)p->P;
  for (int j = 1; j < p->order; ++j) a.ch[j] = p->dt * p->mu[j];
  a.V = (const double*)p->V(0);
  a.vstride = p->P;
  a.tab = (const double*)(p->ws + p->o_p2tab);
  a.oD2 = p->p2_oD2;
  a.tile = (double2*)p->tmp(0);
  a.xbuf = p->u(1 - p->ucur);   // the start-up's second physical buffer, free in the Adams phase
  a.B = p->B();
  a.ring = (double2*)p->ring(0);
  a.S2 = (const double2*)(p->ws + p->o_p2S2);
  a.tw = (const double2*)p->tw(0, 1);
  a.uout = p->u(p->ucur);
  a.bar = (unsigned*)(p->ws + p->o_p2bar);
  a.flag = a.bar + 32 * 9;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t first = p->ev_used;
  if (p->prof) {
    e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(e0, p->stream));
  }
  const hipError_t e = launch_persist2d(a, p->stream);
  if (e == hipErrorCooperativeLaunchTooLarge) {
    (void)hipGetLastError();
    p->persist = false;
    return 1;
  }
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("persistent 2D kernel: ") + hipGetErrorString(e));
  if (e1) {
    HIP_TRY(hipEventRecord(e1, p->stream));
    p->prof_marks.push_back({first, 4});
  }
  // a grid barrier that timed out leaves the run unusable: report it now
  unsigned flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, a.flag, sizeof(flag), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (flag) return fail(TDSE_EDEVICE, "persistent 2D kernel: a grid barrier timed out (co-resident grid not scheduled)");
  p->cur = end;
  return TDSE_OK;
}

// ============================================================ diagnostics
//
// The failure guard: the physical solution u(t_cur) (of every instance of a
// batch) is scanned on the device for entries that are not finite, and its
// squared norm summed; the stream is then synchronized to read the flag.
int guard_check(tdse_plan_s* p) {
  double* acc = (double*)(p->ws + p->o_diag);
  unsigned* flag = (unsigned*)(acc + 2);
  std::vector<tdse_plan_s*> inst;
  if (p->is_batch()) inst = p->sub;
  else inst.push_back(p);
  for (size_t i = 0; i < inst.size(); ++i) {
    const tdse_plan_s* q = inst[i];
    const hipError_t e = launch_guard((const double*)q->u(q->ucur), 2 * q->P, acc, flag, i == 0, p->stream);
    if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("guard kernel: ") + hipGetErrorString(e));
  }
  double h[3] = {0.0, 0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(h, acc, 3 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  unsigned bad = 0;
  std::memcpy(&bad, &h[2], sizeof(bad));
  p->state_norm = std::sqrt(h[0]);
  if (bad) {
    p->state_norm = NAN;
    return fail(TDSE_ENONFINITE, "the state is not finite after step " + std::to_string(p->cur));
  }
  return TDSE_OK;
}

// Drift of the history entry of the current Adams step: What_n as stored in
// the ring (in the transform precision of the plan) against F(V(t_n) u_n)
// recomputed in FP64 from the physical solution, relative L2.
int history_residual(tdse_plan_s* p, double* value) {
  if (p->is_batch() || p->free_space) return fail(TDSE_EUNSUPPORTED, "the residual is kept for single periodic plans");
  if (!p->bound || !(p->cur > p->ns && p->cur < p->nsteps))
    return fail(TDSE_ESTATE, "the residual needs a state past the Adams start and before T");
  const int n = p->cur, nh = p->order - 1;
  const bool split = p->precision == TDSE_FP32_SPLIT;
  double2* X = p->u(1 - p->ucur);                                  // free in the Adams phase
  double2* Y = split ? (double2*)p->ring_slot(0, 0) : (double2*)(p->ws + p->o_dbuf);
  LineArgs a = base_args(p, 0);
  col_geom(p, 0, a);
  a.mode = C_FWD;
  a.src = p->u(p->ucur);
  a.dst = X;
  set_V(p, 0, a, p->t_at(n));
  a.alpha_re = 0.0; a.alpha_im = 0.0; a.beta_re = 1.0; a.beta_im = 0.0;
  int s = launch(p, 0, true, a);
  if (s) return s;
  LineArgs r = base_args(p, 0);
  row_geom(p, 0, r);
  r.mode = R_FWD;
  r.src = X;
  r.fdst = Y;
  s = launch(p, 0, false, r);
  if (s) return s;
  double* acc = (double*)(p->ws + p->o_diag);
  const void* W = p->ring_slot(1, n % nh);
  const hipError_t e = launch_diffnorm(split ? (const float2*)W : nullptr, split ? nullptr : (const double2*)W, Y, p->P,
                                       acc, (unsigned*)(acc + 2), p->stream);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("residual kernel: ") + hipGetErrorString(e));
  double h[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *value = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
  return TDSE_OK;
}

// Step m of one instance (write_u: leave u(t_m) in the physical buffer).
int do_step(tdse_plan_s* p, int m, bool write_u) {
  if (p->free_space) return fs_step(p, m, write_u);
  int s = TDSE_OK;
  if (m <= p->ns) {
    if (m == 1) s = op_history(p, 0);
    if (!s) s = op_richardson(p, m);
    if (!s) s = op_history(p, m);
    return s;
  }
  if (m == p->ns + 1) {
    if (p->ns == 0) s = op_history(p, 0);
    if (!s) s = op_am_init(p);
  }
  if (!s) s = op_am_step(p, m, write_u);
  return s;
}

// ================================================================ batches
//
// A batch runs independent periodic instances that share the order, the
// number of steps, the start-up length and the precision, so that every
// instance takes the same sequence of passes.  At bind, the sequence of each
// instance is recorded once (the launch arguments of every pass of the run),
// the i-th passes of all instances are grouped, and their arguments are
// stored in a device table; a step is then one batched launch per pass (and
// per schedule family present), each workgroup taking one tile of one
// instance.

int batch_default_ept(bool col, int N) {
  if (N == 1) return 1;
  if (N % 3 == 0) return 6;
  if (col) return (N >= 256 && N <= 1024) ? 4 : 8;
  return N >= 2048 ? 8 : 4;
}

bool batch_len_ok(int N) {
  for (int e : {1, 4, 6, 8, 12})
    if (batch_schedule_ok(N, e)) return true;
  return false;
}

int batch_len(const tdse_plan_s* q, int kind) { return kind == 0 ? q->M1 : q->M2; }
int batch_lines(const tdse_plan_s* q, int kind) { return kind == 0 ? q->M2 : q->M1; }

int64_t tile_base(const tdse_plan_s* p, int kind, int g) {
  return kind == 0 ? g * p->cap_tiles[0] : 2 * p->cap_tiles[0] + g * p->cap_tiles[1];
}

// An instance whose field has no component along its last axis at any time
// the scheme samples (step times and start-up sub-step times): its phase
// increments along that axis are zero, and its row passes may form that
// axis' factors of E^(j) as powers of E^(1)'s.
bool last_axis_field_free(const tdse_plan_s* q) {
  const int last = q->dim - 1;
  double ph[3];
  for (int m = 0; m <= q->nsteps; ++m) {
    q->tf.phi(q->t_at(m), ph);
    if (ph[last] != 0.0) return false;
  }
  for (int m = 1; m <= std::min(q->ns, q->nsteps); ++m)
    for (int l = 0; l < q->L; ++l)
      for (int k = 1; k < (1 << l); ++k) {
        q->tf.phi(q->t_at(m - 1) + k * q->dt / (1 << l), ph);
        if (ph[last] != 0.0) return false;
      }
  return true;
}

// Tile table of one pass kind and buffer stage from per-instance schedules,
// ordered by schedule family; uploaded synchronously.
int batch_tiles(tdse_plan_s* p, int kind, int g, const std::vector<int>& ept) {
  const int prec = p->sub[0]->st[g].prec;
  std::vector<BatchTile> fam[NFAM];
  tdse_plan_s::TileSet& ts = p->tiles[kind][g];
  ts.off = tile_base(p, kind, g);
  for (int f = 0; f < NFAM; ++f) ts.lds[f] = 0;
  for (size_t i = 0; i < p->sub.size(); ++i) {
    const tdse_plan_s* q = p->sub[i];
    const int N = batch_len(q, kind), e = ept[i];
    int f = batch_family(N, e);
    if (f < 0) return fail(TDSE_EINVAL, "no batched schedule for this line length");
    if (kind == 1 && last_axis_field_free(q)) f += 3;
    const int LPW = BATCH_THREADS / (N / e);
    const int nl = batch_lines(q, kind);
    const int nt = (nl + LPW - 1) / LPW;
    for (int b = 0; b < nt; ++b) fam[f].push_back(BatchTile{(int32_t)i, b * LPW, b, nt, N * 64 + e, 0});
    ts.lds[f] = std::max(ts.lds[f], batch_lds_bytes(prec, kind == 0, N, e));
  }
  std::vector<BatchTile> all;
  for (int f = 0; f < NFAM; ++f) {
    ts.first[f] = (int)all.size();
    ts.cnt[f] = (int)fam[f].size();
    if (ts.lds[f] > p->lds_max) return fail(TDSE_EINVAL, "batched schedule exceeds the LDS of a workgroup");
    all.insert(all.end(), fam[f].begin(), fam[f].end());
  }
  if ((int64_t)all.size() > p->cap_tiles[kind]) return fail(TDSE_EINVAL, "tile table overflow");
  HIP_TRY(hipStreamSynchronize(p->stream));
  HIP_TRY(hipMemcpy(p->ws + p->o_tiles + ts.off * sizeof(BatchTile), all.data(), all.size() * sizeof(BatchTile),
                    hipMemcpyHostToDevice));
  return TDSE_OK;
}

// Group the i-th recorded launches of all instances.
int batch_group(std::vector<std::vector<RecLaunch>>& rl, std::vector<tdse_plan_s::GLaunch>& out,
                std::vector<LineArgs>& args, std::vector<tdse_plan_s::Narrow>& nar) {
  const size_t n = rl.size(), L = rl[0].size();
  for (size_t i = 1; i < n; ++i)
    if (rl[i].size() != L) return fail(TDSE_EINVAL, "batch instances take different pass sequences");
  for (size_t k = 0; k < L; ++k) {
    const RecLaunch& r0 = rl[0][k];
    for (size_t i = 1; i < n; ++i)
      if (rl[i][k].kind != r0.kind || rl[i][k].g != r0.g)
        return fail(TDSE_EINVAL, "batch instances take different pass sequences");
    tdse_plan_s::GLaunch gl{r0.kind, r0.g, r0.timed, 0};
    if (r0.kind == 2) {
      gl.arg0 = (int64_t)nar.size();
      for (size_t i = 0; i < n; ++i) nar.push_back({rl[i][k].nsrc, rl[i][k].ndst, rl[i][k].nn});
    } else {
      gl.arg0 = (int64_t)args.size();
      for (size_t i = 0; i < n; ++i) args.push_back(rl[i][k].a);
    }
    out.push_back(gl);
  }
  return TDSE_OK;
}

// record step m of every instance (instances' clocks at m - 1)
int batch_record_step(tdse_plan_s* p, int m, bool write_u, std::vector<tdse_plan_s::GLaunch>& out,
                      std::vector<LineArgs>& args, std::vector<tdse_plan_s::Narrow>& nar) {
  std::vector<std::vector<RecLaunch>> rl(p->sub.size());
  for (size_t i = 0; i < p->sub.size(); ++i) {
    tdse_plan_s* q = p->sub[i];
    q->rec = &rl[i];
    const int s = do_step(q, m, write_u);
    q->rec = nullptr;
    if (s) return s;
  }
  return batch_group(rl, out, args, nar);
}

// Record the whole run: seg[m] for m = 1..nsteps, seg_last (step nsteps with
// output), the args table and the narrowings.  Workspace pointers come from
// the instances' current bindings.
int batch_record(tdse_plan_s* p) {
  const int N = p->nsteps;
  p->seg.assign(N + 1, {});
  p->seg_last.clear();
  p->ucur_after.assign(N + 1, 0);
  p->bargs.clear();
  p->narrows.clear();
  for (tdse_plan_s* q : p->sub) q->ucur = 0;
  for (int m = 1; m <= N; ++m) {
    const int s = batch_record_step(p, m, false, p->seg[m], p->bargs, p->narrows);
    if (s) return s;
    p->ucur_after[m] = p->sub[0]->ucur;
  }
  if (N > p->sub[0]->ns) {
    const int s = batch_record_step(p, N, true, p->seg_last, p->bargs, p->narrows);
    if (s) return s;
  } else {
    p->seg_last = p->seg[N];
  }
  for (tdse_plan_s* q : p->sub) q->ucur = 0;
  return TDSE_OK;
}

int batch_exec(tdse_plan_s* p, const std::vector<tdse_plan_s::GLaunch>& L, const char* args_dev,
               const std::vector<tdse_plan_s::Narrow>& nar) {
  const size_t n = p->sub.size();
  for (const tdse_plan_s::GLaunch& gl : L) {
    if (gl.kind == 2) {
      for (size_t i = 0; i < n; ++i) {
        const tdse_plan_s::Narrow& w = nar[gl.arg0 + i];
        const hipError_t e = launch_narrow((const double2*)w.src, (float2*)w.dst, w.n, p->stream);
        if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("narrow: ") + hipGetErrorString(e));
      }
      continue;
    }
    const tdse_plan_s::TileSet& ts = p->tiles[gl.kind][gl.g];
    const int prec = p->sub[0]->st[gl.g].prec;
    const LineArgs* args = (const LineArgs*)args_dev + gl.arg0;
    const BatchTile* tiles = (const BatchTile*)(p->ws + p->o_tiles) + ts.off;
    const bool timed = p->prof && gl.timed;
    // the families touch disjoint instances: with more than one, the later
    // ones go to side streams (not when each launch is being timed)
    int nfam = 0;
    for (int f = 0; f < NFAM; ++f) nfam += ts.cnt[f] > 0;
    const bool fork = nfam > 1 && !timed && p->fam_fork;
    if (fork) HIP_TRY(hipEventRecord(p->fam_fork, p->stream));
    int side = 0;
    bool on_main = false;
    for (int f = 0; f < NFAM; ++f) {
      if (!ts.cnt[f]) continue;
      hipStream_t s = p->stream;
      if (fork && on_main) {
        s = p->fam_st[side++];
        HIP_TRY(hipStreamWaitEvent(s, p->fam_fork, 0));
      }
      on_main = true;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const size_t first = p->ev_used;
      if (timed) {
        e0 = next_event(p);
        e1 = next_event(p);
        if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
      }
      const hipError_t e = launch_batch_pass(prec, gl.kind == 0, f, args, tiles + ts.first[f], ts.cnt[f], ts.lds[f],
                                             s, e0, e1);
      if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("batched launch: ") + hipGetErrorString(e));
      if (e0) p->prof_marks.push_back({first, gl.kind});
    }
    for (int i = 0; i < side; ++i) {
      HIP_TRY(hipEventRecord(p->fam_join[i], p->fam_st[i]));
      HIP_TRY(hipStreamWaitEvent(p->stream, p->fam_join[i], 0));
    }
  }
  return TDSE_OK;
}

int batch_step(tdse_plan_s* p, int k) {
  if (!p->batch_ready) return fail(TDSE_ESTATE, "tdse_bind must come first");
  const int end = p->cur + k;
  const char* args = p->ws + p->o_args;
  for (int m = p->cur + 1; m <= end; ++m) {
    int s;
    if (m < end || m <= p->sub[0]->ns) {
      s = batch_exec(p, p->seg[m], args, p->narrows);
    } else if (m == p->nsteps) {
      s = batch_exec(p, p->seg_last, args, p->narrows);
    } else {
      // a run that stops inside the Adams phase: step m with output,
      // recorded now into the table of such steps
      std::vector<tdse_plan_s::GLaunch> L;
      std::vector<LineArgs> a;
      std::vector<tdse_plan_s::Narrow> nar;
      for (tdse_plan_s* q : p->sub) q->ucur = p->ucur_after[m - 1];
      s = batch_record_step(p, m, true, L, a, nar);
      if (s) return s;
      if (a.size() > p->cap_targs) return fail(TDSE_EINVAL, "output step table overflow");
      HIP_TRY(hipStreamSynchronize(p->stream));
      HIP_TRY(hipMemcpy(p->ws + p->o_targs, a.data(), a.size() * sizeof(LineArgs), hipMemcpyHostToDevice));
      s = batch_exec(p, L, p->ws + p->o_targs, nar);
    }
    if (s) return s;
    p->cur = m;
  }
  for (tdse_plan_s* q : p->sub) {
    q->ucur = p->ucur_after[end];
    q->cur = end;
  }
  return TDSE_OK;
}

// Plan a batch: instances planned one by one, then a dry recording of the
// run (no device memory touched) to size the argument tables.
int plan_batch(const tdse_problem_t* probs, int count, tdse_plan_s** out) {
  std::unique_ptr<tdse_plan_s> p(new (std::nothrow) tdse_plan_s());
  if (!p) return fail(TDSE_ENOMEM, "host allocation failed");
  size_t off = 0;
  int64_t elem = 0;
  for (int i = 0; i < count; ++i) {
    if (probs[i].domain != TDSE_PERIODIC) return fail(TDSE_EUNSUPPORTED, "batches hold periodic instances");
    if (probs[i].dim == 3) return fail(TDSE_EUNSUPPORTED, "batches take 1D and 2D instances");
    if (probs[i].V_kind == TDSE_V_SAMPLED) return fail(TDSE_EUNSUPPORTED, "batches take stored fields or the moving well");
    tdse_plan_s* q = nullptr;
    const int s = tdse_plan(&probs[i], &q);
    if (s) return s;
    if (q->run1d || q->persist) {   // batches march every instance with the batched passes
      q->run1d = false;
      q->persist = false;
      q->total = q->total_core;
    }
    p->sub.push_back(q);
    const tdse_plan_s* q0 = p->sub[0];
    if (q->order != q0->order || q->nsteps != q0->nsteps || q->ns != q0->ns || q->precision != q0->precision)
      return fail(TDSE_EINVAL, "batch instances must share order, nsteps, n_start and precision");
    for (int kind = 0; kind < 2; ++kind)
      if (!batch_len_ok(batch_len(q, kind)))
        return fail(TDSE_EUNSUPPORTED, "batched line lengths: 64..2048 (2^a) or 192..1536 (3 * 2^a)");
    p->sub_off.push_back(off);
    p->sub_elem.push_back(elem);
    off = align256(off + q->total);
    elem += q->P;
  }
  tdse_plan_s* q0 = p->sub[0];
  p->dim = q0->dim;
  p->order = q0->order;
  p->ns = q0->ns;
  p->nsteps = q0->nsteps;
  p->precision = q0->precision;
  p->P = elem;
  p->dt = q0->dt;
  p->T = q0->T;
  // dry recording with placeholder workspaces
  for (size_t i = 0; i < p->sub.size(); ++i) p->sub[i]->ws = (char*)(uintptr_t)(4096 + p->sub_off[i]);
  int s = batch_record(p.get());
  if (s) return s;
  p->cap_args = p->bargs.size();
  size_t tcap = 0;
  for (int m = q0->ns + 1; m <= std::min(q0->ns + 2, p->nsteps); ++m) {
    std::vector<tdse_plan_s::GLaunch> L;
    std::vector<LineArgs> a;
    std::vector<tdse_plan_s::Narrow> nar;
    for (tdse_plan_s* q : p->sub) q->ucur = p->ucur_after[m - 1];
    s = batch_record_step(p.get(), m, true, L, a, nar);
    if (s) return s;
    tcap = std::max(tcap, a.size());
  }
  for (tdse_plan_s* q : p->sub) {
    q->ws = nullptr;
    q->ucur = 0;
  }
  p->cap_targs = tcap;
  p->bargs.clear();
  p->bargs.shrink_to_fit();
  p->narrows.clear();
  p->seg.clear();
  p->seg_last.clear();
  for (int kind = 0; kind < 2; ++kind) {
    p->cap_tiles[kind] = 0;
    for (tdse_plan_s* q : p->sub) p->cap_tiles[kind] += batch_lines(q, kind);
    p->ept[kind].resize(p->sub.size());
    for (size_t i = 0; i < p->sub.size(); ++i) p->ept[kind][i] = batch_default_ept(kind == 0, batch_len(p->sub[i], kind));
  }
  p->o_args = off;
  off = align256(off + p->cap_args * sizeof(LineArgs));
  p->o_targs = off;
  off = align256(off + std::max<size_t>(p->cap_targs, 1) * sizeof(LineArgs));
  p->o_tiles = off;
  off = align256(off + (size_t)(2 * p->cap_tiles[0] + 2 * p->cap_tiles[1]) * sizeof(BatchTile));
  p->o_diag = off;
  off = align256(off + 64);
  p->total = off;
  *out = p.release();
  return TDSE_OK;
}

int bind_batch(tdse_plan_s* p) {
  int dev = 0, v = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (!p->fam_fork) {   // default priority, non-blocking
    HIP_TRY(hipEventCreateWithFlags(&p->fam_fork, hipEventDisableTiming));
    for (int i = 0; i < NFAM - 1; ++i) {
      HIP_TRY(hipStreamCreateWithFlags(&p->fam_st[i], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&p->fam_join[i], hipEventDisableTiming));
    }
  }
  HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  p->lds_max = (size_t)v;
  for (size_t i = 0; i < p->sub.size(); ++i) {
    const int s = tdse_bind(p->sub[i], p->ws + p->sub_off[i], p->sub[i]->total, p->stream);
    if (s) return s;
  }
  int s = batch_record(p);
  if (s) return s;
  if (p->bargs.size() > p->cap_args) return fail(TDSE_EINVAL, "argument table overflow");
  HIP_TRY(hipMemcpy(p->ws + p->o_args, p->bargs.data(), p->bargs.size() * sizeof(LineArgs), hipMemcpyHostToDevice));
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<int> def(p->sub.size());
    for (size_t i = 0; i < p->sub.size(); ++i) def[i] = batch_default_ept(kind == 0, batch_len(p->sub[i], kind));
    s = batch_tiles(p, kind, 0, def);
    if (!s) s = batch_tiles(p, kind, 1, p->ept[kind]);
    if (s) return s;
  }
  p->batch_ready = true;
  return TDSE_OK;
}

// Per-length schedule search on the Adams passes: for each pass kind and
// each distinct line length, every compiled schedule that fits the LDS is
// timed over `reps` launches of a recorded Adams step and the fastest kept.
int autotune_batch(tdse_plan_s* p, int reps) {
  const int ns = p->sub[0]->ns;
  const int m = std::min(p->nsteps - 1, ns + 2);
  if (m <= ns) return TDSE_OK;   // no Adams step to time
  hipEvent_t t0 = next_event(p), t1 = next_event(p);
  if (!t0 || !t1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  const bool prof = p->prof;
  p->prof = false;
  int status = TDSE_OK;
  for (int kind = 0; kind < 2 && !status; ++kind) {
    std::vector<tdse_plan_s::GLaunch> one;
    for (const tdse_plan_s::GLaunch& gl : p->seg[m])
      if (gl.kind == kind && gl.timed) one.push_back(gl);
    if (one.empty()) continue;
    one.resize(1);
    std::vector<int> lens;
    for (tdse_plan_s* q : p->sub) lens.push_back(batch_len(q, kind));
    std::vector<int> uniq(lens);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    for (int N : uniq) {
      int best = -1;
      float best_ms = 0.f;
      for (int e : {1, 4, 6, 8, 12}) {
        if (!batch_schedule_ok(N, e)) continue;
        const int prec = p->sub[0]->st[1].prec;
        if (batch_lds_bytes(prec, kind == 0, N, e) > p->lds_max) continue;
        std::vector<int> trial(p->ept[kind]);
        for (size_t i = 0; i < lens.size(); ++i)
          if (lens[i] == N) trial[i] = e;
        status = batch_tiles(p, kind, 1, trial);
        if (!status) status = batch_exec(p, one, p->ws + p->o_args, p->narrows);   // warm-up
        if (status) break;
        if (hipEventRecord(t0, p->stream) != hipSuccess) { status = fail(TDSE_EDEVICE, "hipEventRecord"); break; }
        for (int r = 0; r < reps && !status; ++r) status = batch_exec(p, one, p->ws + p->o_args, p->narrows);
        if (status) break;
        float ms = 0.f;
        if (hipEventRecord(t1, p->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
            hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
          status = fail(TDSE_EDEVICE, "autotune timing failed");
          break;
        }
        if (best < 0 || ms < best_ms) {
          best = e;
          best_ms = ms;
        }
      }
      if (status) break;
      for (size_t i = 0; i < lens.size(); ++i)
        if (lens[i] == N) p->ept[kind][i] = best;
    }
    if (!status) status = batch_tiles(p, kind, 1, p->ept[kind]);
  }
  p->prof = prof;
  p->ev_used = 0;
  p->prof_marks.clear();
  p->drop_graph();
  p->cur = -1;   // the timing runs overwrote the state
  return status;
}


// ================================================================ adjoint
//
// Reverse-mode derivative of J(u_N) (dJ = Re <lam, du_N>) with respect to the
// stepwise field samples A_m and to u0, for the FP64 scheme.  Forward: the
// start-up states u_0..u_ns are kept and the Adams state (B and the history
// ring) is checkpointed every K steps.  Reverse: per segment of K Adams steps
// the forward is recomputed from its checkpoint, keeping B_n and What_n, and
// the adjoint recurrence runs backwards (adjoint_kernels.hip):
//   beta_N = F^-H conj(S_N) lam,
//   beta_n = conj(E^(1)_{n+1}) beta_{n+1} + G_n^H omega_n,   G_n^H = F conj(S_n) V_n F^-1,
//   omega_m = i dt sum_j c_{m,j} conj(E^(j)_{m+j}) beta_{m+j},
// then the start-up sub-steps are reversed one by one.  Every phase factor
// contributes sum_k k_a Re(conj(adjoint of its output) i E x) to dJ/d(dphi_a)
// of its interval, and dJ/dA_m adds these with the interval's overlap with
// step m.

struct AdjLayout {
  int K = 1, C = 0, H = 1, nblk = 1, L = 1, nsub_max = 1;
  int64_t P = 1, rows = 0;
  size_t o_ustore = 0, o_ck = 0, o_bseg = 0, o_wwin = 0, o_beta = 0, o_omega = 0, o_omsu = 0, o_Z = 0;
  size_t o_phys[3] = {0, 0, 0}, o_modes[2] = {0, 0}, o_bvirt = 0, o_subv = 0, o_subg = 0, o_ph = 0;
  size_t o_part = 0, o_red = 0, o_csr = 0, o_gA = 0, csr_bytes = 0, total = 0;
  size_t ck_bytes = 0;
};

AdjLayout adj_layout(const tdse_plan_s* p, int K) {
  AdjLayout L;
  const int N = p->nsteps, ns = std::min(p->ns, N);
  L.H = p->order - 1;
  L.L = p->order / 2;
  L.nsub_max = 1 << (L.L - 1);
  L.P = p->P;
  L.nblk = (int)((p->P + 255) / 256);
  const int iters = N - 1 - ns;   // Adams iterations n = ns+1 .. N-1
  if (K <= 0) K = std::max(1, (int)std::ceil(std::sqrt((double)std::max(iters, 1))));
  L.K = K;
  L.C = N > ns ? std::max(1, (iters + K - 1) / K) : 0;
  const size_t a = (size_t)p->P * sizeof(double2);
  L.ck_bytes = (size_t)(1 + L.H) * a;
  L.rows = (N > ns ? (int64_t)(N - ns) * 2 * MAXH : 0) + (int64_t)ns * ((1 << L.L) - 1) * 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.o_ustore = take((size_t)(ns + 1) * a);
  L.o_ck = take((size_t)L.C * L.ck_bytes);
  L.o_bseg = take((size_t)K * a);
  L.o_wwin = take((size_t)(K + L.H) * a);
  L.o_beta = take(8 * a);
  L.o_omega = take(a);
  L.o_omsu = take((size_t)L.H * a);
  L.o_Z = take(a);
  for (int i = 0; i < 3; ++i) L.o_phys[i] = take(a);
  for (int i = 0; i < 2; ++i) L.o_modes[i] = take(a);
  L.o_bvirt = take(a);
  L.o_subv = take((size_t)L.nsub_max * a);
  L.o_subg = take((size_t)L.nsub_max * a);
  L.o_ph = take((size_t)ADJ_PH * (p->M1 + p->M2) * sizeof(double2));
  L.o_part = take((size_t)L.rows * L.nblk * sizeof(double));
  L.o_red = take((size_t)L.rows * sizeof(double));
  // field-gradient map: per sample (m, component) the rows that overlap it
  const int64_t nA = (int64_t)N * p->dim;
  const int64_t nnz = ((int64_t)(N - ns) * (L.H * (L.H + 1) / 2) + (int64_t)ns * ((1 << L.L) - 1)) * p->dim;
  // rowptr, then the row indices and the weights, each 256-byte aligned (as laid out below)
  L.csr_bytes = align256((size_t)(nA + 1) * sizeof(int)) + align256((size_t)nnz * sizeof(int)) +
                (size_t)nnz * sizeof(double) + 8;
  L.o_csr = take(L.csr_bytes);
  L.o_gA = take((size_t)nA * sizeof(double));
  L.total = off;
  return L;
}

struct AdjRun {
  tdse_plan_s* p;
  char* w;
  AdjLayout L;
  struct Row {
    double ta, tb;
    int axis;
  };
  std::vector<Row> rows;   // partial-sum row -> interval and internal axis
  double2* at(size_t off, int64_t i = 0) const { return (double2*)(w + off) + i * L.P; }
};

int adj_err(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return TDSE_OK;
}

// dst = fft2((alpha + beta V(t)) src) * scale   (physical -> modes, unnormalized FFT)
int adj_fft2(tdse_plan_s* p, const double2* src, double2* dst, double scale, double ar, double ai, double br, double bi,
             double t) {
  LineArgs a = base_args(p, 0);
  col_geom(p, 0, a);
  a.mode = C_FWD;
  a.src = src;
  a.dst = p->tmp(0);
  p->fV_at(t, a.fV);
  a.alpha_re = ar; a.alpha_im = ai; a.beta_re = br; a.beta_im = bi;
  a.scale = scale;
  int s = launch(p, 0, true, a);
  if (s) return s;
  LineArgs r = base_args(p, 0);
  row_geom(p, 0, r);
  r.mode = R_FWD;
  r.src = p->tmp(0);
  r.fdst = dst;
  return launch(p, 0, false, r);
}

// unnormalized inverse FFT of modes src, then / (1 + i csolve V(t)) into dst (physical);
// with zdst, the column pass's forward transform of V u / P lands in tmp and a
// row FFT of it in zdst (G^H when csolve = -mu_0 dt)
int adj_ifft2(tdse_plan_s* p, const double2* src, double2* dst, double csolve, double t, double2* zdst = nullptr) {
  LineArgs r = base_args(p, 0);
  row_geom(p, 0, r);
  r.mode = R_INV;
  r.Bm = (double2*)src;
  r.dst = p->tmp(0);
  int s = launch(p, 0, false, r);
  if (s) return s;
  LineArgs c = base_args(p, 0);
  col_geom(p, 0, c);
  c.mode = C_SOLVE;
  c.src = p->tmp(0);
  c.dst = p->tmp(0);
  c.csolve = csolve;
  p->fV_at(t, c.fV);
  c.uout = dst;   // may be null
  s = launch(p, 0, true, c);
  if (s || !zdst) return s;
  LineArgs f = base_args(p, 0);
  row_geom(p, 0, f);
  f.mode = R_FWD;
  f.src = p->tmp(0);
  f.fdst = zdst;
  return launch(p, 0, false, f);
}

int adj_point(tdse_plan_s* p, const double2* in, double2* out, double t, double ar, double ai, double br, double bi,
              double sc, bool divide, bool acc) {
  AdjPoint a;
  std::memset(&a, 0, sizeof(a));
  a.P = p->P;
  a.in = in;
  a.out = out;
  a.V = (const double*)p->V(0);
  a.nV = p->nV;
  a.vstride = p->P;
  p->fV_at(t, a.fV);
  a.ar = ar; a.ai = ai; a.br = br; a.bi = bi; a.s = sc;
  a.divide = divide;
  a.accumulate = acc;
  return adj_err(launch_adj_point(a, p->stream), "adjoint pointwise");
}

// phase entries e: E over [tb - tau, tb]
struct AdjPh {
  AdjPhase q;
  explicit AdjPh(const tdse_plan_s* p, double2* ph) {
    std::memset(&q, 0, sizeof(q));
    q.M1 = p->M1;
    q.M2 = p->M2;
    q.ph = ph;
  }
  void set(const tdse_plan_s* p, int e, double tb, double tau) {
    double pb[3], pa[3];
    p->tf.phi(tb, pb);
    p->tf.phi(tb - tau, pa);
    q.tau[e] = tau;
    if (p->dim == 2) {
      q.dphi1[e] = pb[0] - pa[0];
      q.dphi2[e] = pb[1] - pa[1];
    } else {
      q.dphi1[e] = 0.0;
      q.dphi2[e] = pb[0] - pa[0];
    }
    q.nj = std::max(q.nj, e + 1);
  }
};

int adj_copy(tdse_plan_s* p, void* dst, const void* src, size_t bytes) {
  return adj_err(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, p->stream), "adjoint copy");
}

// host threads (and streams) of a batch plan's adjoint
int adj_workers(const tdse_plan_s* p) { return std::max(1, std::min(p->adj_streams, (int)p->sub.size())); }

int adjoint_single(tdse_plan_s* p, char* w, size_t wbytes, int K, const void* u0, const void* lam, int on_device,
                   double* dF_dA, void* dF_du0) {
  if (p->free_space) return fail(TDSE_EUNSUPPORTED, "the adjoint covers the periodic scheme");
  if (p->dim == 3) return fail(TDSE_EUNSUPPORTED, "the adjoint covers 1D and 2D plans");
  if (p->vkind != TDSE_V_FIELDS) return fail(TDSE_EUNSUPPORTED, "the adjoint takes potentials from stored fields");
  if (p->tf.A_kind != TDSE_A_STEPWISE) return fail(TDSE_EUNSUPPORTED, "the adjoint differentiates stepwise field samples");
  AdjRun R;
  R.p = p;
  R.w = w;
  R.L = adj_layout(p, K);
  const AdjLayout& L = R.L;
  if (wbytes < L.total) return fail(TDSE_ENOMEM, "adjoint workspace smaller than tdse_adjoint_workspace_size");
  if (((uintptr_t)w) & 255) return fail(TDSE_EINVAL, "adjoint workspace must be 256-byte aligned");
  const int N = p->nsteps, ns = std::min(p->ns, N), H = L.H;
  const double dt = p->dt;
  const std::vector<double>& mu = p->mu;
  const size_t a = (size_t)p->P * sizeof(double2);
  const double invP = 1.0 / (double)p->P;
  const hipStream_t st = p->stream;
  p->drop_graph();
  const bool prof = p->prof;
  p->prof = false;
  p->force_fp64 = true;
  int s = TDSE_OK;
  auto done = [&](int status) {
    p->force_fp64 = false;
    p->prof = prof;
    p->cur = -1;   // the recomputation overwrote the state
    return status;
  };
  // ---- forward with storage
  s = tdse_set_state(p, u0, on_device);
  if (s) return done(s);
  p->force_fp64 = true;
  if (on_device) s = adj_copy(p, R.at(L.o_phys[2]), lam, a);
  else s = adj_err(hipMemcpyAsync(R.at(L.o_phys[2]), lam, a, hipMemcpyHostToDevice, st), "adjoint seed");
  if (!s) s = adj_copy(p, R.at(L.o_ustore, 0), p->u(p->ucur), a);
  for (int m = 1; m <= ns && !s; ++m) {
    s = do_step(p, m, false);
    if (!s) s = adj_copy(p, R.at(L.o_ustore, m), p->u(p->ucur), a);
  }
  if (s) return done(s);
  auto ck = [&](int c) { return w + L.o_ck + (size_t)c * L.ck_bytes; };
  if (N > ns) {
    if (ns == 0) s = op_history(p, 0);
    if (!s) s = op_am_init(p);
    if (!s) s = adj_copy(p, ck(0), p->B(), a);
    if (!s) s = adj_copy(p, ck(0) + a, p->ring(0), (size_t)H * a);
    for (int m = ns + 1; m <= N - 1 && !s; ++m) {
      s = op_am_step(p, m, false);
      const int sidx = m + 1 - (ns + 1);
      if (!s && sidx % L.K == 0 && sidx / L.K < L.C) {
        s = adj_copy(p, ck(sidx / L.K), p->B(), a);
        if (!s) s = adj_copy(p, ck(sidx / L.K) + a, p->ring(0), (size_t)H * a);
      }
    }
  }
  if (s) return done(s);
  // ---- reverse sweep
  s = adj_err(hipMemsetAsync(w + L.o_beta, 0, 8 * a, st), "adjoint clear");
  if (!s && L.rows) s = adj_err(hipMemsetAsync(w + L.o_part, 0, (size_t)L.rows * L.nblk * sizeof(double), st), "clear");
  if (s) return done(s);
  R.rows.assign((size_t)L.rows, AdjRun::Row{0.0, 0.0, 0});
  double2* beta = R.at(L.o_beta);
  auto bslot = [&](int idx) { return (idx >= ns + 1 && idx <= N) ? idx % 8 : -1; };
  auto cfac = [&](int m, int j) {   // coefficient of What_m in B_{m+j}
    if (j == 1) return m >= ns + 1 ? mu[0] + mu[1] : mu[1];
    return mu[j];
  };
  AdjPh PH(p, R.at(L.o_ph));
  const double2* Bvirt = R.at(L.o_bvirt);
  // one adjoint Adams iteration at n: beta_n, the partials of step n+1, omega_{n-1}
  auto am_iter = [&](int n, int beta_mode, bool grad, const double2* Bn, const double2* const* Wx,
                     double2* omega_out) -> int {
    PH.q.nj = 0;
    for (int j = 1; j <= H; ++j) {
      PH.set(p, j - 1, (n + 1) * dt, j * dt);
      PH.set(p, H + j - 1, (n - 1 + j) * dt, j * dt);
    }
    int e = adj_err(launch_adj_phase(PH.q, st), "adjoint phases");
    if (e) return e;
    AdjAm A;
    std::memset(&A, 0, sizeof(A));
    A.M1 = p->M1;
    A.M2 = p->M2;
    A.H = H;
    A.P = p->P;
    A.ph = PH.q.ph;
    A.beta = beta;
    A.slot_b1 = bslot(n + 1);
    A.slot_bn = n % 8;
    A.beta_mode = beta_mode;
    A.Z = R.at(L.o_Z);
    A.omega = omega_out;
    for (int j = 2; j <= H; ++j) A.slot_bj[j] = bslot(n - 1 + j);
    for (int j = 1; j <= H; ++j) A.wj[j] = (n - 1 + j >= ns + 1 && n - 1 + j <= N && n - 1 >= 0) ? dt * cfac(n - 1, j) : 0.0;
    A.has_grad = grad;
    A.nblk = L.nblk;
    if (grad) {
      const int64_t g0 = (int64_t)(n - ns) * 2 * MAXH;
      A.part = (double*)(w + L.o_part) + g0 * L.nblk;
      A.Bn = Bn;
      for (int j = 1; j <= H; ++j) {
        A.Wx[j] = Wx[j];
        A.cx[j] = j == 1 ? dt * (mu[0] + mu[1]) : dt * mu[j];
        for (int ax = 0; ax < 2; ++ax) R.rows[g0 + 2 * (j - 1) + ax] = AdjRun::Row{(n + 1 - j) * dt, (n + 1) * dt, ax};
      }
    }
    return adj_err(launch_adj_am(A, st), "adjoint Adams step");
  };
  auto omsu = [&](int m) { return R.at(L.o_omsu, m - (ns + 1 - H)); };
  if (N > ns) {
    // beta_N = F^-H conj(S_N) lam = fft2(lam / (1 - i mu_0 dt V(t_N)))
    s = adj_point(p, R.at(L.o_phys[2]), R.at(L.o_phys[0]), N * dt, 1.0, 0.0, 0.0, -mu[0] * dt, 1.0, true, false);
    if (!s) s = adj_fft2(p, R.at(L.o_phys[0]), beta + (int64_t)(N % 8) * p->P, 1.0, 1.0, 0.0, 0.0, 0.0, N * dt);
    if (!s) s = am_iter(N, 2, false, nullptr, nullptr, R.at(L.o_omega));
    if (!s && N - 1 <= ns) s = adj_copy(p, omsu(N - 1), R.at(L.o_omega), a);
    for (int c = L.C - 1; c >= 0 && !s; --c) {
      const int sc = ns + 1 + c * L.K;
      const int ec = std::min(sc + L.K - 1, N - 1);
      const int w0 = sc - H;   // window slot 0 holds What_{sc-H}
      s = adj_copy(p, p->B(), ck(c), a);
      if (!s) s = adj_copy(p, p->ring(0), ck(c) + a, (size_t)H * a);
      if (!s) {
        LineArgs r = base_args(p, 0);
        row_geom(p, 0, r);
        r.mode = R_INV;
        r.dst = p->tmp(0);
        s = launch(p, 0, false, r);
      }
      for (int i = std::max(w0, 0); i < sc && !s; ++i) s = adj_copy(p, R.at(L.o_wwin, i - w0), (char*)p->ring(0) + (size_t)(i % H) * a, a);
      // B_n into its segment slot before step n; What_{n-1}, which step n-1
      // left in the ring, into the window in the same launch
      auto ring_slot = [&](int m) { return (const double2*)((char*)p->ring(0) + (size_t)(m % H) * a); };
      for (int n = sc; n <= ec && !s; ++n) {
        if (n == sc) s = adj_copy(p, R.at(L.o_bseg, 0), p->B(), a);
        else
          s = adj_err(launch_adj_copy2(p->P, R.at(L.o_bseg, n - sc), p->B(), R.at(L.o_wwin, n - 1 - w0),
                                       ring_slot(n - 1), p->stream),
                      "adjoint copy");
        if (!s) s = op_am_step(p, n, false);
      }
      if (!s && ec >= sc) s = adj_copy(p, R.at(L.o_wwin, ec - w0), ring_slot(ec), a);
      for (int n = ec; n >= sc && !s; --n) {
        // Z = G_n^H omega_n = F conj(S_n) V_n F^-1 omega_n
        s = adj_ifft2(p, R.at(L.o_omega), nullptr, -mu[0] * dt, n * dt, R.at(L.o_Z));
        const double2* Wx[MAXH + 1] = {nullptr};
        for (int j = 1; j <= H; ++j) Wx[j] = R.at(L.o_wwin, (j == 1 ? n : n + 1 - j) - w0);
        if (!s) s = am_iter(n, 1, true, R.at(L.o_bseg, n - sc), Wx, R.at(L.o_omega));
        if (!s && n - 1 <= ns) s = adj_copy(p, omsu(n - 1), R.at(L.o_omega), a);
      }
    }
    if (s) return done(s);
    // step ns+1 formed B from F u_ns: B_virt = F u_ns + i mu_0 dt What_ns gives x_1
    {
      const int w0 = ns + 1 - H;
      s = adj_fft2(p, R.at(L.o_ustore, ns), R.at(L.o_modes[0]), invP, 1.0, 0.0, 0.0, 0.0, ns * dt);
      if (!s) s = adj_err(launch_adj_axpy(p->P, R.at(L.o_modes[0]), R.at(L.o_wwin, ns - w0), 0.0, mu[0] * dt,
                                          R.at(L.o_bvirt), st), "adjoint axpy");
      const double2* Wx[MAXH + 1] = {nullptr};
      for (int j = 1; j <= H; ++j) Wx[j] = R.at(L.o_wwin, (j == 1 ? ns : ns + 1 - j) - w0);
      if (!s) s = am_iter(ns, 0, true, Bvirt, Wx, ns >= 1 ? R.at(L.o_omega) : nullptr);
      if (!s && ns >= 1 && ns - 1 >= ns + 1 - H) s = adj_copy(p, omsu(ns - 1), R.at(L.o_omega), a);
      for (int n = ns - 1; n >= std::max(1, ns + 2 - H) && !s; --n) {
        s = am_iter(n, 0, false, nullptr, nullptr, R.at(L.o_omega));
        if (!s) s = adj_copy(p, omsu(n - 1), R.at(L.o_omega), a);
      }
    }
    if (s) return done(s);
    // g_u_ns = ifftn(conj(E^(1)_{ns+1}) beta_{ns+1}) + V_ns ifftn(omega_ns)
    PH.q.nj = 0;
    PH.set(p, 0, (ns + 1) * dt, dt);
    s = adj_err(launch_adj_phase(PH.q, st), "adjoint phases");
    if (!s) s = adj_copy(p, R.at(L.o_modes[0]), beta + (int64_t)((ns + 1) % 8) * p->P, a);
    if (!s) {
      AdjSub S;
      std::memset(&S, 0, sizeof(S));
      S.M1 = p->M1; S.M2 = p->M2; S.mode = 2; S.P = p->P; S.ph = PH.q.ph; S.y = R.at(L.o_modes[0]);
      S.nblk = L.nblk;
      s = adj_err(launch_adj_sub(S, st), "adjoint phase");
    }
    if (!s) s = adj_ifft2(p, R.at(L.o_modes[0]), R.at(L.o_phys[0]), 0.0, ns * dt);
    if (!s) s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[1]), ns * dt, invP, 0.0, 0.0, 0.0, 1.0, false, false);
    if (!s) s = adj_ifft2(p, omsu(ns), R.at(L.o_phys[0]), 0.0, ns * dt);
    if (!s) s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[1]), ns * dt, 0.0, 0.0, invP, 0.0, 1.0, false, true);
  } else {
    s = adj_copy(p, R.at(L.o_phys[1]), R.at(L.o_phys[2]), a);
  }
  if (s) return done(s);
  // ---- start-up sub-steps, newest first; g_u in phys[1], g_u_{m-1} built in phys[2]
  int64_t row = (N > ns ? (int64_t)(N - ns) * 2 * MAXH : 0);
  for (int m = ns; m >= 1 && !s; --m) {
    const double t0 = (m - 1) * dt;
    if (N > ns && m - 1 >= ns + 1 - H) {
      s = adj_ifft2(p, omsu(m - 1), R.at(L.o_phys[0]), 0.0, t0);
      if (!s) s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[2]), t0, 0.0, 0.0, invP, 0.0, 1.0, false, false);
    } else {
      s = adj_err(hipMemsetAsync(R.at(L.o_phys[2]), 0, a, st), "adjoint clear");
    }
    for (int l = 0; l < L.L && !s; ++l) {
      const int nsub = 1 << l;
      const double d = dt / nsub;
      // recompute the level's sub-step inputs v_s and g_s = F((1 - i d/2 V) v_s)
      s = adj_copy(p, R.at(L.o_subv, 0), R.at(L.o_ustore, m - 1), a);
      for (int k = 0; k < nsub && !s; ++k) {
        const double tau = t0 + k * d;
        s = adj_fft2(p, R.at(L.o_subv, k), R.at(L.o_subg, k), invP, 1.0, 0.0, 0.0, -0.5 * d, tau);
        if (s || k == nsub - 1) continue;
        PH.q.nj = 0;
        PH.set(p, 0, tau + d, d);
        s = adj_err(launch_adj_phase(PH.q, st), "adjoint phases");
        if (s) break;
        AdjSub S;
        std::memset(&S, 0, sizeof(S));
        S.M1 = p->M1; S.M2 = p->M2; S.mode = 1; S.P = p->P; S.ph = PH.q.ph; S.y = R.at(L.o_modes[1]);
        S.g = R.at(L.o_subg, k); S.nblk = L.nblk;
        s = adj_err(launch_adj_sub(S, st), "adjoint phase");
        if (!s) s = adj_ifft2(p, R.at(L.o_modes[1]), R.at(L.o_subv, k + 1), 0.5 * d, tau + d);
      }
      // reverse the level: g_v = r_l g_u_m
      if (!s) s = adj_point(p, R.at(L.o_phys[1]), R.at(L.o_phys[0]), t0, p->rich[l], 0.0, 0.0, 0.0, 1.0, false, false);
      for (int k = nsub - 1; k >= 0 && !s; --k) {
        const double tau = t0 + k * d;
        s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[0]), tau + d, 1.0, 0.0, 0.0, -0.5 * d, 1.0, true, false);
        if (!s) s = adj_fft2(p, R.at(L.o_phys[0]), R.at(L.o_modes[1]), 1.0, 1.0, 0.0, 0.0, 0.0, tau);
        if (s) break;
        PH.q.nj = 0;
        PH.set(p, 0, tau + d, d);
        s = adj_err(launch_adj_phase(PH.q, st), "adjoint phases");
        if (s) break;
        AdjSub S;
        std::memset(&S, 0, sizeof(S));
        S.M1 = p->M1; S.M2 = p->M2; S.mode = 0; S.P = p->P; S.ph = PH.q.ph; S.y = R.at(L.o_modes[1]);
        S.g = R.at(L.o_subg, k); S.nblk = L.nblk;
        S.part = (double*)(w + L.o_part) + row * L.nblk;
        for (int ax = 0; ax < 2; ++ax) R.rows[row + ax] = AdjRun::Row{tau, tau + d, ax};
        row += 2;
        s = adj_err(launch_adj_sub(S, st), "adjoint phase");
        if (!s) s = adj_ifft2(p, R.at(L.o_modes[1]), R.at(L.o_phys[0]), 0.0, tau);
        if (!s) s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[0]), tau, 1.0, 0.0, 0.0, 0.5 * d, invP, false, false);
      }
      if (!s) s = adj_point(p, R.at(L.o_phys[0]), R.at(L.o_phys[2]), t0, 1.0, 0.0, 0.0, 0.0, 1.0, false, true);
    }
    if (!s) s = adj_copy(p, R.at(L.o_phys[1]), R.at(L.o_phys[2]), a);
  }
  if (s) return done(s);
  // ---- dJ/dA: reduce the partials, then map rows to samples
  const int64_t nA = (int64_t)N * p->dim;
  std::vector<std::vector<std::pair<int, double>>> by(nA);
  for (int64_t r = 0; r < row; ++r) {
    const AdjRun::Row& q = R.rows[r];
    if (q.tb <= q.ta) continue;
    const int comp = p->dim == 2 ? q.axis : (q.axis == 1 ? 0 : -1);
    if (comp < 0) continue;
    const int m0 = std::max(0, (int)std::floor(q.ta / dt + 1e-9));
    const int m1 = std::min(N, (int)std::ceil(q.tb / dt - 1e-9));
    for (int mm = m0; mm < m1; ++mm) {
      const double ov = std::min(q.tb, (mm + 1) * dt) - std::max(q.ta, mm * dt);
      if (ov > 0) by[(int64_t)mm * p->dim + comp].push_back({(int)r, ov});
    }
  }
  std::vector<int> rowptr(nA + 1, 0), src;
  std::vector<double> wt;
  for (int64_t o = 0; o < nA; ++o) {
    for (auto& e : by[o]) {
      src.push_back(e.first);
      wt.push_back(e.second);
    }
    rowptr[o + 1] = (int)src.size();
  }
  const size_t b_rp = rowptr.size() * sizeof(int), b_src = src.size() * sizeof(int), b_wt = wt.size() * sizeof(double);
  const size_t o_src = align256(b_rp), o_wt = align256(o_src + b_src);
  if (o_wt + b_wt + 8 > L.csr_bytes) return done(fail(TDSE_EINVAL, "adjoint map overflow"));
  std::vector<char> csr(o_wt + b_wt + 8, 0);
  std::memcpy(csr.data(), rowptr.data(), b_rp);
  if (b_src) std::memcpy(csr.data() + o_src, src.data(), b_src);
  if (b_wt) std::memcpy(csr.data() + o_wt, wt.data(), b_wt);
  s = adj_err(launch_adj_reduce((double*)(w + L.o_part), (double*)(w + L.o_red), (int)row, L.nblk, st), "adjoint reduce");
  if (!s) s = adj_err(hipStreamSynchronize(st), "adjoint sync");
  // on the plan's own stream: a synchronous copy on the null stream would
  // order against every other stream's work (and serialize concurrent adjoints)
  if (!s) s = adj_err(hipMemcpyAsync(w + L.o_csr, csr.data(), csr.size(), hipMemcpyHostToDevice, st), "adjoint map upload");
  if (!s) s = adj_err(hipStreamSynchronize(st), "adjoint sync");   // csr is host memory of this call
  if (!s) {
    char* cb = w + L.o_csr;
    s = adj_err(launch_adj_to_A((double*)(w + L.o_red), (const int*)cb, (const int*)(cb + o_src),
                                (const double*)(cb + o_wt), (double*)(w + L.o_gA), (int)nA, st), "adjoint map");
  }
  if (!s && dF_dA) s = adj_err(hipMemcpyAsync(dF_dA, w + L.o_gA, nA * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  if (!s && dF_du0)
    s = adj_err(hipMemcpyAsync(dF_du0, R.at(L.o_phys[1]), a, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st),
                "copy");
  if (!s) s = adj_err(hipStreamSynchronize(st), "adjoint sync");
  return done(s);
}

bool good_len(int M) { return M >= 8 && M <= 3072 && M % 2 == 0 && line_length_supported(M); }

}  // namespace

// ================================================================ C ABI

extern "C" {

const char* tdse_status_string(int status) {
  switch (status) {
    case TDSE_OK: return "TDSE_OK";
    case TDSE_EINVAL: return "TDSE_EINVAL: invalid argument";
    case TDSE_EUNSUPPORTED: return "TDSE_EUNSUPPORTED: not supported by the library";
    case TDSE_ENOMEM: return "TDSE_ENOMEM: workspace missing or too small";
    case TDSE_EDEVICE: return "TDSE_EDEVICE: HIP runtime error";
    case TDSE_ENONFINITE: return "TDSE_ENONFINITE: non-finite state";
    case TDSE_ESTATE: return "TDSE_ESTATE: call out of order";
    default: return "unknown status";
  }
}

const char* tdse_last_error(void) { return g_last_error.c_str(); }

int tdse_plan(const tdse_problem_t* prob, tdse_plan_t* out) {
  if (!prob || !out) return fail(TDSE_EINVAL, "NULL argument");
  *out = nullptr;
  if (prob->dim < 1 || prob->dim > 3) return fail(TDSE_EINVAL, "dim must be 1, 2 or 3");
  if (prob->dim == 3) {
    if (prob->V_kind == TDSE_V_MOVING_WELL) return fail(TDSE_EUNSUPPORTED, "3D takes stored or sampled potentials");
    if ((int64_t)prob->M[0] * prob->M[1] * prob->M[2] > ((int64_t)1 << 28))
      return fail(TDSE_EINVAL, "3D grid larger than 2^28 points");
  }
  if (prob->domain != TDSE_PERIODIC && prob->domain != TDSE_FREE) return fail(TDSE_EINVAL, "unknown domain");
  if (prob->precision != TDSE_FP64 && prob->precision != TDSE_FP32_SPLIT) return fail(TDSE_EINVAL, "unknown precision");
  const bool free_dom = prob->domain == TDSE_FREE;
  if (free_dom && prob->precision != TDSE_FP64) return fail(TDSE_EUNSUPPORTED, "the free-space scheme runs in FP64 only");
  for (int a = 0; a < prob->dim && !free_dom; ++a)
    if (!good_len(prob->M[a])) return fail(TDSE_EINVAL, "grid size must be 2^a or 3*2^a, 8..3072");
  if (!(prob->T > 0.0) || prob->nsteps < 1) return fail(TDSE_EINVAL, "need T > 0 and nsteps >= 1");
  if (prob->order < 2 || prob->order > 8 || prob->order % 2) return fail(TDSE_EINVAL, "order must be 2, 4, 6 or 8");
  const bool well = prob->V_kind == TDSE_V_MOVING_WELL;
  const bool sampled = prob->V_kind == TDSE_V_SAMPLED;
  if (prob->V_kind != TDSE_V_FIELDS && !well && !sampled) return fail(TDSE_EINVAL, "bad V_kind");
  if (sampled) {
    if (!prob->V_fields) return fail(TDSE_EINVAL, "sampled V: V_fields missing");
    int64_t pts = 1;
    for (int a = 0; a < std::max(1, std::min(3, (int)prob->dim)); ++a) pts *= std::max(1, (int)prob->M[a]);
    if (prob->nsteps < 1 || (double)(prob->nsteps + 1) * (double)pts * 8.0 > (double)((int64_t)64 << 30))
      return fail(TDSE_EINVAL, "sampled V: (nsteps + 1) samples must fit 64 GiB");
  }
  if (well) {
    if (prob->domain != TDSE_PERIODIC) return fail(TDSE_EUNSUPPORTED, "the moving well is a periodic potential");
    if (!(prob->V_params[1] > 0.0 && prob->V_params[1] <= 1.0))
      return fail(TDSE_EINVAL, "moving well: need 0 < beta <= 1 (at most three periodic images per axis)");
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(prob->V_params[k])) return fail(TDSE_EINVAL, "moving well: non-finite parameter");
  } else if (!sampled && (prob->nV < 1 || prob->nV > MAXV || !prob->V_fields)) {
    return fail(TDSE_EINVAL, "need 1..8 potential fields");
  }
  if (prob->f_kind == TDSE_F_SIN && !prob->f_params) return fail(TDSE_EINVAL, "f_params missing");
  if (prob->f_kind == TDSE_F_CALLBACK && !prob->f_fn) return fail(TDSE_EINVAL, "f_fn missing");
  if (prob->f_kind < 0 || prob->f_kind > 2) return fail(TDSE_EINVAL, "bad f_kind");
  if ((prob->A_kind == TDSE_A_PULSE_SIN2 || prob->A_kind == TDSE_A_PULSE_COS2) && !prob->A_params)
    return fail(TDSE_EINVAL, "A_params missing");
  if (prob->A_kind == TDSE_A_STEPWISE && !prob->A_steps) return fail(TDSE_EINVAL, "A_steps missing");
  if (prob->A_kind == TDSE_A_CALLBACK && !prob->A_fn) return fail(TDSE_EINVAL, "A_fn missing");
  if (prob->A_kind < 0 || prob->A_kind > 4) return fail(TDSE_EINVAL, "bad A_kind");

  tdse_plan_s* p = new (std::nothrow) tdse_plan_s();
  if (!p) return fail(TDSE_ENOMEM, "host allocation failed");
  p->dim = prob->dim;
  if (prob->dim == 3) {
    p->M0 = prob->M[0];
    p->Mmid = prob->M[1];
    p->M1 = prob->M[0] * prob->M[1];
    p->M2 = prob->M[2];
  } else {
    p->M1 = prob->dim == 2 ? prob->M[0] : 1;
    p->M2 = prob->dim == 2 ? prob->M[1] : prob->M[0];
  }
  p->P = (int64_t)p->M1 * p->M2;
  p->order = prob->order;
  p->ns = prob->n_start < 0 ? prob->order - 2 : prob->n_start;
  if (p->ns < prob->order - 2) {
    delete p;
    return fail(TDSE_EINVAL, "n_start must be at least order - 2");
  }
  p->L = prob->order / 2;
  p->nsteps = prob->nsteps;
  p->T = prob->T;
  p->dt = prob->T / prob->nsteps;
  p->nV = well ? 0 : (sampled ? 1 : prob->nV);
  if (sampled) {
    p->vkind = TDSE_V_SAMPLED;
    p->nsamp = (int64_t)prob->nsteps + 1;
  }
  if (well) {
    p->vkind = TDSE_V_MOVING_WELL;
    p->well[0] = prob->V_params[0];
    p->well[1] = 1.0 / (2.0 * prob->V_params[1] * prob->V_params[1]);
    // |x - centre + 2 pi k| <= 9.2 beta with |x - centre| <= pi
    p->well_k = std::floor((9.2 * prob->V_params[1] + M_PI) / (2.0 * M_PI));
    p->well[2] = prob->V_params[2];
    p->well[3] = prob->V_params[3];
  }
  p->precision = prob->precision;
  p->mu = adams_weights(p->order);
  p->rich = richardson_weights(p->L);
  const bool split = p->precision == TDSE_FP32_SPLIT;
  for (int g = 0; g < 2; ++g) {
    tdse_plan_s::Stage& S = p->st[g];
    const bool sp = split && g == 1;
    S.prec = sp ? P_SPLIT : P_FP64;
    S.cplx = sp ? 8 : 16;
    // the potential stays FP64 in both forms: rounded to FP32 it would be a
    // fixed perturbation of the Hamiltonian whose error grows linearly in time
    S.real = 8;
    const int64_t nfields = sampled ? p->nsamp : p->nV;
    if (g == 0 && nfields > 0)
      S.Vhost.assign((const char*)prob->V_fields, (const char*)(prob->V_fields + (size_t)nfields * p->P));
  }

  TimeFns& tf = p->tf;
  tf.dim = p->dim;
  tf.nV = p->nV;
  tf.nsteps = p->nsteps;
  tf.dt = p->dt;
  tf.f_kind = prob->f_kind;
  if (prob->f_kind == TDSE_F_SIN) tf.f_params.assign(prob->f_params, prob->f_params + 2 * p->nV);
  tf.f_fn = prob->f_fn;
  tf.f_ctx = prob->f_ctx;
  tf.A_kind = prob->A_kind;
  if (prob->A_kind == TDSE_A_PULSE_SIN2 || prob->A_kind == TDSE_A_PULSE_COS2)
    tf.A_params.assign(prob->A_params, prob->A_params + 3 + p->dim);
  if (prob->A_kind == TDSE_A_STEPWISE) tf.A_steps.assign(prob->A_steps, prob->A_steps + (size_t)p->nsteps * p->dim);
  tf.A_fn = prob->A_fn;
  tf.A_ctx = prob->A_ctx;
  tf.prepare();

  if (free_dom) {
    p->Vsrc.assign(prob->V_fields, prob->V_fields + (size_t)(sampled ? p->nsamp : p->nV) * p->P);
    p->st[0].Vhost.clear();
    p->st[1].Vhost.clear();
    const int s = plan_free(p, prob);
    if (s) {
      delete p;
      return s;
    }
    p->o_diag = p->total;
    p->total = align256(p->total + 64);
    *out = p;
    return TDSE_OK;
  }

  for (int g = 0; g < 2; ++g) {
    p->st[g].tw1 = twiddles(p->col_len(), p->st[g].prec == P_SPLIT);
    p->st[g].tw2 = twiddles(p->M2, p->st[g].prec == P_SPLIT);
    if (p->Mmid) p->st[g].tw3 = twiddles(p->Mmid, p->st[g].prec == P_SPLIT);
  }

  size_t off = 0;
  const size_t cbytes = (size_t)p->P * sizeof(double2);   // complex128 buffers
  p->o_B = off; off = align256(off + cbytes);
  p->o_u[0] = off; off = align256(off + cbytes);
  p->o_u[1] = off; off = align256(off + cbytes);
  for (int g = 0; g < (split ? 2 : 1); ++g) {
    tdse_plan_s::Stage& S = p->st[g];
    const size_t tbytes = (size_t)p->P * S.cplx;
    S.o_ring = off; off = align256(off + (size_t)(p->order - 1) * tbytes);
    S.o_tmp = off; off = align256(off + tbytes);
    if (g == 0) {
      S.o_V = off;
      off = align256(off + S.Vhost.size());
    } else {
      S.o_V = p->st[0].o_V;   // one FP64 copy of the potential serves both stages
    }
    S.o_tw1 = off; off = align256(off + S.tw1.size());
    S.o_tw2 = off; off = align256(off + S.tw2.size());
    S.o_tw3 = off; off = align256(off + S.tw3.size());
  }
  if (!split) {
    p->st[1] = p->st[0];
    p->st[1].Vhost.clear();   // no second upload
    p->st[1].tw1.clear();
    p->st[1].tw2.clear();
    p->st[1].tw3.clear();
  }
  p->o_ph = off; off = align256(off + (size_t)(p->order - 1) * (p->M1 + p->M2) * sizeof(double2));
  if (split) {   // the same table rounded to complex64, read by the split row pass
    p->o_ph32 = off;
    off = align256(off + (size_t)(p->order - 1) * (p->M1 + p->M2) * sizeof(float2));
  }
  p->o_diag = off; off = align256(off + 64);
  if (!split) {
    p->o_dbuf = off;
    off = align256(off + cbytes);
  }
  p->total_core = off;
  if (p->dim == 2 && !split && p->M1 == p->M2 && persist2d_supported(p->M2) && p->vkind == TDSE_V_FIELDS &&
      p->nsteps > p->ns + 1) {
    p->persist = true;
    build_persist2d(p);
    p->o_p2tab = off; off = align256(off + p->p2tab.size() * sizeof(double));
    p->o_p2S2 = off; off = align256(off + p->p2S2.size() * sizeof(double2));
    p->o_p2bar = off; off = align256(off + P2_BAR_WORDS * sizeof(unsigned));
  }
  if (p->dim == 1 && !split && run1d_supported(p->M2) && p->vkind != TDSE_V_SAMPLED) {
    p->run1d = true;
    build_run1d(p);
    p->o_r1tab = off; off = align256(off + p->r1tab.size() * sizeof(double));
    p->o_r1stab = off; off = align256(off + p->r1stab.size() * sizeof(double2));
  }
  p->total = off;
  *out = p;
  return TDSE_OK;
}

int tdse_workspace_size(tdse_plan_t p, size_t* bytes) {
  if (!p || !bytes) return fail(TDSE_EINVAL, "NULL argument");
  *bytes = p->total;
  return TDSE_OK;
}

int tdse_bind(tdse_plan_t p, void* ws, size_t bytes, void* stream) {
  if (!p || !ws) return fail(TDSE_EINVAL, "NULL argument");
  if (bytes < p->total) return fail(TDSE_ENOMEM, "workspace smaller than tdse_workspace_size");
  if (((uintptr_t)ws) & 255) return fail(TDSE_EINVAL, "workspace must be 256-byte aligned");
  p->drop_graph();
  p->ws = (char*)ws;
  p->ws_bytes = bytes;
  p->stream = (hipStream_t)stream;
  if (p->is_batch()) {
    p->batch_ready = false;
    const int s = bind_batch(p);
    if (s) return s;
    p->bound = true;
    p->cur = -1;
    return TDSE_OK;
  }
  for (int g = 0; g < 2; ++g) {
    const tdse_plan_s::Stage& S = p->st[g];
    if (!S.Vhost.empty())
      HIP_TRY(hipMemcpyAsync(p->ws + S.o_V, S.Vhost.data(), S.Vhost.size(), hipMemcpyHostToDevice, p->stream));
    if (!S.tw1.empty())
      HIP_TRY(hipMemcpyAsync(p->ws + S.o_tw1, S.tw1.data(), S.tw1.size(), hipMemcpyHostToDevice, p->stream));
    if (!S.tw2.empty())
      HIP_TRY(hipMemcpyAsync(p->ws + S.o_tw2, S.tw2.data(), S.tw2.size(), hipMemcpyHostToDevice, p->stream));
    if (!S.tw3.empty())
      HIP_TRY(hipMemcpyAsync(p->ws + S.o_tw3, S.tw3.data(), S.tw3.size(), hipMemcpyHostToDevice, p->stream));
  }
  if (p->run1d) {
    const int s = upload_run1d(p);
    if (s) return s;
  }
  if (p->persist) {
    const int s = upload_persist2d(p);
    if (s) return s;
  }
  if (p->free_space) {
    HIP_TRY(hipMemcpyAsync(p->ws + p->o_Vf, p->Vsrc.data(), p->Vsrc.size() * sizeof(double), hipMemcpyHostToDevice,
                           p->stream));
    for (int a = 0; a < (p->dim == 3 ? 3 : 2); ++a)
      HIP_TRY(hipMemcpyAsync(p->ws + p->fx[a].o_tab, p->fx[a].tables.data(), p->fx[a].tables.size(),
                             hipMemcpyHostToDevice, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->bound = true;
  p->cur = -1;
  return TDSE_OK;
}

int tdse_set_state(tdse_plan_t p, const void* u0, int32_t on_device) {
  if (!p || !u0) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->bound) return fail(TDSE_ESTATE, "tdse_bind must come first");
  if (p->is_batch()) {
    for (size_t i = 0; i < p->sub.size(); ++i) {
      const int s = tdse_set_state(p->sub[i], (const double2*)u0 + p->sub_elem[i], on_device);
      if (s) return s;
    }
    p->cur = 0;
    return TDSE_OK;
  }
  p->ucur = 0;
  p->uh_cur = 0;
  const size_t bytes = (size_t)p->P * sizeof(double2);
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(p->u(0), u0, bytes, hipMemcpyDeviceToDevice, p->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(p->u(0), u0, bytes, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  p->cur = 0;
  return TDSE_OK;
}

namespace {
int step_range(tdse_plan_s* p, int k);
}

int tdse_step(tdse_plan_t p, int32_t k) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "tdse_set_state must come first");
  if (k < 0) return fail(TDSE_EINVAL, "negative step count");
  if (p->cur + k > p->nsteps) return fail(TDSE_ESTATE, "stepping past T");
  if (p->guard_every <= 0) return step_range(p, k);
  // guarded: pieces of at most guard_every steps, each followed by the check
  while (k > 0) {
    const int c = std::min(k, p->guard_every);
    int s = step_range(p, c);
    if (!s) s = guard_check(p);
    if (s) return s;
    k -= c;
  }
  return TDSE_OK;
}

namespace {
int step_range(tdse_plan_s* p, int k) {
  if (p->is_batch()) return batch_step(p, k);
  const int end = p->cur + k;
  if (p->run1d) return k > 0 ? run1d_step(p, end) : TDSE_OK;
  if (p->persist && p->persist_on && end > p->ns + 1) {
    // start-up and the Adams start by the passes, the rest in one persistent launch
    for (int m = p->cur + 1; m <= p->ns + 1; ++m) {
      const int s = do_step(p, m, m == end);
      if (s) return s;
      p->cur = m;
    }
    const int s = persist2d_step(p, end, true);
    if (s <= 0) return s;
  }
  for (int m = p->cur + 1; m <= end; ++m) {
    const int s = do_step(p, m, m == end);
    if (s) return s;
    p->cur = m;
  }
  return TDSE_OK;
}
}  // namespace

int tdse_get_state(tdse_plan_t p, void* u, int32_t on_device) {
  if (!p || !u) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "no state");
  if (p->is_batch()) {
    for (size_t i = 0; i < p->sub.size(); ++i) {
      const int s = tdse_get_state(p->sub[i], (double2*)u + p->sub_elem[i], on_device);
      if (s) return s;
    }
    return TDSE_OK;
  }
  const size_t bytes = (size_t)p->P * sizeof(double2);
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(u, p->u(p->ucur), bytes, hipMemcpyDeviceToDevice, p->stream));
    return TDSE_OK;
  }
  HIP_TRY(hipMemcpyAsync(u, p->u(p->ucur), bytes, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const double* d = (const double*)u;
  for (size_t i = 0; i < 2 * (size_t)p->P; ++i)
    if (!std::isfinite(d[i])) return fail(TDSE_ENONFINITE, "state is not finite");
  return TDSE_OK;
}

// ---------------------------------------------- evaluation at arbitrary points

namespace {
struct FarLayout {
  size_t uh = 0, e1 = 0, e2 = 0, S = 0, total = 0;
};
FarLayout far_layout(const tdse_plan_s* p, int nx, int ny) {
  FarLayout L;
  const size_t N1 = (size_t)p->fx[0].N, N2 = (size_t)p->fx[1].N, z = sizeof(double2);
  size_t off = 0;
  L.uh = off; off = align256(off + (size_t)p->NM * z);
  L.e2 = off; off = align256(off + N2 * ny * z);
  if (p->dim == 2) {
    L.e1 = off; off = align256(off + N1 * nx * z);
    L.S = off; off = align256(off + N1 * ny * z);
  }
  L.total = off;
  return L;
}
int far_check(const tdse_plan_s* p, int nx, int ny) {
  if (p->is_batch() || !p->free_space) return fail(TDSE_EUNSUPPORTED, "evaluation at arbitrary points is for free-space plans");
  if (p->dim == 3) return fail(TDSE_EUNSUPPORTED, "evaluation at arbitrary points covers 1D and 2D plans");
  if (ny < 1 || nx < 1 || ny > (1 << 24) || nx > (1 << 24)) return fail(TDSE_EINVAL, "need 1 <= nx, ny <= 2^24");
  if (p->dim == 1 && nx != 1) return fail(TDSE_EINVAL, "a 1D plan takes nx = 1");
  // every table and product launch must fit a one-dimensional grid
  const int64_t N1 = p->fx[0].N, N2 = p->fx[1].N, lim = (int64_t)1 << 30;
  if (N2 * ny > lim || N1 * nx > lim || ((N1 + 31) / 32) * ((ny + 31) / 32) > lim ||
      ((nx + 31) / 32) * ((ny + 31) / 32) > lim)
    return fail(TDSE_EINVAL, "too many evaluation points");
  return TDSE_OK;
}
}  // namespace

int tdse_far_workspace_size(tdse_plan_t p, int32_t nx, int32_t ny, size_t* bytes) {
  if (!p || !bytes) return fail(TDSE_EINVAL, "NULL argument");
  const int s = far_check(p, nx, ny);
  if (s) return s;
  *bytes = far_layout(p, nx, ny).total;
  return TDSE_OK;
}

namespace {
// u at the tensor grid xs x ys from the mode state, with `work` (L.total
// bytes) holding uhat, the two tables and the first product; `timed`: the
// first product may be bracketed by profiling events
int far_eval(tdse_plan_s* p, const double* xs, int32_t nx, const double* ys, int32_t ny, void* out, char* w,
             const FarLayout& L, bool timed) {
  int s = TDSE_OK;
  double2* uh = (double2*)(w + L.uh);
  // uhat at the current time
  if (p->cur == 0) {
    s = fs_forward(p, 0.0, 1.0, 0.0, 0.0, 0.0, uh);   // F u0 (Section 3.3)
  } else if (p->cur <= p->ns) {
    HIP_TRY(hipMemcpyAsync(uh, p->UH(p->uh_cur), (size_t)p->NM * sizeof(double2), hipMemcpyDeviceToDevice, p->stream));
  } else if (p->cur == p->nsteps) {
    // uhat_N = B_N - i mu_0 dt F(V(t_N) u_N) (the implicit Adams step's mode update)
    s = fs_forward(p, p->t_at(p->nsteps), 0.0, 0.0, 0.0, -p->mu[0] * p->dt, uh);
    if (!s) {
      const hipError_t e = launch_adj_axpy(p->NM, p->B(), uh, 1.0, 0.0, uh, p->stream);
      if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("axpy: ") + hipGetErrorString(e));
    }
  } else {
    return fail(TDSE_ESTATE, "the mode state is kept at t = 0, the start-up steps and t = T only");
  }
  if (s) return s;
  const CFAxis a1 = cf_axis(p, 0), a2 = cf_axis(p, 1);
  const int N1 = a1.N, N2 = a2.N;
  double2* E2 = (double2*)(w + L.e2);
  hipError_t e = launch_far_table(a2.zeta, a2.wq, N2, ys, ny, E2, p->stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t first = p->ev_used;
  if (p->prof && timed) {
    e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) return fail(TDSE_EDEVICE, "hipEventCreate failed");
  }
  if (p->dim == 1) {
    // u(y_j) = sum_k uhat[k] E2[k][j]
    if (e == hipSuccess) e = launch_far_gemm(1, ny, N2, uh, N2, 1, E2, ny, 1, (double2*)out, ny, p->stream, e0, e1);
  } else {
    double2* E1 = (double2*)(w + L.e1);
    double2* S = (double2*)(w + L.S);
    if (e == hipSuccess) e = launch_far_table(a1.zeta, a1.wq, N1, xs, nx, E1, p->stream);
    // S[k1][j] = sum_k2 uhat[k1][k2] E2[k2][j]; u[i][j] = sum_k1 E1[k1][i] S[k1][j]
    if (e == hipSuccess) e = launch_far_gemm(N1, ny, N2, uh, N2, 1, E2, ny, 1, S, ny, p->stream, e0, e1);
    if (e == hipSuccess) e = launch_far_gemm(nx, ny, N1, E1, 1, nx, S, ny, 1, (double2*)out, ny, p->stream);
  }
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("far-evaluation kernels: ") + hipGetErrorString(e));
  if (e0) p->prof_marks.push_back({first, 2});
  return TDSE_OK;
}
}  // namespace

int tdse_far_eval(tdse_plan_t p, const double* xs, int32_t nx, const double* ys, int32_t ny, void* out, void* work,
                  size_t bytes) {
  if (!p || !ys || !out || !work || (p->dim == 2 && !xs)) return fail(TDSE_EINVAL, "NULL argument");
  int s = far_check(p, nx, ny);
  if (s) return s;
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "no state");
  const FarLayout L = far_layout(p, nx, ny);
  if (bytes < L.total) return fail(TDSE_ENOMEM, "far-evaluation workspace too small");
  if (((uintptr_t)work) % 256) return fail(TDSE_EINVAL, "far-evaluation workspace must be 256-byte aligned");
  return far_eval(p, xs, nx, ys, ny, out, (char*)work, L, true);
}

int tdse_far_eval_noalloc(tdse_plan_t p, const double* xs, int32_t nx, const double* ys, int32_t ny, void* out) {
  if (!p || !ys || !out || (p->dim == 2 && !xs)) return fail(TDSE_EINVAL, "NULL argument");
  int s = far_check(p, nx, ny);
  if (s) return s;
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "no state");
  const FarLayout L = far_layout(p, nx, ny);
  if (L.total > FAR_SCRATCH_BYTES)
    return fail(TDSE_ENOMEM, "tdse_far_eval_noalloc: needs " + std::to_string(L.total) + " bytes of workspace, above its " +
                                 std::to_string(FAR_SCRATCH_BYTES) + "-byte library array; use tdse_far_eval");
  void* scr = nullptr;
  const hipError_t e = far_scratch(&scr);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("library scratch array: ") + hipGetErrorString(e));
  return far_eval(p, xs, nx, ys, ny, out, (char*)scr, L, false);
}

int tdse_run(tdse_plan_t p, const void* u0, void* uT, int32_t on_device) {
  int s = tdse_set_state(p, u0, on_device);
  if (s) return s;
  if (!p->use_graph || p->prof) {
    s = tdse_step(p, p->nsteps);
    if (s) return s;
    return tdse_get_state(p, uT, on_device);
  }
  // with persistent Adams steps the graph holds the start-up and the Adams
  // start; the persistent launch (one per run) follows it outside the graph
  const int pre = (p->persist && p->persist_on) ? p->ns + 1 : p->nsteps;
  if (!p->gexec) {
    // capture the whole step sequence once; kernel arguments depend only on
    // the plan and the bound workspace
    HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    const int guard = p->guard_every;
    p->guard_every = 0;   // the check synchronizes: it runs after the replay
    s = tdse_step(p, pre);
    p->guard_every = guard;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      p->cur = -1;
      return s;
    }
    if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = g;
    e = hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      p->drop_graph();
      return fail(TDSE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    p->graph_ucur = p->ucur;
  }
  HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
  p->cur = pre;
  if (p->guard_every > 0) {
    s = guard_check(p);
    if (s) return s;
  }
  p->ucur = p->graph_ucur;
  for (tdse_plan_s* q : p->sub) {
    q->ucur = p->ucur_after[p->nsteps];
    q->cur = p->nsteps;
  }
  if (pre < p->nsteps) {
    s = tdse_step(p, p->nsteps - pre);
    if (s) return s;
  }
  return tdse_get_state(p, uT, on_device);
  // (a guarded run checks the state after the graph and after every guarded piece)
}

int tdse_graph(tdse_plan_t p, int32_t enable) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (enable && !p->stream) return fail(TDSE_EINVAL, "graph replay needs a non-default stream");
  p->use_graph = enable != 0;
  if (!p->use_graph) p->drop_graph();
  return TDSE_OK;
}

int tdse_query(tdse_plan_t p, int32_t key, double* value) {
  if (!p || !value) return fail(TDSE_EINVAL, "NULL argument");
  if (p->is_batch()) {
    const int n = (int)p->sub.size();
    if (key == TDSE_Q_INSTANCES) { *value = n; return TDSE_OK; }
    if (key == TDSE_Q_RESIDUAL) return history_residual(p, value);
    if (key == TDSE_Q_STATE_NORM) {
      if (p->state_norm < 0.0) return fail(TDSE_ESTATE, "no guard check has run");
      *value = p->state_norm;
      return TDSE_OK;
    }
    if (key == TDSE_Q_MODES) { *value = (double)p->P; return TDSE_OK; }
    if (key == TDSE_Q_STEPS_DONE) { *value = (double)p->cur; return TDSE_OK; }
    if (key >= TDSE_Q_INST_OFFSET && key < TDSE_Q_INST_OFFSET + n) {
      *value = (double)p->sub_elem[key - TDSE_Q_INST_OFFSET];
      return TDSE_OK;
    }
    if (key >= TDSE_Q_INST_EPT_COL && key < TDSE_Q_INST_EPT_COL + n) {
      *value = p->ept[0][key - TDSE_Q_INST_EPT_COL];
      return TDSE_OK;
    }
    if (key >= TDSE_Q_INST_EPT_ROW && key < TDSE_Q_INST_EPT_ROW + n) {
      *value = p->ept[1][key - TDSE_Q_INST_EPT_ROW];
      return TDSE_OK;
    }
    if (key == TDSE_Q_BYTES_PER_STEP || key == TDSE_Q_BYTES_COL || key == TDSE_Q_BYTES_ROW) {
      double sum = 0.0;
      for (tdse_plan_s* q : p->sub) {
        double v = 0.0;
        const int s = tdse_query(q, key, &v);
        if (s) return s;
        sum += v;
      }
      *value = sum;
      return TDSE_OK;
    }
    if (key < TDSE_Q_PROF_MS_COL || key > TDSE_Q_PROF_N_ROW) return tdse_query(p->sub[0], key, value);
  }
  if (key == TDSE_Q_MODES) { *value = (double)p->P; return TDSE_OK; }
  if (key == TDSE_Q_STEPS_DONE) { *value = (double)p->cur; return TDSE_OK; }
  if (key == TDSE_Q_DT) { *value = p->dt; return TDSE_OK; }
  if (key == TDSE_Q_RESIDUAL) return history_residual(p, value);
  if (key == TDSE_Q_STATE_NORM) {
    if (p->state_norm < 0.0) return fail(TDSE_ESTATE, "no guard check has run");
    *value = p->state_norm;
    return TDSE_OK;
  }
  if (key == TDSE_Q_PATH) {
    *value = p->run1d ? 1.0 : (p->persist && p->persist_on) ? 2.0 : 0.0;
    return TDSE_OK;
  }
  if (p->free_space && p->dim == 3 && key == TDSE_Q_BYTES_MID) {
    *value = 16.0 * (double)p->fx[0].N * p->fx[1].M * ((double)p->fx[2].N + p->fx[2].M);
    return TDSE_OK;
  }
  if (p->free_space && (key == TDSE_Q_BYTES_PER_STEP || key == TDSE_Q_BYTES_COL || key == TDSE_Q_BYTES_ROW)) {
    // column pass: tile (N1 x M2) in and out (32 per element) and the
    // potential fields (8 nV per grid point); row pass: tile in and out,
    // B in and out (32 per mode), n-2 history reads and one write (16 (n-1))
    // 3D: the row tile is N0 Nm M2, the column pass moves the N0 Mm M2 grid
    // array, and each middle-axis pass moves both (16 per element each)
    const bool d3 = p->dim == 3;
    const double Nm = d3 ? p->fx[2].N : 1.0, Mm = d3 ? p->fx[2].M : 1.0;
    const double tile = (double)p->fx[0].N * Nm * p->fx[1].M, grid = (double)p->fx[0].N * Mm * p->fx[1].M;
    const double col = 32.0 * grid + 8.0 * p->nV * (double)p->P;
    const double row = 32.0 * tile + (32.0 + 16.0 * (p->order - 1)) * (double)p->NM;
    const double mid = d3 ? 16.0 * (tile + grid) : 0.0;
    *value = key == TDSE_Q_BYTES_COL ? col : key == TDSE_Q_BYTES_ROW ? row : col + row + 2.0 * mid;
    return TDSE_OK;
  }
  if (key == TDSE_Q_FS_H) {
    if (!p->free_space) return fail(TDSE_EINVAL, "not a free-space plan");
    *value = p->H;
    return TDSE_OK;
  }
  {
    // per-axis contour keys: (field, physical axis)
    int field = -1, axis = 0;
    if (key >= TDSE_Q_FS_MODES && key < TDSE_Q_FS_MODES + 2) field = 0, axis = key - TDSE_Q_FS_MODES;
    else if (key >= TDSE_Q_FS_NE && key < TDSE_Q_FS_NE + 2) field = 1, axis = key - TDSE_Q_FS_NE;
    else if (key >= TDSE_Q_FS_H_AXIS && key < TDSE_Q_FS_H_AXIS + 2) field = 2, axis = key - TDSE_Q_FS_H_AXIS;
    else if (key >= TDSE_Q_FS_HSTEP && key < TDSE_Q_FS_HSTEP + 2) field = 3, axis = key - TDSE_Q_FS_HSTEP;
    else if (key >= TDSE_Q_FS_NU && key < TDSE_Q_FS_NU + 2) field = 4, axis = key - TDSE_Q_FS_NU;
    else if (key >= TDSE_Q_FS_K && key < TDSE_Q_FS_K + 2) field = 5, axis = key - TDSE_Q_FS_K;
    else if (key >= TDSE_Q_FS_CHEB && key < TDSE_Q_FS_CHEB + 2) field = 6, axis = key - TDSE_Q_FS_CHEB;
    else if (key >= TDSE_Q_FS_AXIS2 && key < TDSE_Q_FS_AXIS2 + 7) field = key - TDSE_Q_FS_AXIS2, axis = 2;
    if (field >= 0) {
      if (!p->free_space) return fail(TDSE_EINVAL, "not a free-space plan");
      if (axis >= p->dim) return fail(TDSE_EINVAL, "axis out of range");
      const int fa = fx_of(p->dim, axis);
      const tdse_plan_s::FAxis& F = p->fx[fa];
      switch (field) {
        case 0: *value = (double)F.N; break;
        case 1: *value = (double)F.NE; break;
        case 2: *value = p->Hfx[fa]; break;
        case 3: *value = F.h; break;
        case 4: *value = F.nu; break;
        case 5: *value = p->Hfx[fa] + (2.0 * 7 + F.NE - 1) * F.h; break;   // the last equispaced node is K - kappa h
        default: *value = F.NT; break;
      }
      return TDSE_OK;
    }
  }
  if ((key >= TDSE_Q_ALPERT_X && key < TDSE_Q_ALPERT_X + 16) || (key >= TDSE_Q_ALPERT_W && key < TDSE_Q_ALPERT_W + 16)) {
    if (!p->free_space) return fail(TDSE_EINVAL, "not a free-space plan");
    const bool xs = key < TDSE_Q_ALPERT_W;
    const int k = key - (xs ? TDSE_Q_ALPERT_X : TDSE_Q_ALPERT_W);
    if (k >= (int)p->alp_x.size()) return fail(TDSE_EINVAL, "Alpert index out of range");
    *value = xs ? p->alp_x[k] : p->alp_w[k];
    return TDSE_OK;
  }
  if (key == TDSE_Q_BYTES_PER_STEP) {
    // per mode: B in/out (32), history ring n-2 reads + 1 write (16 (n-1)),
    // two tile round trips (64), the potential fields (8 nV)
    const double c = (double)p->st[1].cplx, r = (double)p->st[1].real;
    const double per = 32.0 + c * (p->order - 1) + (p->dim == 3 ? 8 * c : p->dim == 2 ? 4 * c : 2 * c) + r * p->nV;
    *value = per * (double)p->P;
    return TDSE_OK;
  }
  if ((key >= TDSE_Q_PROF_MS_COL && key <= TDSE_Q_PROF_N_ROW) || key == TDSE_Q_PROF_MS_FAR ||
      key == TDSE_Q_PROF_N_FAR || key == TDSE_Q_PROF_MS_RUN1D || key == TDSE_Q_PROF_N_RUN1D ||
      key == TDSE_Q_PROF_MS_PERSIST || key == TDSE_Q_PROF_N_PERSIST || key == TDSE_Q_PROF_MS_MID ||
      key == TDSE_Q_PROF_N_MID) {
    const int kind = (key == TDSE_Q_PROF_MS_FAR || key == TDSE_Q_PROF_N_FAR)        ? 2
                     : (key == TDSE_Q_PROF_MS_RUN1D || key == TDSE_Q_PROF_N_RUN1D) ? 3
                     : (key == TDSE_Q_PROF_MS_PERSIST || key == TDSE_Q_PROF_N_PERSIST) ? 4
                     : (key == TDSE_Q_PROF_MS_MID || key == TDSE_Q_PROF_N_MID) ? 5
                     : ((key == TDSE_Q_PROF_MS_COL || key == TDSE_Q_PROF_N_COL) ? 0 : 1);
    const bool count = key == TDSE_Q_PROF_N_COL || key == TDSE_Q_PROF_N_ROW || key == TDSE_Q_PROF_N_FAR ||
                       key == TDSE_Q_PROF_N_RUN1D || key == TDSE_Q_PROF_N_PERSIST || key == TDSE_Q_PROF_N_MID;
    if (!p->prof_marks.empty()) HIP_TRY(hipStreamSynchronize(p->stream));
    double ms = 0.0, nk = 0.0;
    for (auto& mk : p->prof_marks) {
      if (mk.second != kind) continue;
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, p->ev_pool[mk.first], p->ev_pool[mk.first + 1]));
      ms += t;
      nk += 1.0;
    }
    *value = count ? nk : ms;
    return TDSE_OK;
  }
  if (key == TDSE_Q_BYTES_MID) {   // 3D middle-axis pass: tile in and out
    if (!p->Mmid) return fail(TDSE_EINVAL, "no middle axis (3D plans only)");
    *value = 2.0 * (double)p->st[1].cplx * (double)p->P;
    return TDSE_OK;
  }
  if (key == TDSE_Q_BYTES_COL || key == TDSE_Q_BYTES_ROW) {
    // column pass: tile in and out (32) + the potential fields (8 nV);
    // row pass: tile in and out (32), B in and out (32), n-2 history reads and
    // one history write (16 (n-1))
    const double c = (double)p->st[1].cplx, r = (double)p->st[1].real;
    const double per = key == TDSE_Q_BYTES_COL ? 2 * c + r * p->nV : 32.0 + 2 * c + c * (p->order - 1);
    *value = per * (double)p->P;
    return TDSE_OK;
  }
  if (key >= TDSE_Q_MU && key < TDSE_Q_MU + p->order) { *value = p->mu[key - TDSE_Q_MU]; return TDSE_OK; }
  if (key >= TDSE_Q_RICHARDSON && key < TDSE_Q_RICHARDSON + p->L) { *value = p->rich[key - TDSE_Q_RICHARDSON]; return TDSE_OK; }
  if (key >= TDSE_Q_PHI && key < TDSE_Q_PHI + p->dim) {
    double ph[3];
    p->tf.phi(p->T, ph);
    *value = ph[key - TDSE_Q_PHI];
    return TDSE_OK;
  }
  return fail(TDSE_EINVAL, "unknown query key");
}

int tdse_configure(tdse_plan_t p, int32_t key, int32_t value) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (key == TDSE_CFG_PERSISTENT) {
    if (value != 0 && value != 1) return fail(TDSE_EINVAL, "TDSE_CFG_PERSISTENT takes 0 or 1");
    if (p->cur > 0 && p->cur < p->nsteps) return fail(TDSE_ESTATE, "change the step path before or after a run");
    p->persist_on = value != 0;
    p->drop_graph();
    return TDSE_OK;
  }
  if (key == TDSE_CFG_GUARD) {
    if (value < 0) return fail(TDSE_EINVAL, "TDSE_CFG_GUARD takes a step count >= 0");
    p->guard_every = value;
    p->drop_graph();
    return TDSE_OK;
  }
  return fail(TDSE_EINVAL, "unknown configuration key");
}

int tdse_profile(tdse_plan_t p, int32_t enable) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  p->prof = enable != 0;
  p->ev_used = 0;
  p->prof_marks.clear();
  return TDSE_OK;
}

int tdse_plan_batch(const tdse_problem_t* probs, int32_t count, tdse_plan_t* out) {
  if (!probs || !out) return fail(TDSE_EINVAL, "NULL argument");
  *out = nullptr;
  if (count < 1 || count > 4096) return fail(TDSE_EINVAL, "count must be 1..4096");
  return plan_batch(probs, count, out);
}

int tdse_autotune(tdse_plan_t p, int32_t reps) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (!p->is_batch()) return fail(TDSE_EUNSUPPORTED, "autotuning applies to batch plans");
  if (!p->bound) return fail(TDSE_ESTATE, "tdse_bind must come first");
  if (reps < 1 || reps > 1000) return fail(TDSE_EINVAL, "reps must be 1..1000");
  return autotune_batch(p, reps);
}

int tdse_set_instance_state(tdse_plan_t p, int32_t instance, const void* u0, int32_t on_device) {
  if (!p || !u0) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->is_batch()) return instance == 0 ? tdse_set_state(p, u0, on_device) : fail(TDSE_EINVAL, "instance out of range");
  if (instance < 0 || instance >= (int)p->sub.size()) return fail(TDSE_EINVAL, "instance out of range");
  if (!p->bound) return fail(TDSE_ESTATE, "tdse_bind must come first");
  const int s = tdse_set_state(p->sub[instance], u0, on_device);
  if (s) return s;
  bool all = true;
  for (tdse_plan_s* q : p->sub) all = all && q->cur == 0;
  p->cur = all ? 0 : -1;
  return TDSE_OK;
}

int tdse_get_instance_state(tdse_plan_t p, int32_t instance, void* u, int32_t on_device) {
  if (!p || !u) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->is_batch()) return instance == 0 ? tdse_get_state(p, u, on_device) : fail(TDSE_EINVAL, "instance out of range");
  if (instance < 0 || instance >= (int)p->sub.size()) return fail(TDSE_EINVAL, "instance out of range");
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "no state");
  return tdse_get_state(p->sub[instance], u, on_device);
}


int tdse_set_field(tdse_plan_t p, const double* A_steps) {
  if (!p || !A_steps) return fail(TDSE_EINVAL, "NULL argument");
  if (p->is_batch()) {
    size_t off = 0;
    for (tdse_plan_s* q : p->sub) {
      const int s = tdse_set_field(q, A_steps + off);
      if (s) return s;
      off += (size_t)q->nsteps * q->dim;
    }
    p->drop_graph();
    if (p->batch_ready) {
      const int s = batch_record(p);
      if (s) return s;
      HIP_TRY(hipStreamSynchronize(p->stream));
      HIP_TRY(hipMemcpy(p->ws + p->o_args, p->bargs.data(), p->bargs.size() * sizeof(LineArgs), hipMemcpyHostToDevice));
    }
    return TDSE_OK;
  }
  if (p->tf.A_kind != TDSE_A_STEPWISE) return fail(TDSE_EINVAL, "tdse_set_field needs a stepwise-field plan");
  p->tf.A_steps.assign(A_steps, A_steps + (size_t)p->nsteps * p->dim);
  p->tf.prepare();
  p->drop_graph();
  if (p->run1d) {
    build_run1d(p);
    if (p->bound) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      HIP_TRY(hipMemcpy(p->ws + p->o_r1tab, p->r1tab.data(), p->r1tab.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  if (p->persist) {
    build_persist2d(p);
    if (p->bound) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      HIP_TRY(hipMemcpy(p->ws + p->o_p2tab, p->p2tab.data(), p->p2tab.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  return TDSE_OK;
}

int tdse_adjoint_workspace_size(tdse_plan_t p, int32_t checkpoint_every, size_t* bytes) {
  if (!p || !bytes) return fail(TDSE_EINVAL, "NULL argument");
  size_t b = 0;
  if (p->is_batch()) {
    for (tdse_plan_s* q : p->sub) b = std::max(b, adj_layout(q, checkpoint_every).total);
    b = align256(b) * (size_t)adj_workers(p);
  } else {
    b = adj_layout(p, checkpoint_every).total;
  }
  *bytes = b;
  return TDSE_OK;
}

int tdse_adjoint_streams(tdse_plan_t p, int32_t streams) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (streams < 1 || streams > 16) return fail(TDSE_EINVAL, "streams must be 1..16");
  p->adj_streams = streams;
  return TDSE_OK;
}

int tdse_adjoint(tdse_plan_t p, void* ws, size_t bytes, int32_t checkpoint_every, const void* u0, const void* lambda_T,
                 int32_t on_device, double* dF_dA, void* dF_du0) {
  if (!p || !ws || !u0 || !lambda_T) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->bound) return fail(TDSE_ESTATE, "tdse_bind must come first");
  if (!p->is_batch()) return adjoint_single(p, (char*)ws, bytes, checkpoint_every, u0, lambda_T, on_device, dF_dA, dF_du0);
  const int nsub = (int)p->sub.size();
  std::vector<size_t> aoff(nsub + 1, 0);
  size_t slice = 0;
  for (int i = 0; i < nsub; ++i) {
    aoff[i + 1] = aoff[i] + (size_t)p->sub[i]->nsteps * p->sub[i]->dim;
    slice = std::max(slice, adj_layout(p->sub[i], checkpoint_every).total);
  }
  slice = align256(slice);
  const int T = adj_workers(p);
  if (bytes < slice * (size_t)T) return fail(TDSE_ENOMEM, "adjoint workspace smaller than tdse_adjoint_workspace_size");
  auto one = [&](int i, char* w) {
    tdse_plan_s* q = p->sub[i];
    const int64_t e = p->sub_elem[i];
    return adjoint_single(q, w, slice, checkpoint_every, (const double2*)u0 + e, (const double2*)lambda_T + e,
                          on_device, dF_dA ? dF_dA + aoff[i] : nullptr,
                          dF_du0 ? (void*)((double2*)dF_du0 + e) : nullptr);
  };
  if (T == 1) {
    for (int i = 0; i < nsub; ++i) {
      const int s = one(i, (char*)ws);
      if (s) return s;
    }
    p->cur = -1;
    return TDSE_OK;
  }
  // T workers, worker t takes instances t, t + T, ...: a stream each
  // (non-blocking, default priority), ordered after the work already on the
  // bound stream, and the bound stream ordered after all of them
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::vector<hipStream_t> streams(T, nullptr);
  std::vector<hipEvent_t> evs(T + 1, nullptr);
  int s = TDSE_OK;
  auto cleanup = [&]() {
    for (hipStream_t x : streams)
      if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t x : evs)
      if (x) (void)hipEventDestroy(x);
  };
  for (int k = 0; k <= T && !s; ++k) s = adj_err(hipEventCreateWithFlags(&evs[k], hipEventDisableTiming), "adjoint event");
  for (int t = 0; t < T && !s; ++t) s = adj_err(hipStreamCreateWithFlags(&streams[t], hipStreamNonBlocking), "adjoint stream");
  if (!s) s = adj_err(hipEventRecord(evs[T], p->stream), "adjoint event");
  for (int t = 0; t < T && !s; ++t) s = adj_err(hipStreamWaitEvent(streams[t], evs[T], 0), "adjoint wait");
  if (s) {
    cleanup();
    return s;
  }
  std::vector<int> st(T, TDSE_OK);
  std::vector<std::string> msg(T);
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) {
    pool.emplace_back([&, t]() {
      if (hipSetDevice(dev) != hipSuccess) {
        st[t] = TDSE_EDEVICE;
        msg[t] = "adjoint worker: hipSetDevice failed";
        return;
      }
      char* w = (char*)ws + (size_t)t * slice;
      for (int i = t; i < nsub && st[t] == TDSE_OK; i += T) {
        tdse_plan_s* q = p->sub[i];
        hipStream_t keep = q->stream;
        q->stream = streams[t];
        st[t] = one(i, w);
        q->stream = keep;
      }
      if (st[t]) msg[t] = g_last_error;   // the error text is per thread
    });
  }
  for (std::thread& th : pool) th.join();
  for (int t = 0; t < T; ++t) {
    if (!s && st[t]) s = fail(st[t], msg[t]);
    if (hipEventRecord(evs[t], streams[t]) == hipSuccess) (void)hipStreamWaitEvent(p->stream, evs[t], 0);
  }
  for (hipStream_t x : streams) (void)hipStreamSynchronize(x);
  cleanup();
  p->cur = -1;
  return s;
}

void tdse_destroy(tdse_plan_t p) { delete p; }

}  // extern "C"
