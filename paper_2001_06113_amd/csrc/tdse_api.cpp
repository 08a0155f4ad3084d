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
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
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

  void A_at(double t, double* out) const {
    if (A_kind == TDSE_A_CALLBACK) {
      A_fn(t, out, A_ctx);
    } else {
      for (int a = 0; a < dim; ++a) out[a] = 0.0;
    }
  }

  void gl_piece(double a, double b, double* out) const {
    double tmp[2];
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
      double piece[2];
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
    for (int a = 0; a < 2; ++a) out[a] = 0.0;
    switch (A_kind) {
      case TDSE_A_PULSE_SIN2: {
        const double s = pulse_integral(t, A_params[0], A_params[1], A_params[2]);
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
          double piece[2] = {0, 0};
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

struct tdse_plan_s {
  int dim = 1, M1 = 1, M2 = 1;
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
    size_t o_ring = 0, o_tmp = 0, o_V = 0, o_tw1 = 0, o_tw2 = 0;
    std::vector<char> Vhost, tw1, tw2;   // host copies uploaded at bind
  } st[2];
  // workspace layout
  size_t o_B = 0, o_u[2] = {0, 0}, o_ph = 0, total = 0;
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
  ~tdse_plan_s() {
    drop_graph();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }

  double2* B() const { return (double2*)(ws + o_B); }
  void* ring(int g) const { return ws + st[g].o_ring; }
  void* ring_slot(int g, int s) const { return ws + st[g].o_ring + (size_t)s * P * st[g].cplx; }
  void* tmp(int g) const { return ws + st[g].o_tmp; }
  double2* u(int i) const { return (double2*)(ws + o_u[i]); }
  const void* V(int g) const { return ws + st[g].o_V; }
  double2* ph() const { return (double2*)(ws + o_ph); }
  const void* tw(int g, int axis) const { return ws + (axis == 0 ? st[g].o_tw1 : st[g].o_tw2); }
  bool split() const { return precision == TDSE_FP32_SPLIT; }

  double t_at(int m) const { return m * dt; }
  void fV_at(double t, double* f) const {
    for (int r = 0; r < MAXV; ++r) f[r] = r < nV ? tf.f(r, t) : 0.0;
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
  a.V = p->V(g);
  a.nV = p->nV;
  a.vstride = p->P;
  a.scale = 1.0 / (double)p->P;
  a.ring = p->ring(g);
  a.ring_stride = p->P;
  a.Bm = p->B();
  a.ph = p->ph();
  a.slot_w = -1;
  return a;
}

// column-pass geometry: lines are the M2 columns, elements step by M2
void col_geom(const tdse_plan_s* p, int g, LineArgs& a) {
  a.line_stride = 1;
  a.elem_stride = p->M2;
  a.nlines = p->M2;
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
  double pb[2], pa[2];
  if (stepgrid) p->tf.phi(p->t_at(m_b), pb);
  else p->tf.phi(t_b, pb);
  for (int j = 1; j <= nj; ++j) {
    if (stepgrid) p->tf.phi(p->t_at(m_b - j), pa);
    else p->tf.phi(t_b - j * tau, pa);
    a.req.tau[j - 1] = j * tau;
    if (p->dim == 2) {
      a.req.dphi1[j - 1] = pb[0] - pa[0];
      a.req.dphi2[j - 1] = pb[1] - pa[1];
    } else {
      a.req.dphi1[j - 1] = 0.0;
      a.req.dphi2[j - 1] = pb[0] - pa[0];
    }
  }
}

int launch(const tdse_plan_s* p, int g, bool col, const LineArgs& a, hipEvent_t e0 = nullptr,
           hipEvent_t e1 = nullptr) {
  const int prec = p->st[g].prec;
  hipError_t e = col ? launch_col_pass(prec, p->M1, a, p->stream, e0, e1)
                     : launch_row_pass(prec, p->M2, a, p->stream, e0, e1);
  if (e != hipSuccess) return fail(TDSE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
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
  p->fV_at(p->t_at(m), a.fV);
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
    p->fV_at(t, a.fV);
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
      p->fV_at(ts1, c.fV);
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
  if (p->split()) {
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
  p->fV_at(p->t_at(m), c.fV);
  c.csolve = p->mu[0] * p->dt;
  c.uout = p->u(p->ucur);
  return launch(p, g, true, c);
}

// Implicit Adams step m (eq. (uadamsk)), stage 1.
int op_am_step(tdse_plan_s* p, int m, bool write_u) {
  const int n = p->order, g = 1;
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
  p->fV_at(p->t_at(m), c.fV);
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
  return launch_timed(p, g, false, r);
}

bool good_len(int M) { return M >= 8 && M <= 3072 && M % 2 == 0 && line_length_supported(M); }

}  // namespace

// ================================================================ C ABI

extern "C" {

const char* tdse_status_string(int status) {
  switch (status) {
    case TDSE_OK: return "TDSE_OK";
    case TDSE_EINVAL: return "TDSE_EINVAL: invalid argument";
    case TDSE_EUNSUPPORTED: return "TDSE_EUNSUPPORTED: not supported by this build";
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
  if (prob->dim != 1 && prob->dim != 2) return fail(prob->dim == 3 ? TDSE_EUNSUPPORTED : TDSE_EINVAL, "dim must be 1 or 2");
  if (prob->domain != TDSE_PERIODIC) return fail(TDSE_EUNSUPPORTED, "free-space domain is not available in this build");
  if (prob->precision != TDSE_FP64 && prob->precision != TDSE_FP32_SPLIT) return fail(TDSE_EINVAL, "unknown precision");
  for (int a = 0; a < prob->dim; ++a)
    if (!good_len(prob->M[a])) return fail(TDSE_EINVAL, "grid size must be 2^a or 3*2^a, 8..3072");
  if (!(prob->T > 0.0) || prob->nsteps < 1) return fail(TDSE_EINVAL, "need T > 0 and nsteps >= 1");
  if (prob->order < 2 || prob->order > 8 || prob->order % 2) return fail(TDSE_EINVAL, "order must be 2, 4, 6 or 8");
  if (prob->nV < 1 || prob->nV > MAXV || !prob->V_fields) return fail(TDSE_EINVAL, "need 1..8 potential fields");
  if (prob->f_kind == TDSE_F_SIN && !prob->f_params) return fail(TDSE_EINVAL, "f_params missing");
  if (prob->f_kind == TDSE_F_CALLBACK && !prob->f_fn) return fail(TDSE_EINVAL, "f_fn missing");
  if (prob->f_kind < 0 || prob->f_kind > 2) return fail(TDSE_EINVAL, "bad f_kind");
  if (prob->A_kind == TDSE_A_PULSE_SIN2 && !prob->A_params) return fail(TDSE_EINVAL, "A_params missing");
  if (prob->A_kind == TDSE_A_STEPWISE && !prob->A_steps) return fail(TDSE_EINVAL, "A_steps missing");
  if (prob->A_kind == TDSE_A_CALLBACK && !prob->A_fn) return fail(TDSE_EINVAL, "A_fn missing");
  if (prob->A_kind < 0 || prob->A_kind > 3) return fail(TDSE_EINVAL, "bad A_kind");

  tdse_plan_s* p = new (std::nothrow) tdse_plan_s();
  if (!p) return fail(TDSE_ENOMEM, "host allocation failed");
  p->dim = prob->dim;
  p->M1 = prob->dim == 2 ? prob->M[0] : 1;
  p->M2 = prob->dim == 2 ? prob->M[1] : prob->M[0];
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
  p->nV = prob->nV;
  p->precision = prob->precision;
  p->mu = adams_weights(p->order);
  p->rich = richardson_weights(p->L);
  const bool split = p->precision == TDSE_FP32_SPLIT;
  for (int g = 0; g < 2; ++g) {
    tdse_plan_s::Stage& S = p->st[g];
    const bool sp = split && g == 1;
    S.prec = sp ? P_SPLIT : P_FP64;
    S.cplx = sp ? 8 : 16;
    S.real = sp ? 4 : 8;
    const size_t n = (size_t)p->nV * p->P;
    S.Vhost.resize(n * S.real);
    for (size_t q = 0; q < n; ++q) {
      if (sp) ((float*)S.Vhost.data())[q] = (float)prob->V_fields[q];
      else ((double*)S.Vhost.data())[q] = prob->V_fields[q];
    }
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
  if (prob->A_kind == TDSE_A_PULSE_SIN2) tf.A_params.assign(prob->A_params, prob->A_params + 3 + p->dim);
  if (prob->A_kind == TDSE_A_STEPWISE) tf.A_steps.assign(prob->A_steps, prob->A_steps + (size_t)p->nsteps * p->dim);
  tf.A_fn = prob->A_fn;
  tf.A_ctx = prob->A_ctx;
  tf.prepare();

  for (int g = 0; g < 2; ++g) {
    p->st[g].tw1 = twiddles(p->M1, p->st[g].prec == P_SPLIT);
    p->st[g].tw2 = twiddles(p->M2, p->st[g].prec == P_SPLIT);
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
    S.o_V = off; off = align256(off + S.Vhost.size());
    S.o_tw1 = off; off = align256(off + S.tw1.size());
    S.o_tw2 = off; off = align256(off + S.tw2.size());
  }
  if (!split) {
    p->st[1] = p->st[0];
    p->st[1].Vhost.clear();   // no second upload
    p->st[1].tw1.clear();
    p->st[1].tw2.clear();
  }
  p->o_ph = off; off = align256(off + (size_t)(p->order - 1) * (p->M1 + p->M2) * sizeof(double2));
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
  for (int g = 0; g < 2; ++g) {
    const tdse_plan_s::Stage& S = p->st[g];
    if (S.Vhost.empty()) continue;
    HIP_TRY(hipMemcpyAsync(p->ws + S.o_V, S.Vhost.data(), S.Vhost.size(), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->ws + S.o_tw1, S.tw1.data(), S.tw1.size(), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->ws + S.o_tw2, S.tw2.data(), S.tw2.size(), hipMemcpyHostToDevice, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->bound = true;
  p->cur = -1;
  return TDSE_OK;
}

int tdse_set_state(tdse_plan_t p, const void* u0, int32_t on_device) {
  if (!p || !u0) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->bound) return fail(TDSE_ESTATE, "tdse_bind must come first");
  p->ucur = 0;
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

int tdse_step(tdse_plan_t p, int32_t k) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "tdse_set_state must come first");
  if (k < 0) return fail(TDSE_EINVAL, "negative step count");
  if (p->cur + k > p->nsteps) return fail(TDSE_ESTATE, "stepping past T");
  const int end = p->cur + k;
  for (int m = p->cur + 1; m <= end; ++m) {
    int s = TDSE_OK;
    if (m <= p->ns) {
      if (m == 1) s = op_history(p, 0);
      if (!s) s = op_richardson(p, m);
      if (!s) s = op_history(p, m);
    } else {
      if (m == p->ns + 1) {
        if (p->ns == 0) s = op_history(p, 0);
        if (!s) s = op_am_init(p);
      }
      if (!s) s = op_am_step(p, m, m == end);
    }
    if (s) return s;
    p->cur = m;
  }
  return TDSE_OK;
}

int tdse_get_state(tdse_plan_t p, void* u, int32_t on_device) {
  if (!p || !u) return fail(TDSE_EINVAL, "NULL argument");
  if (!p->bound || p->cur < 0) return fail(TDSE_ESTATE, "no state");
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

int tdse_run(tdse_plan_t p, const void* u0, void* uT, int32_t on_device) {
  int s = tdse_set_state(p, u0, on_device);
  if (s) return s;
  if (!p->use_graph || p->prof) {
    s = tdse_step(p, p->nsteps);
    if (s) return s;
    return tdse_get_state(p, uT, on_device);
  }
  if (!p->gexec) {
    // capture the whole step sequence once; kernel arguments depend only on
    // the plan and the bound workspace
    HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    s = tdse_step(p, p->nsteps);
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
  p->cur = p->nsteps;
  p->ucur = p->graph_ucur;
  return tdse_get_state(p, uT, on_device);
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
  if (key == TDSE_Q_MODES) { *value = (double)p->P; return TDSE_OK; }
  if (key == TDSE_Q_STEPS_DONE) { *value = (double)p->cur; return TDSE_OK; }
  if (key == TDSE_Q_DT) { *value = p->dt; return TDSE_OK; }
  if (key == TDSE_Q_BYTES_PER_STEP) {
    // per mode: B in/out (32), history ring n-2 reads + 1 write (16 (n-1)),
    // two tile round trips (64), the potential fields (8 nV)
    const double c = (double)p->st[1].cplx, r = (double)p->st[1].real;
    const double per = 32.0 + c * (p->order - 1) + (p->dim == 2 ? 4 * c : 2 * c) + r * p->nV;
    *value = per * (double)p->P;
    return TDSE_OK;
  }
  if (key >= TDSE_Q_PROF_MS_COL && key <= TDSE_Q_PROF_N_ROW) {
    const int kind = (key == TDSE_Q_PROF_MS_COL || key == TDSE_Q_PROF_N_COL) ? 0 : 1;
    const bool count = key >= TDSE_Q_PROF_N_COL;
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
    double ph[2];
    p->tf.phi(p->T, ph);
    *value = ph[key - TDSE_Q_PHI];
    return TDSE_OK;
  }
  return fail(TDSE_EINVAL, "unknown query key");
}

int tdse_profile(tdse_plan_t p, int32_t enable) {
  if (!p) return fail(TDSE_EINVAL, "NULL plan");
  p->prof = enable != 0;
  p->ev_used = 0;
  p->prof_marks.clear();
  return TDSE_OK;
}

void tdse_destroy(tdse_plan_t p) { delete p; }

}  // extern "C"
