// ThreadSanitizer driver (host CPU build, test harness only): a batch plan's
// adjoint run from several host threads through the C ABI, on the emulated
// kernels, compared bit for bit with the one-thread run.
//
// The batch holds uneven periodic instances with stepwise fields, so every
// worker re-enters the per-instance forward recomputation, checkpointing and
// reverse sweep that the library's worker pool runs concurrently; any data
// race in that host code is reported by the sanitizer (exit code 66).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "tdse.h"

namespace {

struct Inst {
  int dim, M0, M1;
  std::vector<double> V, A;
  std::vector<double> u0;   // interleaved complex
  int P() const { return dim == 2 ? M0 * M1 : M0; }
};

Inst make(int dim, int M0, int M1, int nsteps, int seed) {
  Inst I{dim, M0, M1, {}, {}, {}};
  const int P = I.P();
  I.V.resize(P);
  I.u0.resize(2 * (size_t)P);
  const double pi = 3.14159265358979323846;
  double nrm = 0.0;
  for (int i = 0; i < P; ++i) {
    const int a = dim == 2 ? i / M1 : i, b = dim == 2 ? i % M1 : 0;
    const double x = -pi + 2 * pi * a / M0, y = dim == 2 ? -pi + 2 * pi * b / M1 : 0.0;
    I.V[i] = -(2.0 + seed) * std::cos(x) - (dim == 2 ? 1.5 * std::cos(y + 0.3) : 0.0);
    const double g = std::exp(-((x - 0.2 * seed) * (x - 0.2 * seed) + y * y) / 0.3);
    I.u0[2 * i] = g * std::cos(x);
    I.u0[2 * i + 1] = g * std::sin(2 * x);
    nrm += g * g;
  }
  for (double& v : I.u0) v /= std::sqrt(nrm);
  I.A.resize((size_t)nsteps * dim);
  for (int m = 0; m < nsteps; ++m)
    for (int c = 0; c < dim; ++c) I.A[(size_t)m * dim + c] = 0.7 * std::sin(0.9 * m + seed + c);
  return I;
}

int check(int s, const char* what) {
  if (s) {
    std::fprintf(stderr, "%s: %s (%s)\n", what, tdse_status_string(s), tdse_last_error());
    std::exit(2);
  }
  return s;
}

}  // namespace

// Negative control: two threads increment one counter with no
// synchronization, a race the sanitizer must report (it proves the
// instrumentation is active in this build).
int planted_race() {
  static int counter = 0;
  std::thread a([] { for (int i = 0; i < 1000; ++i) ++counter; });
  std::thread b([] { for (int i = 0; i < 1000; ++i) ++counter; });
  a.join();
  b.join();
  std::printf("planted race: counter %d\n", counter);
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "--planted-race") == 0) return planted_race();
  // small enough for the sanitizer's cost on the emulated fibers: order 4
  // (two Richardson start-up steps of three sub-steps each), then two
  // implicit Adams steps; two instances, so two workers run at once
  const int nsteps = 4;
  std::vector<Inst> inst = {make(1, 64, 1, nsteps, 0), make(2, 64, 64, nsteps, 1)};
  std::vector<tdse_problem_t> probs(inst.size());
  for (size_t i = 0; i < inst.size(); ++i) {
    tdse_problem_t& p = probs[i];
    std::memset(&p, 0, sizeof(p));
    p.dim = inst[i].dim;
    p.domain = TDSE_PERIODIC;
    p.M[0] = inst[i].M0;
    p.M[1] = inst[i].M1;
    p.T = 0.1;
    p.nsteps = nsteps;
    p.order = 4;
    p.n_start = -1;
    p.precision = TDSE_FP64;
    p.nV = 1;
    p.V_fields = inst[i].V.data();
    p.A_kind = TDSE_A_STEPWISE;
    p.A_steps = inst[i].A.data();
  }
  tdse_plan_t plan = nullptr;
  check(tdse_plan_batch(probs.data(), (int)probs.size(), &plan), "tdse_plan_batch");
  size_t wsb = 0;
  check(tdse_workspace_size(plan, &wsb), "tdse_workspace_size");
  std::vector<char> wsraw(wsb + 512);
  char* ws = wsraw.data() + ((256 - ((uintptr_t)wsraw.data() & 255)) & 255);
  check(tdse_bind(plan, ws, wsb, nullptr), "tdse_bind");
  size_t total = 0, nA = 0;
  for (const Inst& I : inst) {
    total += I.P();
    nA += (size_t)nsteps * I.dim;
  }
  std::vector<double> u0(2 * total), lam(2 * total);
  size_t o = 0;
  for (const Inst& I : inst) {
    std::memcpy(&u0[2 * o], I.u0.data(), 2 * sizeof(double) * I.P());
    for (int i = 0; i < I.P(); ++i) {   // a dipole-like seed: x_a u0
      const int a = I.dim == 2 ? i / I.M1 : i;
      const double x = -3.14159265358979323846 + 2 * 3.14159265358979323846 * a / I.M0;
      lam[2 * (o + i)] = x * I.u0[2 * i];
      lam[2 * (o + i) + 1] = x * I.u0[2 * i + 1];
    }
    o += I.P();
  }
  std::vector<std::vector<double>> gA, g0;
  for (int streams : {1, 2}) {
    check(tdse_adjoint_streams(plan, streams), "tdse_adjoint_streams");
    size_t ab = 0;
    check(tdse_adjoint_workspace_size(plan, 0, &ab), "tdse_adjoint_workspace_size");
    std::vector<char> araw(ab + 512);
    char* aw = araw.data() + ((256 - ((uintptr_t)araw.data() & 255)) & 255);
    std::vector<double> ga(nA), gu(2 * total);
    check(tdse_adjoint(plan, aw, ab, 0, u0.data(), lam.data(), 1, ga.data(), gu.data()), "tdse_adjoint");
    gA.push_back(ga);
    g0.push_back(gu);
  }
  int bad = 0;
  for (size_t r = 1; r < gA.size(); ++r) {
    if (std::memcmp(gA[r].data(), gA[0].data(), nA * sizeof(double)) != 0) bad |= 1;
    if (std::memcmp(g0[r].data(), g0[0].data(), 2 * total * sizeof(double)) != 0) bad |= 2;
  }
  double mx = 0.0;
  for (double v : gA[0]) mx = std::fmax(mx, std::fabs(v));
  tdse_destroy(plan);
  std::printf("batch adjoint from 1 and 2 threads: %s (max |dJ/dA| %.3e, %zu samples)\n",
              bad ? "DIFFER" : "bitwise equal", mx, nA);
  return bad ? 1 : (mx > 0.0 ? 0 : 3);
}
