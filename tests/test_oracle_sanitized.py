"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, g++) and driven through every entry point of mps_oracle.h on
small 2-D and 3-D tanks: every pressure model, gradient, source and
Laplacian option, the two-phase model with the eddy viscosity, the
dual-number rollout and the warm-started run.  Any out-of-bounds access,
use after free, leak or undefined operation ends the driver with an error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "mps_oracle.h"

static unsigned long long rng = 2105;
static double urand() {                       // uniform in [0, 1)
  rng = rng * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(rng >> 11) / 9007199254740992.0;
}

struct Case { std::vector<double> pos, vel; std::vector<int8_t> type; };

// fluid block of m^dim on the lattice, 2 wall + 2 dummy layers below,
// positions jittered by 5 % of l0, random velocities
static Case tank(int dim, int m, double l0) {
  Case c;
  int lo = -4, hi = m + 4;
  int nz = dim == 3 ? 1 : 0;
  for (int k = (dim == 3 ? lo : 0); k < (dim == 3 ? hi : 1); ++k)
    for (int j = -4; j < m; ++j)
      for (int i = lo; i < hi; ++i) {
        bool fluid = j >= 0 && i >= 0 && i < m && (nz == 0 || (k >= 0 && k < m));
        bool below = j < 0;
        if (!fluid && !below) continue;
        int8_t t = fluid ? 0 : (j >= -2 ? 1 : 2);
        double x[3] = {(i + 0.5) * l0, (j + 0.5) * l0, (k + 0.5) * l0};
        if (dim == 3) { x[2] = x[1]; x[1] = (k + 0.5) * l0; }
        for (int a = 0; a < dim; ++a) {
          double jit = fluid ? 0.1 * (urand() - 0.5) * l0 : 0.0;
          c.pos.push_back(x[a] + jit);
          c.vel.push_back(fluid ? 0.1 * (urand() - 0.5) : 0.0);
        }
        c.type.push_back(t);
      }
  return c;
}

static orc_params params(int dim, double l0, const Case& c) {
  orc_params P = {};
  P.dim = dim; P.pmode = 0; P.kernel = 0; P.grad = 0; P.clamp = 1;
  P.max_neigh = 300; P.cg_maxit = 10000;
  P.l0 = l0; P.re_n = 2.1 * l0; P.re_lap = (dim == 2 ? 4.0 : 3.1) * l0;
  P.rho = 1000; P.nu = 1e-6; P.g[dim - 1] = -9.81; P.dt = 5e-4; P.beta = 0.97;
  P.c0 = 20; P.gamma = 7; P.alpha = 1e-7; P.cg_tol = 1e-9;
  P.cell_size = P.re_lap * (1.0 + std::ldexp(1.0, -20));
  size_t n = c.type.size();
  for (int a = 0; a < dim; ++a) {
    double mn = 1e30, mx = -1e30;
    for (size_t i = 0; i < n; ++i) {
      mn = std::fmin(mn, c.pos[i * dim + a]);
      mx = std::fmax(mx, c.pos[i * dim + a]);
    }
    P.grid_lo[a] = mn - P.cell_size;
    P.grid_n[a] = (int)std::ceil((mx + 3 * P.cell_size - P.grid_lo[a]) / P.cell_size);
  }
  for (int a = dim; a < 3; ++a) P.grid_n[a] = 1;
  return P;
}

#define CHECK(x) do { int s_ = (x); if (s_ != 0) { std::printf("FAIL %s -> %d\n", #x, s_); return 1; } } while (0)

static int run(int dim, int m) {
  const double l0 = 0.01;
  Case c = tank(dim, m, l0);
  const int64_t n = (int64_t)c.type.size();
  orc_params P = params(dim, l0, c);
  double n0, lam; int32_t cnt;
  CHECK(orc_lattice_constants(dim, l0, P.re_n, 0, &n0, &lam, &cnt));
  std::vector<int32_t> count(n), list((size_t)n * P.max_neigh), cell(n);
  CHECK(orc_neighbors_brute(&P, n, c.pos.data(), c.type.data(), count.data(), list.data()));
  CHECK(orc_neighbors_cells(&P, n, c.pos.data(), c.type.data(), cell.data(), count.data(), list.data()));
  std::vector<double> us(n * dim), rs(n * dim), ns(n), diag(n), b(n), aval((size_t)n * P.max_neigh),
      p(n), ph(n), gp(n * dim), nut(n), pos(n * dim), vel(n * dim);
  std::vector<int8_t> flags(n), type(n);
  orc_step_out o = {cell.data(), count.data(), list.data(), us.data(), rs.data(), ns.data(),
                    flags.data(), diag.data(), b.data(), aval.data(), p.data(), ph.data(),
                    gp.data(), nut.data(), pos.data(), vel.data(), type.data(), 0, 0.0};
  // every option of the pressure step
  const int opts[][5] = {  // pmode, grad, source, laplacian, kernel
      {0, 0, 0, 0, 0}, {0, 1, 0, 0, 0}, {0, 0, 1, 0, 0}, {0, 0, 2, 0, 0},
      {0, 0, 0, 1, 0}, {0, 1, 2, 1, 0}, {1, 0, 0, 0, 1}, {1, 1, 0, 0, 1}};
  for (auto& op : opts) {
    orc_params Q = P;
    Q.pmode = op[0]; Q.grad = op[1]; Q.source = op[2]; Q.laplacian = op[3]; Q.kernel = op[4];
    CHECK(orc_step(&Q, n, c.pos.data(), c.vel.data(), c.type.data(), nullptr, nullptr, nullptr, &o));
  }
  CHECK(orc_step(&P, n, c.pos.data(), c.vel.data(), c.type.data(), flags.data(), nullptr, nullptr, &o));
  // two-phase with the eddy viscosity
  std::vector<double> rho_i(n), nu_i(n), rho_s(n);
  for (int64_t i = 0; i < n; ++i) {
    bool heavy = c.pos[i * dim + dim - 1] > 0.5 * m * l0;
    rho_i[i] = heavy ? 1500 : 1000;
    nu_i[i] = heavy ? 1e-5 : 1e-6;
  }
  CHECK(orc_smoothed_density(&P, n, c.pos.data(), c.type.data(), rho_i.data(), rho_s.data()));
  orc_params S = P; S.smag_cs = 0.12;
  CHECK(orc_step(&S, n, c.pos.data(), c.vel.data(), c.type.data(), nullptr, rho_s.data(), nu_i.data(), &o));
  CHECK(orc_pressure_gradient(&P, n, rs.data(), c.type.data(), p.data(), ph.data(), gp.data()));
  CHECK(orc_pressure_update(&P, n, rs.data(), us.data(), c.type.data(), p.data(), rho_s.data(),
                            pos.data(), vel.data()));
  // runs: cold and warm-started CG
  for (int warm = 0; warm < 2; ++warm) {
    orc_params R = P; R.cg_warm = warm;
    std::vector<double> x = c.pos, u = c.vel, pr(n, 0.0);
    std::vector<int8_t> t = c.type, fl(n);
    int64_t its = 0;
    CHECK(orc_run(&R, n, x.data(), u.data(), t.data(), 5, nullptr, nullptr, pr.data(), fl.data(), &its));
    if (its <= 0) { std::printf("FAIL no CG iterations\n"); return 1; }
  }
  // dual-number rollout (WC and PPE, single and two-phase) and the loss
  std::vector<double> dir(n * dim);
  for (auto& d : dir) d = urand() - 0.5;
  double out[4];
  orc_params WC = P; WC.pmode = 1; WC.kernel = 1; WC.dt = 1e-4;
  CHECK(orc_rollout_grad(&WC, n, c.pos.data(), c.vel.data(), c.type.data(), 3, dir.data(), 1.0, 9.81,
                         nullptr, nullptr, out));
  CHECK(orc_rollout_grad(&S, n, c.pos.data(), c.vel.data(), c.type.data(), 2, dir.data(), 1.0, 9.81,
                         rho_s.data(), nu_i.data(), out));
  double L = orc_loss(&P, n, c.pos.data(), c.vel.data(), c.type.data(), flags.data(), 1.0, 9.81);
  if (!std::isfinite(L)) { std::printf("FAIL loss\n"); return 1; }
  std::printf("dim %d: %lld particles ok\n", dim, (long long)n);
  return 0;
}

int main() {
  orc_set_threads(2);
  if (run(2, 12)) return 1;
  if (run(3, 6)) return 1;
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
           str(src), os.path.join(ROOT, "oracle", "mps_oracle.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "dim 2:" in r.stdout and "dim 3:" in r.stdout
