/*
 * MPS oracle -- TEST INFRASTRUCTURE ONLY (see mps_oracle.h).
 *
 * Plain FP64 C++ written from the equations of arXiv 2105.01677, Section
 * "The Moving Particle Semi-implicit Method":
 *   kernel weight        Eq. 4 (Koshizuka) and the cubic kernel (WC model)
 *   number density       Eq. 5, free surface Eq. 15
 *   Laplacian model      Eq. 7 (also the PPE coefficients)
 *   PPE                  Eq. 13 -> A x = b, assembled row-wise as in the
 *                        listing "PPE assemble GPU code" (dummy neighbours
 *                        give no coupling; alpha/dt^2 on the diagonal);
 *                        sources Eq. 21 (HS) and Eq. 24-25 (ECS); Laplacian
 *                        of pressure Eq. 7 or Eq. 23 (HL)
 *   equation of state    Eq. 16
 *   pressure gradient    standard MPS form, or Eq. 18 (CMPS)
 *   time integration     semi-implicit predictor-corrector, first-order Euler
 * Where the paper is silent or garbled, the reading taken is stated in a
 * comment at the code it concerns.
 *
 * The step is a template on the scalar type so that the same code runs in
 * double and with forward-mode dual numbers (the reference gradient).
 * Discrete decisions (neighbour lists, flags, p-hat argmin, clamps) are taken
 * on the value part, which freezes them exactly as the adjoint does.
 */
#include "mps_oracle.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

enum { FLUID = 0, WALL = 1, DUMMY = 2, GHOST = 3 };
enum { FL_GHOST = -2, FL_DUMMY = -1, FL_INNER = 0, FL_SURFACE = 1 };

/* ---------------------------------------------------------------- duals */
template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0) { for (int k = 0; k < K; ++k) d[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0; }
};
template <int K> Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v + b.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int K> Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v - b.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int K> Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r(-a.v); for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K> Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v * b.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int K> Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v / b.v);
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r; }
template <int K> Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K> Dual<K> operator*(const Dual<K>& a, double b) { return a * Dual<K>(b); }
template <int K> Dual<K> operator*(double a, const Dual<K>& b) { return Dual<K>(a) * b; }
template <int K> Dual<K> operator/(const Dual<K>& a, double b) { return a / Dual<K>(b); }
template <int K> Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }
template <int K> Dual<K> sqrt(const Dual<K>& a) {
  double s = std::sqrt(a.v); Dual<K> r(s);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] / (2.0 * s);
  return r; }

inline double val(double x) { return x; }
template <int K> double val(const Dual<K>& x) { return x.v; }
using std::sqrt;

/* ---------------------------------------------------------- parameters */
struct Consts {
  double n0_n, n0_lap, lam_lap;
};

/* Kernel weights: Eq. 4 (r_e/r - 1) and the cubic kernel (1 - r/r_e)^3,
 * both zero for r >= r_e.  r is a distance, r_e the radius of interaction. */
template <class T>
T weight(int kernel, const T& r, double re) {
  if (!(val(r) < re)) return T(0.0);
  if (kernel == 0) return re / r - 1.0;
  T q = 1.0 - r / re;
  return q * q * q;
}

/* d w / d r of the two kernels (zero for r >= r_e): -r_e / r^2 and
 * -3 (1 - r/r_e)^2 / r_e. */
template <class T>
T dweight(int kernel, const T& r, double re) {
  if (!(val(r) < re)) return T(0.0);
  if (kernel == 0) return -re / (r * r);
  T q = 1.0 - r / re;
  return -3.0 * q * q / re;
}

/* Rate of change of the particle number density of i (Eq. 5) along the
 * motion, Dn_i/Dt = sum_j w'(r_ij) (r_ij . u_ij) / r_ij with r_ij = r_j - r_i,
 * u_ij = u_j - u_i, over the list members within r_e; also n_i itself.  For
 * the kernel of Eq. 4 this is the sum of Eq. 21 (r_e / r^3 times the pair's
 * position and velocity differences, taken with opposite orientations). */
template <class T>
void dn_dt(const orc_params* P, int i, const std::vector<int>& Ls, const std::vector<int>& Lj,
           const std::vector<T>& pos, const std::vector<T>& vel, T* n_out, T* dn_out) {
  const int dim = P->dim;
  T n(0.0), dn(0.0);
  for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
    int j = Lj[e];
    T d[3], du[3], d2(0.0), du_d(0.0);
    for (int a = 0; a < dim; ++a) {
      d[a] = pos[(size_t)j * dim + a] - pos[(size_t)i * dim + a];
      du[a] = vel[(size_t)j * dim + a] - vel[(size_t)i * dim + a];
      d2 = d2 + d[a] * d[a];
      du_d = du_d + d[a] * du[a];
    }
    T r = sqrt(d2);
    if (!(val(r) < P->re_n)) continue;
    n = n + weight(P->kernel, r, P->re_n);
    dn = dn + dweight(P->kernel, r, P->re_n) * du_d / r;
  }
  *n_out = n;
  *dn_out = dn;
}

/* Squared distance between two points, each product and sum rounded in
 * turn: (dx*dx + dy*dy) + dz*dz with dx = x_j - x_i.  The neighbour
 * criterion d^2 < r_e^2 uses this expression on both sides of the parity
 * check, so the lists agree bit for bit. */
inline double dist2(const double* xi, const double* xj, int dim) {
  double dx = xj[0] - xi[0];
  double dy = xj[1] - xi[1];
  double s = dx * dx + dy * dy;
  if (dim == 3) {
    double dz = xj[2] - xi[2];
    s = s + dz * dz;
  }
  return s;
}

Consts constants(const orc_params* P) {
  Consts c;
  int cnt;
  double lam_n;
  orc_lattice_constants(P->dim, P->l0, P->re_n, P->kernel, &c.n0_n, &lam_n, &cnt);
  orc_lattice_constants(P->dim, P->l0, P->re_lap, P->kernel, &c.n0_lap, &c.lam_lap, &cnt);
  return c;
}

/* Whether particle position x lies in the fixed background grid, and its
 * linear cell id (x fastest).  A particle that leaves the grid becomes a
 * ghost and takes no further part. */
bool grid_cell(const orc_params* P, const double* x, int* cell) {
  double inv = 1.0 / P->cell_size;
  int c[3] = {0, 0, 0};
  for (int a = 0; a < P->dim; ++a) {
    double f = std::floor((x[a] - P->grid_lo[a]) * inv);
    if (!(f >= 0.0 && f < (double)P->grid_n[a])) return false;
    c[a] = (int)f;
  }
  *cell = c[0] + P->grid_n[0] * (c[1] + P->grid_n[1] * c[2]);
  return true;
}

/* ------------------------------------------------------ neighbour lists */
struct Lists {
  std::vector<int> start;  // CSR row starts, size n+1
  std::vector<int> idx;    // ascending neighbour ids per row
};

int lists_from_rows(std::vector<std::vector<int>>& rows, int max_neigh, Lists& L) {
  int status = 0;
  size_t n = rows.size();
  L.start.assign(n + 1, 0);
  for (size_t i = 0; i < n; ++i) {
    std::sort(rows[i].begin(), rows[i].end());
    if ((int)rows[i].size() > max_neigh) status = -3;
    L.start[i + 1] = L.start[i] + (int)rows[i].size();
  }
  L.idx.resize(L.start[n]);
  for (size_t i = 0; i < n; ++i)
    std::copy(rows[i].begin(), rows[i].end(), L.idx.begin() + L.start[i]);
  return status;
}

/* The cell-linked list: particles binned into cells of side cell_size >=
 * re_lap; the neighbours of i are searched in its own and the adjacent
 * cells only (Section "Neighbouring search algorithms"). */
int build_lists_cells(const orc_params* P, int n, const double* pos,
                      const int8_t* type, Lists& L, std::vector<int>& cell) {
  const int dim = P->dim;
  const int nx = P->grid_n[0], ny = P->grid_n[1], nz = dim == 3 ? P->grid_n[2] : 1;
  std::vector<std::vector<int>> bins((size_t)nx * ny * nz);
  cell.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    if (type[i] == GHOST) continue;
    int c;
    if (grid_cell(P, pos + (size_t)i * dim, &c)) {
      cell[i] = c;
      bins[c].push_back(i);
    }
  }
  const double re2 = P->re_lap * P->re_lap;
  std::vector<std::vector<int>> rows(n);
  int coincident = 0;
#pragma omp parallel for schedule(guided) reduction(| : coincident)
  for (int i = 0; i < n; ++i) {
    if (cell[i] < 0) continue;
    int ci = cell[i];
    int cx = ci % nx, cy = (ci / nx) % ny, cz = ci / (nx * ny);
    for (int dz = -1; dz <= 1; ++dz) {
      if (dim == 2 && dz != 0) continue;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int x = cx + dx, y = cy + dy, z = cz + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) continue;
          for (int j : bins[x + nx * (y + ny * z)]) {
            if (j == i) continue;
            double d2 = dist2(pos + (size_t)i * dim, pos + (size_t)j * dim, dim);
            if (d2 < re2) {
              rows[i].push_back(j);
              if (d2 == 0.0) coincident = 1;
            }
          }
        }
    }
  }
  int st = lists_from_rows(rows, P->max_neigh, L);
  if (coincident) return -6;
  return st;
}

/* The definition: every pair (i, j), j != i, both in the grid. */
int build_lists_brute(const orc_params* P, int n, const double* pos,
                      const int8_t* type, Lists& L) {
  const int dim = P->dim;
  std::vector<char> active(n, 0);
  for (int i = 0; i < n; ++i) {
    int c;
    active[i] = type[i] != GHOST && grid_cell(P, pos + (size_t)i * dim, &c);
  }
  const double re2 = P->re_lap * P->re_lap;
  std::vector<std::vector<int>> rows(n);
  int coincident = 0;
#pragma omp parallel for schedule(guided) reduction(| : coincident)
  for (int i = 0; i < n; ++i) {
    if (!active[i]) continue;
    for (int j = 0; j < n; ++j) {
      if (j == i || !active[j]) continue;
      double d2 = dist2(pos + (size_t)i * dim, pos + (size_t)j * dim, dim);
      if (d2 < re2) {
        rows[i].push_back(j);
        if (d2 == 0.0) coincident = 1;
      }
    }
  }
  int st = lists_from_rows(rows, P->max_neigh, L);
  if (coincident) return -6;
  return st;
}

void export_lists(const Lists& L, int n, int max_neigh, int32_t* count, int32_t* list) {
  for (int i = 0; i < n; ++i) {
    int c = L.start[i + 1] - L.start[i];
    if (count) count[i] = c;
    if (list) {
      for (int l = 0; l < max_neigh; ++l)
        list[(size_t)i * max_neigh + l] = l < c ? L.idx[L.start[i] + l] : -1;
    }
  }
}

/* ------------------------------------------------------------ PPE solve */
/* Sparse symmetric system: diagonal plus off-diagonal entries per row. */
struct Sparse {
  std::vector<int> start, col;
  std::vector<double> off;   // values
  std::vector<double> diag;
};

void spmv(const Sparse& A, const std::vector<double>& x, std::vector<double>& y) {
  int n = (int)A.diag.size();
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double s = A.diag[i] * x[i];
    for (int k = A.start[i]; k < A.start[i + 1]; ++k) s += A.off[k] * x[A.col[k]];
    y[i] = s;
  }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

/* Conjugate gradients with diagonal (Jacobi) preconditioning, from x = 0
 * (or from x0 when given), to ||b - A x|| <= tol ||b||.  The method's own
 * solver (ICCG) only reaches the same unique solution faster; the oracle
 * needs the solution. */
int cg_solve(const Sparse& A, const std::vector<double>& b, std::vector<double>& x,
             double tol, int maxit, int* iters, double* relres,
             const std::vector<double>* x0 = nullptr) {
  int n = (int)b.size();
  x.assign(n, 0.0);
  double bn = std::sqrt(dot(b, b));
  *iters = 0;
  *relres = 0.0;
  if (bn == 0.0) return 0;
  std::vector<double> r = b, z(n), p(n), q(n);
  if (x0) {
    x = *x0;
    spmv(A, x, q);
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double rn = std::sqrt(dot(r, r));
    *relres = rn / bn;
    if (rn <= tol * bn) return 0;
  }
  for (int i = 0; i < n; ++i) z[i] = r[i] / A.diag[i];
  p = z;
  double rz = dot(r, z);
  for (int it = 1; it <= maxit; ++it) {
    spmv(A, p, q);
    double alpha = rz / dot(p, q);
    for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    double rn = std::sqrt(dot(r, r));
    *iters = it;
    *relres = rn / bn;
    if (rn <= tol * bn) return 0;
    for (int i = 0; i < n; ++i) z[i] = r[i] / A.diag[i];
    double rz2 = dot(r, z);
    double beta = rz2 / rz;
    rz = rz2;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  return -4;
}

/* Solve A(T) p = b(T).  For double this is one CG solve; for duals the
 * value system is solved first, then each tangent system
 * A p' = b' - A' p with the same matrix (forward-mode differentiation of
 * the exact solution). */
template <class T>
struct PPESolve;

template <>
struct PPESolve<double> {
  static int run(const std::vector<int>& start, const std::vector<int>& col,
                 const std::vector<double>& off, const std::vector<double>& diag,
                 const std::vector<double>& b, std::vector<double>& p, double tol,
                 int maxit, int* iters, double* relres,
                 const std::vector<double>* x0 = nullptr) {
    Sparse A{start, col, off, diag};
    return cg_solve(A, b, p, tol, maxit, iters, relres, x0);
  }
};

template <int K>
struct PPESolve<Dual<K>> {
  using T = Dual<K>;
  static int run(const std::vector<int>& start, const std::vector<int>& col,
                 const std::vector<T>& off, const std::vector<T>& diag,
                 const std::vector<T>& b, std::vector<T>& p, double tol, int maxit,
                 int* iters, double* relres, const std::vector<double>* = nullptr) {
    int n = (int)diag.size();
    Sparse A;
    A.start = start;
    A.col = col;
    A.off.resize(off.size());
    A.diag.resize(n);
    for (size_t k = 0; k < off.size(); ++k) A.off[k] = off[k].v;
    for (int i = 0; i < n; ++i) A.diag[i] = diag[i].v;
    std::vector<double> bv(n), pv;
    for (int i = 0; i < n; ++i) bv[i] = b[i].v;
    int st = cg_solve(A, bv, pv, tol, maxit, iters, relres);
    p.assign(n, T(0.0));
    for (int i = 0; i < n; ++i) p[i].v = pv[i];
    for (int k = 0; k < K; ++k) {
      std::vector<double> rhs(n), pk;
      for (int i = 0; i < n; ++i) {
        double s = diag[i].d[k] * pv[i];
        for (int e = start[i]; e < start[i + 1]; ++e) s += off[e].d[k] * pv[col[e]];
        rhs[i] = b[i].d[k] - s;
      }
      int it2; double rr2;
      cg_solve(A, rhs, pk, tol, maxit, &it2, &rr2);
      for (int i = 0; i < n; ++i) p[i].d[k] = pk[i];
    }
    return st;
  }
};

/* ------------------------------------------------------------ the step */
template <class T>
struct Trace {
  std::vector<T> us, rs, nstar, p, phat, gradp, diag, b, nut;
  std::vector<T> aval;   // aligned with the list CSR
  std::vector<int8_t> flags;
  std::vector<int> cell;
  Lists lists;
  int cg_iters = 0;
  double cg_relres = 0.0;
};

/* Integer power by repeated multiplication (gamma = 7 in Eq. 16). */
template <class T>
T ipow(const T& x, int e) {
  T r(1.0);
  for (int k = 0; k < e; ++k) r = r * x;
  return r;
}

template <class T>
void pressure_gradient(const orc_params* P, const Consts& C, int n,
                       const std::vector<T>& rs, const std::vector<int8_t>& type,
                       const std::vector<T>& p, const Lists& L,
                       std::vector<T>& phat, std::vector<T>& gradp) {
  const int dim = P->dim;
  const std::vector<int>& Ls = L.start;
  const std::vector<int>& Lj = L.idx;
  auto dist = [&](int i, int j) {
    T d2(0.0);
    for (int a = 0; a < dim; ++a) {
      T d = rs[(size_t)j * dim + a] - rs[(size_t)i * dim + a];
      d2 = d2 + d * d;
    }
    return sqrt(d2);
  };
  /* 6. p-hat: the minimum pressure over i and its non-dummy neighbours
   *    within re_n at r*.  Needed for every particle in CMPS, fluid only in
   *    the standard gradient. */
  phat.assign(n, T(0.0));
  for (int i = 0; i < n; ++i) {
    if (type[i] != FLUID && type[i] != WALL) continue;
    T m = p[i];
    for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
      int j = Lj[e];
      if (type[j] == DUMMY) continue;
      if (!(val(dist(i, j)) < P->re_n)) continue;
      if (val(p[j]) < val(m)) m = p[j];
    }
    phat[i] = m;
  }

  /* 7. Pressure gradient, fluid only, over non-dummy j within re_n:
   *    standard: grad p_i = d/n0 sum_j (p_j - phat_i)/r^2 (r_j - r_i) w
   *    CMPS (Eq. 18): numerator (p_i + p_j) - (phat_i + phat_j). */
  gradp.assign((size_t)n * dim, T(0.0));
  const double cg = (double)dim / C.n0_n;
#pragma omp parallel for schedule(guided)
  for (int i = 0; i < n; ++i) {
    if (type[i] != FLUID) continue;
    T gp[3] = {T(0.0), T(0.0), T(0.0)};
    for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
      int j = Lj[e];
      if (type[j] == DUMMY) continue;
      T d[3];
      T d2(0.0);
      for (int a = 0; a < dim; ++a) {
        d[a] = rs[(size_t)j * dim + a] - rs[(size_t)i * dim + a];
        d2 = d2 + d[a] * d[a];
      }
      T r = sqrt(d2);
      if (!(val(r) < P->re_n)) continue;
      T w = weight(P->kernel, r, P->re_n);
      T num = P->grad == 0 ? p[j] - phat[i]
                           : (p[i] + p[j]) - (phat[i] + phat[j]);
      T f = num / d2 * w;
      for (int a = 0; a < dim; ++a) gp[a] = gp[a] + f * d[a];
    }
    for (int a = 0; a < dim; ++a) gradp[(size_t)i * dim + a] = cg * gp[a];
  }
}

/* First-order Euler update of the fluid particles (Section "Standard
 * method"): u^{k+1} = u* - dt/rho_i grad p_i, r^{k+1} = r* + dt (u^{k+1} - u*),
 * with rho_i the smoothed density of the two-phase model when given, else
 * the single density rho.  Other particles keep their position and velocity. */
template <class T>
void euler_update(const orc_params* P, int n, const std::vector<int8_t>& type,
                  const std::vector<T>& us, const std::vector<T>& rs,
                  const std::vector<T>& gradp, const double* rho_s, std::vector<T>& pos,
                  std::vector<T>& vel) {
  const int dim = P->dim;
  const double dt = P->dt;
  for (int i = 0; i < n; ++i) {
    if (type[i] != FLUID) continue;
    const double rho_i = rho_s ? rho_s[i] : P->rho;
    for (int a = 0; a < dim; ++a) {
      size_t k = (size_t)i * dim + a;
      T u = us[k] - dt / rho_i * gradp[k];
      pos[k] = rs[k] + dt * (u - us[k]);
      vel[k] = u;
    }
  }
}

template <class T>
int step(const orc_params* P, const Consts& C, const T& nu, const T g[3], int n,
         std::vector<T>& pos, std::vector<T>& vel, std::vector<int8_t>& type,
         const int8_t* flags_override, Trace<T>& tr, const double* rho_s = nullptr,
         const double* nu_i = nullptr) {
  const int dim = P->dim;
  const double dt = P->dt;
  const double rho = P->rho;
  int status = 0;
  /* Two-phase / turbulence extension (Section "Fluid flow models"): per
   * particle smoothed density <rho>_i (fixed before the run) and laminar
   * viscosity nu_i, Smagorinsky eddy viscosity when smag_cs > 0. */
  const bool multi = rho_s || nu_i || P->smag_cs > 0.0;
  auto rho_of = [&](int i) { return rho_s ? rho_s[i] : rho; };

  /* 1. Ghosts: particles outside the grid leave the simulation. */
  std::vector<double> x0((size_t)n * dim);
  for (size_t k = 0; k < x0.size(); ++k) x0[k] = val(pos[k]);
  for (int i = 0; i < n; ++i) {
    int c;
    if (type[i] != GHOST && !grid_cell(P, &x0[(size_t)i * dim], &c)) type[i] = GHOST;
  }

  /* 2. Neighbour lists at r^k, kept for the whole step. */
  int st = build_lists_cells(P, n, x0.data(), type.data(), tr.lists, tr.cell);
  if (st) return st;
  const std::vector<int>& Ls = tr.lists.start;
  const std::vector<int>& Lj = tr.lists.idx;

  /* 3. Explicit viscous + body force prediction (Eq. 2 without pressure,
   *    Laplacian by Eq. 7 with r_e = re_lap), fluid only:
   *    u* = u + dt (nu lap(u) + g),  r* = r + dt u*. */
  const double clap = 2.0 * dim / (C.lam_lap * C.n0_lap);
  tr.us.assign((size_t)n * dim, T(0.0));
  tr.rs.assign((size_t)n * dim, T(0.0));
  /* 3a. Smagorinsky eddy viscosity nu_t = (Cs l0)^2 sqrt(2 S:S) of fluid
   *     particles, S the symmetric part of the MPS velocity gradient
   *     grad u_i = d/n0 sum_j (u_j - u_i) (r_j - r_i)^T w(r)/r^2 (re_n, r^k);
   *     mu_i = <rho>_i (nu_i + nu_t,i). */
  std::vector<T> mu;
  tr.nut.assign(n, T(0.0));
  if (multi) {
    mu.assign(n, T(0.0));
    const double cs2 = (P->smag_cs * P->l0) * (P->smag_cs * P->l0);
#pragma omp parallel for schedule(guided)
    for (int i = 0; i < n; ++i) {
      if (type[i] == GHOST) continue;
      T nut(0.0);
      if (P->smag_cs > 0.0 && type[i] == FLUID) {
        T G[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) G[a][b] = T(0.0);
        const T* ri = &pos[(size_t)i * dim];
        const T* ui = &vel[(size_t)i * dim];
        for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
          int j = Lj[e];
          const T* rj = &pos[(size_t)j * dim];
          const T* uj = &vel[(size_t)j * dim];
          T d[3], d2(0.0);
          for (int a = 0; a < dim; ++a) { d[a] = rj[a] - ri[a]; d2 = d2 + d[a] * d[a]; }
          T r = sqrt(d2);
          if (!(val(r) < P->re_n)) continue;
          T f = weight(P->kernel, r, P->re_n) / d2;
          for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) G[a][b] = G[a][b] + (uj[a] - ui[a]) * d[b] * f;
        }
        T ss(0.0);
        for (int a = 0; a < dim; ++a)
          for (int b = 0; b < dim; ++b) {
            T sab = 0.5 * (G[a][b] + G[b][a]) * ((double)dim / C.n0_n);
            ss = ss + sab * sab;
          }
        if (val(ss) > 0.0) nut = cs2 * sqrt(2.0 * ss);
      }
      tr.nut[i] = nut;
      // with per-particle viscosities, the derivative part of nu (value
      // unused) shifts every laminar viscosity alike
      T nui = nu_i ? T(nu_i[i]) + (nu - T(val(nu))) : nu;
      mu[i] = rho_of(i) * (nui + nut);
    }
  }
#pragma omp parallel for schedule(guided)
  for (int i = 0; i < n; ++i) {
    const T* ri = &pos[(size_t)i * dim];
    const T* ui = &vel[(size_t)i * dim];
    for (int a = 0; a < dim; ++a) {
      tr.us[(size_t)i * dim + a] = ui[a];
      tr.rs[(size_t)i * dim + a] = ri[a];
    }
    if (type[i] != FLUID) continue;
    T lap[3] = {T(0.0), T(0.0), T(0.0)};
    for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
      int j = Lj[e];
      const T* rj = &pos[(size_t)j * dim];
      const T* uj = &vel[(size_t)j * dim];
      T d2(0.0);
      for (int a = 0; a < dim; ++a) { T d = rj[a] - ri[a]; d2 = d2 + d * d; }
      T w = weight(P->kernel, sqrt(d2), P->re_lap);
      if (multi) {
        /* harmonic mean of the dynamic viscosities of the pair */
        T ms = mu[i] + mu[j];
        T muij = val(ms) > 0.0 ? 2.0 * mu[i] * mu[j] / ms : T(0.0);
        w = w * muij;
      }
      for (int a = 0; a < dim; ++a) lap[a] = lap[a] + (uj[a] - ui[a]) * w;
    }
    for (int a = 0; a < dim; ++a) {
      T acc = multi ? clap * lap[a] / rho_of(i) + g[a] : nu * clap * lap[a] + g[a];
      T u = ui[a] + dt * acc;
      tr.us[(size_t)i * dim + a] = u;
      tr.rs[(size_t)i * dim + a] = ri[a] + dt * u;
    }
  }

  /* 4. Particle number density at r* (Eq. 5, r_e = re_n) and the
   *    free-surface flag n* < beta n0 (Eq. 15) for fluid and wall. */
  auto dist = [&](int i, int j) {
    T d2(0.0);
    for (int a = 0; a < dim; ++a) {
      T d = tr.rs[(size_t)j * dim + a] - tr.rs[(size_t)i * dim + a];
      d2 = d2 + d * d;
    }
    return sqrt(d2);
  };
  tr.nstar.assign(n, T(0.0));
  tr.flags.assign(n, (int8_t)FL_INNER);
#pragma omp parallel for schedule(guided)
  for (int i = 0; i < n; ++i) {
    if (type[i] == GHOST) { tr.flags[i] = FL_GHOST; continue; }
    T s(0.0);
    for (int e = Ls[i]; e < Ls[i + 1]; ++e) s = s + weight(P->kernel, dist(i, Lj[e]), P->re_n);
    tr.nstar[i] = s;
    if (type[i] == DUMMY) tr.flags[i] = FL_DUMMY;
    else tr.flags[i] = val(s) < P->beta * C.n0_n ? FL_SURFACE : FL_INNER;
  }
  if (flags_override) {
    for (int i = 0; i < n; ++i)
      if (type[i] == FLUID || type[i] == WALL) tr.flags[i] = flags_override[i];
  }

  /* 5. Pressure. */
  std::vector<double> p_prev;
  if (P->cg_warm && tr.p.size() == (size_t)n)
    for (int i = 0; i < n; ++i) p_prev.push_back(tr.flags[i] == FL_INNER ? val(tr.p[i]) : 0.0);
  tr.p.assign(n, T(0.0));
  tr.diag.assign(n, T(1.0));
  tr.b.assign(n, T(0.0));
  tr.aval.assign(Lj.size(), T(0.0));
  if (P->pmode == 0) {
    /* PPE (Eq. 13) with the Laplacian of Eq. 7, row-wise for inner i:
     *   c_ij = 2d w(r*_ij) / (lambda n0 rho)  for non-dummy j with r* < re_lap
     *   A_ii = sum_j c_ij + alpha/dt^2,  A_ij = -c_ij for inner j
     *   b_i  = (n*_i - n0) / (n0 dt^2)
     * A free-surface neighbour (p = 0, Dirichlet) keeps its c_ij on the
     * diagonal only.  Rows that are not inner are the identity (p = 0). */
    const double cpp = 2.0 * dim / (C.lam_lap * C.n0_lap * rho);
    /* Eq. 23 (HL), printed as (1/n0) sum_j 2 phi_ij r_e / r_ij with a power
     * of r_ij lost: read as (1/n0) sum_j 2 r_e phi_ij / r_ij^3, the one power
     * that gives a Laplacian its units (1/length^2); with the printed factor
     * 2 the sum then reproduces lap |r|^2 = 2d in the continuum limit in two
     * and three dimensions alike (n0 of Eq. 4 at r_e).  Coupling
     * c_ij = 2 r_e / (n0 rho r_ij^3) for r_ij < re_lap. */
    const double chl = 2.0 * P->re_lap / (C.n0_lap * rho);
    std::vector<int> start(n + 1, 0), col;
    std::vector<T> off;
    for (int i = 0; i < n; ++i) {
      if (tr.flags[i] == FL_INNER) {
        T dsum(0.0);
        for (int e = Ls[i]; e < Ls[i + 1]; ++e) {
          int j = Lj[e];
          if (type[j] == DUMMY) continue;
          T r = dist(i, j);
          if (!(val(r) < P->re_lap)) continue;
          T c = P->laplacian == 0 ? cpp * weight(P->kernel, r, P->re_lap)
                                  : chl / (r * r * r);
          if (multi) c = c * (rho * 2.0 / (rho_of(i) + rho_of(j)));
          dsum = dsum + c;
          if (tr.flags[j] == FL_INNER) {
            col.push_back(j);
            off.push_back(-c);
            tr.aval[e] = -c;
          }
        }
        tr.diag[i] = dsum + P->alpha / (dt * dt);
        if (P->source == 0) {
          tr.b[i] = (tr.nstar[i] - C.n0_n) / (C.n0_n * dt * dt);
        } else {
          /* Eq. 21 (HS): the source from Dn/Dt at r*, u*,
           *   b_i = (Dn/Dt)*_i / (n0 dt);
           * Eq. 24-25 (ECS) adds, with n and Dn/Dt at r^k, u^k,
           *   |(n - n0)/n0| (Dn/Dt)/n0 + |dt (Dn/Dt)/n0| (n - n0)/(n0 dt)
           * inside the bracket: b_i = ((Dn/Dt)*_i / n0 + ECS_i) / dt. */
          T nst, dns;
          dn_dt<T>(P, i, Ls, Lj, tr.rs, tr.us, &nst, &dns);
          T q = dns / C.n0_n;
          if (P->source == 2) {
            T nk, dnk;
            dn_dt<T>(P, i, Ls, Lj, pos, vel, &nk, &dnk);
            T e = (nk - C.n0_n) / C.n0_n;
            T g = dnk / C.n0_n;
            T ae = val(e) < 0.0 ? -e : e;
            T ag = val(g) < 0.0 ? -g * dt : g * dt;
            q = q + ae * g + ag * e / dt;
          }
          tr.b[i] = q / dt;
        }
      }
      start[i + 1] = (int)col.size();
    }
    int sst = PPESolve<T>::run(start, col, off, tr.diag, tr.b, tr.p,
                               P->cg_warm ? P->cg_tol : 1e-13,
                               std::max(P->cg_maxit, 100000), &tr.cg_iters,
                               &tr.cg_relres, p_prev.empty() ? nullptr : &p_prev);
    if (sst) status = sst;
    for (int i = 0; i < n; ++i)
      if (tr.flags[i] != FL_INNER) tr.p[i] = T(0.0);
  } else {
    /* Equation of state (Eq. 16): p = rho c0^2/gamma ((n* / n0)^gamma - 1)
     * for fluid and wall particles. */
    const int ge = (int)P->gamma;
    for (int i = 0; i < n; ++i)
      if (type[i] == FLUID || type[i] == WALL) {
        const double B = rho_of(i) * P->c0 * P->c0 / P->gamma;
        tr.p[i] = B * (ipow(tr.nstar[i] / C.n0_n, ge) - 1.0);
      }
  }
  if (P->clamp)
    for (int i = 0; i < n; ++i)
      if (val(tr.p[i]) < 0.0) tr.p[i] = T(0.0);

  /* 6-7. p-hat and the pressure gradient at r*. */
  pressure_gradient<T>(P, C, n, tr.rs, type, tr.p, tr.lists, tr.phat, tr.gradp);

  /* 8. First-order Euler update. */
  euler_update<T>(P, n, type, tr.us, tr.rs, tr.gradp, rho_s, pos, vel);
  return status;
}

/* Loss of a final state: w_ke * mean over active fluid of |u|^2/2 plus
 * w_var * the variance of the vertical coordinate over the fluid particles
 * flagged free surface in the last step (that set is frozen). */
template <class T>
T final_loss(int n, int dim, const std::vector<T>& pos, const std::vector<T>& vel,
             const std::vector<int8_t>& type, const std::vector<int8_t>& flags, double w_ke,
             double w_var) {
  T ke(0.0);
  int nf = 0;
  for (int i = 0; i < n; ++i) {
    if (type[i] != FLUID) continue;
    T s(0.0);
    for (int a = 0; a < dim; ++a) s = s + vel[(size_t)i * dim + a] * vel[(size_t)i * dim + a];
    ke = ke + 0.5 * s;
    ++nf;
  }
  ke = ke / (double)(nf > 0 ? nf : 1);
  T mean(0.0);
  int ns = 0;
  for (int i = 0; i < n; ++i)
    if (type[i] == FLUID && flags[i] == FL_SURFACE) {
      mean = mean + pos[(size_t)i * dim + dim - 1];
      ++ns;
    }
  T var(0.0);
  if (ns > 0) {
    mean = mean / (double)ns;
    for (int i = 0; i < n; ++i)
      if (type[i] == FLUID && flags[i] == FL_SURFACE) {
        T d = pos[(size_t)i * dim + dim - 1] - mean;
        var = var + d * d;
      }
    var = var / (double)ns;
  }
  return w_ke * ke + w_var * var;
}

void to_params(const orc_params* P, double* nu, double g[3]) {
  *nu = P->nu;
  for (int a = 0; a < 3; ++a) g[a] = P->g[a];
}

}  // namespace

/* ---------------------------------------------------------------- C API */
extern "C" {

int orc_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
}

double orc_weight(int kernel, double r, double re) { return weight(kernel, r, re); }

int orc_lattice_constants(int dim, double l0, double re, int kernel, double* n0,
                          double* lambda, int32_t* count) {
  /* n0 = sum_{j != i} w(|r_j - r_i|) over the lattice (Eq. 5 at rest);
   * lambda = sum r^2 w / sum w (the weighted mean of r^2 in Eq. 7). */
  int m = (int)std::ceil(re / l0) + 1;
  double sw = 0.0, sr2w = 0.0;
  int cnt = 0;
  double o[3] = {0.0, 0.0, 0.0};
  for (int a = -m; a <= m; ++a)
    for (int b = -m; b <= m; ++b)
      for (int c = (dim == 3 ? -m : 0); c <= (dim == 3 ? m : 0); ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        double x[3] = {a * l0, b * l0, c * l0};
        double d2 = dist2(o, x, dim);
        if (!(d2 < re * re)) continue;
        double w = weight(kernel, std::sqrt(d2), re);
        sw += w;
        sr2w += d2 * w;
        ++cnt;
      }
  *n0 = sw;
  *lambda = sr2w / sw;
  if (count) *count = cnt;
  return 0;
}

int orc_neighbors_brute(const orc_params* P, int64_t n, const double* pos,
                        const int8_t* type, int32_t* count, int32_t* list) {
  Lists L;
  int st = build_lists_brute(P, (int)n, pos, type, L);
  export_lists(L, (int)n, P->max_neigh, count, list);
  return st;
}

int orc_neighbors_cells(const orc_params* P, int64_t n, const double* pos,
                        const int8_t* type, int32_t* cell, int32_t* count,
                        int32_t* list) {
  Lists L;
  std::vector<int> c;
  std::vector<int8_t> t(type, type + n);
  for (int64_t i = 0; i < n; ++i) {
    int cc;
    if (t[i] != GHOST && !grid_cell(P, pos + i * P->dim, &cc)) t[i] = GHOST;
  }
  int st = build_lists_cells(P, (int)n, pos, t.data(), L, c);
  export_lists(L, (int)n, P->max_neigh, count, list);
  if (cell) for (int64_t i = 0; i < n; ++i) cell[i] = c[i];
  return st;
}

int orc_step(const orc_params* P, int64_t n, const double* pos, const double* vel,
             const int8_t* type, const int8_t* flags_override, const double* rho_s,
             const double* nu_i, orc_step_out* out) {
  Consts C = constants(P);
  const int dim = P->dim;
  std::vector<double> x(pos, pos + n * dim), u(vel, vel + n * dim);
  std::vector<int8_t> t(type, type + n);
  double nu, g[3];
  to_params(P, &nu, g);
  Trace<double> tr;
  int st = step<double>(P, C, nu, g, (int)n, x, u, t, flags_override, tr, rho_s, nu_i);
  if (st == -3 || st == -6) return st;
  auto cp = [&](double* dst, const std::vector<double>& src) {
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(double));
  };
  if (out->cell) for (int64_t i = 0; i < n; ++i) out->cell[i] = tr.cell[i];
  export_lists(tr.lists, (int)n, P->max_neigh, out->count, out->list);
  cp(out->us, tr.us); cp(out->rs, tr.rs); cp(out->nstar, tr.nstar);
  if (out->flags) std::memcpy(out->flags, tr.flags.data(), n);
  cp(out->diag, tr.diag); cp(out->b, tr.b);
  if (out->aval) {
    for (int64_t i = 0; i < n; ++i) {
      int s = tr.lists.start[i], c = tr.lists.start[i + 1] - s;
      for (int l = 0; l < P->max_neigh; ++l)
        out->aval[i * P->max_neigh + l] = l < c ? tr.aval[s + l] : 0.0;
    }
  }
  cp(out->p, tr.p); cp(out->phat, tr.phat); cp(out->gradp, tr.gradp);
  cp(out->nut, tr.nut);
  cp(out->pos, x); cp(out->vel, u);
  if (out->type) std::memcpy(out->type, t.data(), n);
  out->cg_iters = tr.cg_iters;
  out->cg_relres = tr.cg_relres;
  return st;
}

int orc_rollout_grad(const orc_params* P, int64_t n, const double* pos, const double* vel,
                     const int8_t* type, int32_t nsteps, const double* dir, double w_ke,
                     double w_var, const double* rho_s, const double* nu_i, double* out) {
  /* Forward-mode derivative of the loss after nsteps steps along three
   * directions: d/dnu, d/dg_x and <d/du0, dir> (dual numbers through the
   * whole rollout, the PPE solves differentiated exactly). */
  using D = Dual<3>;
  Consts C = constants(P);
  const int dim = P->dim;
  std::vector<D> x(n * dim), u(n * dim);
  for (int64_t k = 0; k < n * dim; ++k) {
    x[k] = D(pos[k]);
    u[k] = D(vel[k]);
    if (dir && type[k / dim] == FLUID) u[k].d[2] = dir[k];
  }
  std::vector<int8_t> t(type, type + n);
  D nu(P->nu);
  nu.d[0] = 1.0;
  D g[3] = {D(P->g[0]), D(P->g[1]), D(P->g[2])};
  g[0].d[1] = 1.0;
  Trace<D> tr;
  int st = 0;
  for (int s = 0; s < nsteps; ++s) {
    st = step<D>(P, C, nu, g, (int)n, x, u, t, nullptr, tr, rho_s, nu_i);
    if (st == -3 || st == -6) return st;
  }
  D L = final_loss<D>((int)n, dim, x, u, t, tr.flags, w_ke, w_var);
  out[0] = L.v;
  out[1] = L.d[0];
  out[2] = L.d[1];
  out[3] = L.d[2];
  return st;
}

int orc_smoothed_density(const orc_params* P, int64_t n, const double* pos,
                         const int8_t* type, const double* rho_i, double* rho_s) {
  /* <rho>_i = sum_j rho_j w(r_ij) / sum_j w(r_ij) over non-dummy neighbours
   * within re_n, for fluid particles; wall and dummy keep their own rho. */
  Lists L;
  std::vector<int> cell;
  std::vector<int8_t> t(type, type + n);
  int st = build_lists_cells(P, (int)n, pos, t.data(), L, cell);
  if (st) return st;
  const int dim = P->dim;
  for (int64_t i = 0; i < n; ++i) {
    rho_s[i] = rho_i[i];
    if (t[i] != FLUID) continue;
    double sw = 0.0, srw = 0.0;
    for (int e = L.start[i]; e < L.start[i + 1]; ++e) {
      int j = L.idx[e];
      if (t[j] == DUMMY) continue;
      double d2 = dist2(pos + i * dim, pos + (int64_t)j * dim, dim);
      double w = weight(P->kernel, std::sqrt(d2), P->re_n);
      sw += w;
      srw += rho_i[j] * w;
    }
    if (sw > 0.0) rho_s[i] = srw / sw;
  }
  return 0;
}

double orc_loss(const orc_params* P, int64_t n, const double* pos, const double* vel,
                const int8_t* type, const int8_t* flags, double w_ke, double w_var) {
  std::vector<double> x(pos, pos + n * P->dim), u(vel, vel + n * P->dim);
  std::vector<int8_t> t(type, type + n), f(flags, flags + n);
  return final_loss<double>((int)n, P->dim, x, u, t, f, w_ke, w_var);
}

int orc_pressure_gradient(const orc_params* P, int64_t n, const double* rs,
                          const int8_t* type, const double* p, double* phat,
                          double* gradp) {
  /* Lists are taken at the given positions (here r*), as the step does. */
  Consts C = constants(P);
  Lists L;
  std::vector<int> cell;
  std::vector<int8_t> t(type, type + n);
  int st = build_lists_cells(P, (int)n, rs, t.data(), L, cell);
  if (st) return st;
  std::vector<double> r(rs, rs + n * P->dim), pp(p, p + n), ph, gp;
  pressure_gradient<double>(P, C, (int)n, r, t, pp, L, ph, gp);
  std::memcpy(phat, ph.data(), n * sizeof(double));
  std::memcpy(gradp, gp.data(), n * P->dim * sizeof(double));
  return 0;
}

int orc_pressure_update(const orc_params* P, int64_t n, const double* rs, const double* us,
                        const int8_t* type, const double* p, const double* rho_s,
                        double* pos_out, double* vel_out) {
  /* p-hat, the pressure gradient of a given pressure field at rs (lists
   * taken at rs) and the Euler update of the step from (rs, us). */
  Consts C = constants(P);
  const int dim = P->dim;
  Lists L;
  std::vector<int> cell;
  std::vector<int8_t> t(type, type + n);
  int st = build_lists_cells(P, (int)n, rs, t.data(), L, cell);
  if (st) return st;
  std::vector<double> r(rs, rs + n * dim), u(us, us + n * dim), pp(p, p + n), ph, gp;
  pressure_gradient<double>(P, C, (int)n, r, t, pp, L, ph, gp);
  std::vector<double> x = r, v = u;
  euler_update<double>(P, (int)n, t, u, r, gp, rho_s, x, v);
  std::memcpy(pos_out, x.data(), x.size() * sizeof(double));
  std::memcpy(vel_out, v.data(), v.size() * sizeof(double));
  return 0;
}

int orc_run(const orc_params* P, int64_t n, double* pos, double* vel, int8_t* type,
            int32_t nsteps, const double* rho_s, const double* nu_i, double* p_out,
            int8_t* flags_out, int64_t* cg_iters_out) {
  Consts C = constants(P);
  const int dim = P->dim;
  std::vector<double> x(pos, pos + n * dim), u(vel, vel + n * dim);
  std::vector<int8_t> t(type, type + n);
  double nu, g[3];
  to_params(P, &nu, g);
  int st = 0;
  Trace<double> tr;
  /* warm start: p_out brings the pressure of the step before the first */
  if (P->cg_warm && p_out) tr.p.assign(p_out, p_out + n);
  int64_t iters = 0;
  for (int s = 0; s < nsteps; ++s) {
    st = step<double>(P, C, nu, g, (int)n, x, u, t, nullptr, tr, rho_s, nu_i);
    iters += tr.cg_iters;
    if (st == -3 || st == -6) break;
  }
  if (cg_iters_out) *cg_iters_out = iters;
  std::memcpy(pos, x.data(), x.size() * sizeof(double));
  std::memcpy(vel, u.data(), u.size() * sizeof(double));
  std::memcpy(type, t.data(), n);
  if (p_out && !tr.p.empty()) std::memcpy(p_out, tr.p.data(), n * sizeof(double));
  if (flags_out && !tr.flags.empty()) std::memcpy(flags_out, tr.flags.data(), n);
  return st;
}

}  // extern "C"
