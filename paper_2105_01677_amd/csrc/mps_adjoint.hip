// Adjoint (reverse-mode derivative) of one MPS step, hand-written.
//
// Forward step being differentiated (per particle i, lists L frozen):
//   S_i  = sum_j (u_j - u_i) w_lap(|r_j - r_i|)                  (Eq. 7)
//   u*_i = u_i + dt (nu C S_i + g),   r*_i = r_i + dt u*_i        (fluid)
//   n*_i = sum_j w_n(|r*_j - r*_i|)                              (Eq. 5)
//   p_i  = max(0, B ((n*_i/n0)^gamma - 1))          (Eq. 16, weakly compr.)
//       or p = max(0, x), A(r*) x = b(n*)           (Eq. 13, PPE)
//   phat_i = p_{a(i)},  a(i) = argmin over i and its neighbours (frozen)
//   G_i  = d/n0 sum_j (p_j - phat_i) h(r*_ij) (r*_j - r*_i),  h = w_n/r^2
//   u'_i = u*_i - dt/rho G_i,   r'_i = r*_i - dt^2/rho G_i        (fluid)
// Two-phase / turbulence model (the forward of Section "Multiphase flow" and
// "Turbulent flow"): nu C S_i becomes C/<rho>_i sum_j (u_j - u_i) w mu_ij with
// mu_ij = 2 mu_i mu_j/(mu_i + mu_j), mu_i = <rho>_i (nu_i + nu_t,i),
// nu_t,i = (Cs l0)^2 sqrt(2 S:S) from the velocity gradient
// V_i = d/n0 sum_j (u_j - u_i) (r_j - r_i)^T h(r) over re_n at r^k; the
// couplings of A carry 2/(<rho>_i + <rho>_j) and the update 1/<rho>_i (both
// constant).  Its reverse adds mu-bar (gathered with the viscous pairs),
// V-bar = nu_t-bar d nu_t/dV and the gather of V-bar into u-bar and r-bar.
// Every reverse sweep is written as a gather: particle k visits its own list
// and collects both ends of each pair (list symmetry: j in L(i) <=> i in
// L(j)), so there are no floating-point atomics and the result is
// bitwise reproducible.  All adjoint arithmetic is FP64 on FP64 positions.
// The free-surface flags, the neighbour lists, the p-hat argmin and the
// clamp masks are those of the forward step (frozen discrete decisions).
#include "mps_internal.h"

namespace mps {

namespace {

__device__ inline int64_t arow() {
  return (int64_t)xcd_block() * ROWS_PER_BLOCK + threadIdx.x / TEAM;
}

template <int DIM>
__device__ inline double dot3(const double (&a)[DIM], const double (&b)[DIM]) {
  double s = a[0] * b[0] + a[1] * b[1];
  if constexpr (DIM == 3) s += a[2] * b[2];
  return s;
}

// w(r) and dw/dr for the kernels of Eq. 4 and the cubic kernel (0 beyond re).
__device__ inline void wdw(int kernel, double r, double re, double* w, double* dw) {
  if (!(r < re)) {
    *w = 0.0;
    *dw = 0.0;
    return;
  }
  if (kernel == MPS_K_KOSHIZUKA) {
    *w = re / r - 1.0;
    *dw = -re / (r * r);
  } else {
    const double q = 1.0 - r / re;
    *w = q * q * q;
    *dw = -3.0 * q * q / re;
  }
}

// w, dw/dr and d2w/dr2 (0 beyond re).
__device__ inline void wdw2(int kernel, double r, double re, double* w, double* dw,
                            double* d2w) {
  wdw(kernel, r, re, w, dw);
  if (!(r < re)) {
    *d2w = 0.0;
  } else if (kernel == MPS_K_KOSHIZUKA) {
    *d2w = 2.0 * re / (r * r * r);
  } else {
    *d2w = 6.0 * (1.0 - r / re) / (re * re);
  }
}

// Effective (clamped) pressure of the forward step.
__device__ inline double peff(const View& v, int64_t j) {
  const double x = v.p[j];
  return (v.clamp && x < 0.0) ? 0.0 : x;
}

}  // namespace

// p-hat argmin of every fluid particle (and, with the gradient of Eq. 18,
// every wall particle: both ends of a pair carry p-hat there), with the
// same cut-off precision as the forward kernels.  Ties go to the smaller
// sorted index.
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_phat_arg(View v, AdjView a) {
  const int64_t row = arow();
  const int t = team_lane();
  if (row >= v.n) return;
  double m = peff(v, row);
  int32_t am = (int32_t)row;
  const int8_t ty = v.type[row];
  if (ty == MPS_FLUID || (v.grad == MPS_GRAD_CMPS && ty == MPS_WALL)) {
    const int cnt = v.nb_count[row];
    for (int l = t; l < cnt; l += TEAM) {
      const int32_t j = v.nb_list[sl_index(row, l, v.kpad)];
      if (v.type[j] == MPS_DUMMY) continue;
      bool in;
      if constexpr (MIXED) {
        const float4 fi = v.rsf[row], fj = v.rsf[j];
        const int32_t pa = __float_as_int(DIM == 2 ? fi.z : fi.w);
        const int32_t pb = __float_as_int(DIM == 2 ? fj.z : fj.w);
        float d0 = (fj.x - fi.x) + (float)(ucx(pb) - ucx(pa)) * v.cs32;
        float d1 = (fj.y - fi.y) + (float)(ucy(pb) - ucy(pa)) * v.cs32;
        float r2 = d0 * d0 + d1 * d1;
        if constexpr (DIM == 3) {
          float d2 = (fj.z - fi.z) + (float)(ucz(pb) - ucz(pa)) * v.cs32;
          r2 += d2 * d2;
        }
        in = r2 < (float)v.re_n2;
      } else {
        double xi[DIM], xj[DIM];
        load_vec<DIM>(v.rs, row, xi);
        load_vec<DIM>(v.rs, j, xj);
        double r2 = 0.0;
#pragma unroll
        for (int q = 0; q < DIM; ++q) r2 += (xj[q] - xi[q]) * (xj[q] - xi[q]);
        in = r2 < v.re_n2;
      }
      if (!in) continue;
      const double pj = peff(v, j);
      if (pj < m || (pj == m && j < am)) {
        m = pj;
        am = j;
      }
    }
#pragma unroll
    for (int o = 1; o < TEAM; o <<= 1) {
      const double m2 = __shfl_xor(m, o, TEAM);
      const int32_t a2 = __shfl_xor(am, o, TEAM);
      if (m2 < m || (m2 == m && a2 < am)) {
        m = m2;
        am = a2;
      }
    }
  }
  if (t == 0) a.arg[row] = am;
}

// (1) G-bar from the Euler update; the identity parts of u*-bar, r*-bar.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_update(View v, AdjView a) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= v.n) return;
  double ub[DIM], rb[DIM], gb[DIM];
  load_vec<DIM>(a.vel_bar, i, ub);
  load_vec<DIM>(a.pos_bar, i, rb);
  const bool fl = v.type[i] == MPS_FLUID;
  const double rho = v.rho_s ? v.rho_s[i] : v.rho;
#pragma unroll
  for (int q = 0; q < DIM; ++q)
    gb[q] = fl ? -(v.dt / rho) * ub[q] - (v.dt * v.dt / rho) * rb[q] : 0.0;
  store_vec<DIM>(a.gbar, i, gb);
  store_vec<DIM>(a.rs_bar, i, rb);
  store_vec<DIM>(a.ut, i, ub);  // u*-bar so far (r*-bar added later)
}

// h(r) = w(r)/r^2 and dh/dr.
__device__ inline void hdh(int kernel, double r, double re, double* h, double* dh) {
  double w, dw;
  wdw(kernel, r, re, &w, &dw);
  *h = w / (r * r);
  *dh = dw / (r * r) - 2.0 * w / (r * r * r);
}

// (2) Reverse of the pressure gradient.  For particle k:
//   as owner (k fluid):       phat-bar_k, and r*-bar_k -= d-bar_kj
//   as neighbour (k non-dummy) of fluid i: p-bar_k, r*-bar_k += d-bar_ik
// with d-bar_ij = d/n0 num_ij (h G-bar_i + h'/r (d_ij . G-bar_i) d_ij),
// num_ij = p_j - phat_i (standard form) or (p_i + p_j) - (phat_i + phat_j)
// (Eq. 18, which also gives the owner a p-bar and the neighbour a
// phat-bar for every pair).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_gradient(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  const int8_t tk = v.type[k];
  if (tk == MPS_GHOST) {
    if (t == 0) {
      a.phat_bar[k] = 0.0;
      a.pbar[k] = 0.0;
    }
    return;
  }
  const double cgd = (double)DIM / v.n0_n;
  double xk[DIM], gk[DIM];
  load_vec<DIM>(v.rs, k, xk);
  load_vec<DIM>(a.gbar, k, gk);
  const bool cmps = v.grad == MPS_GRAD_CMPS;
  const double pk = peff(v, k);
  const double phk = tk == MPS_FLUID || (cmps && tk == MPS_WALL) ? peff(v, a.arg[k]) : 0.0;
  double phb = 0.0, pb = 0.0, rb[DIM];
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = 0.0;
  const int cnt = v.nb_count[k];
  for (int l = t; l < cnt; l += TEAM) {
    const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
    const int8_t tj = v.type[j];
    double xj[DIM], d[DIM];
    load_vec<DIM>(v.rs, j, xj);
#pragma unroll
    for (int q = 0; q < DIM; ++q) d[q] = xj[q] - xk[q];  // d_kj = r*_j - r*_k
    const double r = sqrt(dot3<DIM>(d, d));
    if (!(r < v.re_n)) continue;
    double h, dh;
    hdh(v.kernel, r, v.re_n, &h, &dh);
    if (tk == MPS_FLUID && tj != MPS_DUMMY) {
      // k is the owner of pair (k, j)
      const double gd = dot3<DIM>(gk, d);
      phb -= cgd * h * gd;
      double num = peff(v, j) - phk;
      if (cmps) {
        pb += cgd * h * gd;
        num += pk - peff(v, a.arg[j]);
      }
      const double c = cgd * num;
#pragma unroll
      for (int q = 0; q < DIM; ++q) rb[q] -= c * (h * gk[q] + dh / r * gd * d[q]);
    }
    if (tj == MPS_FLUID && tk != MPS_DUMMY) {
      // k is the neighbour in pair (j, k): d_jk = -d
      double gj[DIM];
      load_vec<DIM>(a.gbar, j, gj);
      const double gd = -dot3<DIM>(gj, d);
      pb += cgd * h * gd;
      double num = pk - peff(v, a.arg[j]);
      if (cmps) {
        phb -= cgd * h * gd;
        num += peff(v, j) - phk;
      }
      const double c = cgd * num;
#pragma unroll
      for (int q = 0; q < DIM; ++q) rb[q] += c * (h * gj[q] - dh / r * gd * d[q]);
    }
  }
  phb = team_sum(phb);
  pb = team_sum(pb);
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = team_sum(rb[q]);
  if (t == 0) {
    a.phat_bar[k] = tk == MPS_FLUID || (cmps && tk == MPS_WALL) ? phb : 0.0;
    a.pbar[k] = pb;
    double r0[DIM];
    load_vec<DIM>(a.rs_bar, k, r0);
#pragma unroll
    for (int q = 0; q < DIM; ++q) r0[q] += rb[q];
    store_vec<DIM>(a.rs_bar, k, r0);
  }
}

// (3) phat-bar routed to the argmin particle (gather), then through the
// clamp; weakly compressible: through the equation of state into n*-bar;
// PPE: the right-hand side x-bar of the transposed solve (inner rows).
__global__ __launch_bounds__(BLOCK) void k_adj_route(View v, AdjView a, int wc) {
  const int64_t m = arow();
  const int t = team_lane();
  if (m >= v.n) return;
  double s = 0.0;
  const int cnt = v.nb_count[m];
  for (int l = t; l < cnt; l += TEAM) {
    const int32_t i = v.nb_list[sl_index(m, l, v.kpad)];
    // (phat-bar is 0 on particles without a p-hat)
    const int8_t ti = v.type[i];
    if ((ti == MPS_FLUID || ti == MPS_WALL) && a.arg[i] == (int32_t)m) s += a.phat_bar[i];
  }
  s = team_sum(s);
  if (t != 0) return;
  const int8_t tm = v.type[m];
  if ((tm == MPS_FLUID || tm == MPS_WALL) && a.arg[m] == (int32_t)m) s += a.phat_bar[m];
  double pb = a.pbar[m] + s;
  const double x = v.p[m];
  if (v.clamp && !(x > 0.0)) pb = 0.0;
  const int8_t ty = v.type[m];
  if (wc) {
    double nb = 0.0;
    if (ty == MPS_FLUID || ty == MPS_WALL) {
      const double B = (v.rho_s ? v.rho_s[m] : v.rho) * v.c0 * v.c0 / (double)v.gamma_i;
      const double q = v.nstar[m] / v.n0_n;
      double qg1 = 1.0;
      for (int e = 0; e < v.gamma_i - 1; ++e) qg1 *= q;
      nb = pb * B * (double)v.gamma_i * qg1 / v.n0_n;
    }
    a.nbar[m] = nb;
  } else {
    a.pbar[m] = v.flags[m] == MPS_FLAG_INNER ? pb : 0.0;  // x-bar
  }
}

// (3b, PPE) after A lambda = x-bar: b-bar = lambda.  Source of Eq. 13,
// b_i = (n*_i - n0)/(n0 dt^2): n*-bar.  Source of Eq. 21 (HS),
// b_i = (Dn/Dt)*_i / (n0 dt) with Dn_i/Dt = sum_j g(r) (d . du), g = w_n'/r,
// d = r*_j - r*_i, du = u*_j - u*_i over the list within re_n: per pair
// (gathered from both ends, beta = lambda/(n0 dt) on the unknowns)
//   r*-bar_k -= (beta_k + beta_j) (g du + (d . du) g'/r d),
//   u*-bar_k -= (beta_k + beta_j) g d.
// r*-bar from the couplings c_ij = cpp w_lap(r*_ij) (Eq. 7) or chl /
// r*_ij^3 (Eq. 23, HL), times the two-phase factor, whose cotangent over
// both rows of the pair is -(lambda_i - lambda_j)(x_i - x_j) (x and lambda
// vanish on rows that are not unknowns).  The pairs are those of the
// forward step (the cut-offs are frozen decisions).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_ppe(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  const int8_t tk = v.type[k];
  const bool ik = v.flags[k] == MPS_FLAG_INNER;
  const double lk = ik ? a.lam[k] : 0.0;
  const double xk = ik ? v.p[k] : 0.0;
  // the HS term (Dn/Dt)*/(n0 dt) is part of both Dn/Dt sources
  const bool hs = v.source == MPS_SRC_HS || v.source == MPS_SRC_HS_ECS;
  const double cb = 1.0 / (v.n0_n * v.dt);
  const double bk = lk * cb;
  double rb[DIM], ub[DIM];
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = ub[q] = 0.0;
  if (tk != MPS_GHOST) {
    double pk[DIM], uk[DIM];
    load_vec<DIM>(v.rs, k, pk);
    if (hs) load_vec<DIM>(v.us, k, uk);
    const double cpp = 2.0 * DIM / (v.lam_lap * v.n0_lap * v.rho);
    const double chl = 2.0 * v.re_lap / (v.n0_lap * v.rho);
    const bool hl = v.laplacian == MPS_LAP_HL;
    const int cnt = v.nb_count[k];
    for (int l = t; l < cnt; l += TEAM) {
      const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
      const int8_t tj = v.type[j];
      const bool ij = v.flags[j] == MPS_FLAG_INNER;
      const bool cpl = tk != MPS_DUMMY && tj != MPS_DUMMY && (ik || ij);
      const bool src = hs && (ik || ij);
      if (!cpl && !src) continue;
      double pj[DIM], d[DIM];
      load_vec<DIM>(v.rs, j, pj);
#pragma unroll
      for (int q = 0; q < DIM; ++q) d[q] = pj[q] - pk[q];
      const double r = sqrt(dot3<DIM>(d, d));
      const double lj = ij ? a.lam[j] : 0.0;
      if (cpl && r < v.re_lap) {
        double w, dw;
        wdw(v.kernel, r, v.re_lap, &w, &dw);
        const double xj = ij ? v.p[j] : 0.0;
        const double cbar = -(lk - lj) * (xk - xj);
        // dc/dr; two-phase: 1/rho -> 2/(<rho>_k + <rho>_j) (constant per pair)
        const double dcdr = hl ? -3.0 * chl / ((r * r) * (r * r)) : cpp * dw;
        const double fac = v.rho_s ? v.rho * 2.0 / (v.rho_s[k] + v.rho_s[j]) : 1.0;
        const double f = cbar * fac * dcdr / r;
#pragma unroll
        for (int q = 0; q < DIM; ++q) rb[q] -= f * d[q];  // r*_k is the "i" end
      }
      if (src && r < v.re_n) {
        double uj[DIM], du[DIM];
        load_vec<DIM>(v.us, j, uj);
#pragma unroll
        for (int q = 0; q < DIM; ++q) du[q] = uj[q] - uk[q];
        double w, dw, d2w;
        wdw2(v.kernel, r, v.re_n, &w, &dw, &d2w);
        const double g = dw / r, gpr = (d2w - dw / r) / (r * r);  // g'(r)/r
        const double sb = bk + lj * cb, dd = dot3<DIM>(d, du);
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          rb[q] -= sb * (g * du[q] + dd * gpr * d[q]);
          ub[q] -= sb * g * d[q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      rb[q] = team_sum(rb[q]);
      if (hs) ub[q] = team_sum(ub[q]);
    }
  }
  if (t == 0) {
    a.nbar[k] = ik && !hs ? lk / (v.n0_n * v.dt * v.dt) : 0.0;
    double r0[DIM];
    load_vec<DIM>(a.rs_bar, k, r0);
#pragma unroll
    for (int q = 0; q < DIM; ++q) r0[q] += rb[q];
    store_vec<DIM>(a.rs_bar, k, r0);
    if (hs) {
      double u0[DIM];
      load_vec<DIM>(a.ut, k, u0);
#pragma unroll
      for (int q = 0; q < DIM; ++q) u0[q] += ub[q];
      store_vec<DIM>(a.ut, k, u0);
    }
  }
}

// (3c, ECS) The terms of Eq. 24-25 at r^k, u^k (the step input):
//   b_i += (|e_i| g_i + |g_i dt| e_i / dt) / dt,  e = (n - n0)/n0,
//   g = (Dn/Dt)/n0, both summed over the list within re_n at r^k.
// (a) per particle: n and Dn/Dt at r^k again, then n-bar = e-bar/n0 and
// (Dn/Dt)-bar = g-bar/n0 with e-bar = q-bar (s_e g + |g|), g-bar = q-bar
// (|e| + s_g e), q-bar = lambda/dt and s the sign (+1 at 0) -- into the
// phat-bar and p-bar arrays, free once the transposed solve is done;
// (b) the gather of both into the input cotangents, pairs from both ends
// (the Dn/Dt reverse as for HS, at r^k, u^k):
//   r-bar_k -= (nbar_k + nbar_j) w'/r d + (beta_k + beta_j) (g du + (d.du) g'/r d),
//   u-bar_k -= (beta_k + beta_j) g d,     d = r_j - r_k, du = u_j - u_k.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_ecs_a(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  const bool ik = v.flags[k] == MPS_FLAG_INNER;
  const double lk = ik ? a.lam[k] : 0.0;
  double n = 0.0, dn = 0.0;
  if (ik) {
    double xk[DIM], uk[DIM];
    load_vec<DIM>(v.pos, k, xk);
    load_vec<DIM>(v.vel, k, uk);
    const int cnt = v.nb_count[k];
    for (int l = t; l < cnt; l += TEAM) {
      const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
      double xj[DIM], uj[DIM], d[DIM], du[DIM];
      load_vec<DIM>(v.pos, j, xj);
      load_vec<DIM>(v.vel, j, uj);
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        d[q] = xj[q] - xk[q];
        du[q] = uj[q] - uk[q];
      }
      const double r2 = dot3<DIM>(d, d);
      if (!(r2 < v.re_n2)) continue;
      const double r = sqrt(r2);
      double w, dw;
      wdw(v.kernel, r, v.re_n, &w, &dw);
      n += w;
      dn += dw * dot3<DIM>(d, du) / r;
    }
    n = team_sum(n);
    dn = team_sum(dn);
  }
  if (t == 0) {
    const double qb = lk / v.dt;
    const double e = (n - v.n0_n) / v.n0_n, g = dn / v.n0_n;
    const double se = e < 0.0 ? -1.0 : 1.0, sg = g < 0.0 ? -1.0 : 1.0;
    a.phat_bar[k] = ik ? qb * (se * g + fabs(g)) / v.n0_n : 0.0;
    a.pbar[k] = ik ? qb * (fabs(e) + sg * e) / v.n0_n : 0.0;
  }
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_ecs_b(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  if (v.type[k] == MPS_GHOST) return;
  double xk[DIM], uk[DIM], rb[DIM], ub[DIM];
  load_vec<DIM>(v.pos, k, xk);
  load_vec<DIM>(v.vel, k, uk);
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = ub[q] = 0.0;
  const double nk = a.phat_bar[k], bk = a.pbar[k];
  const int cnt = v.nb_count[k];
  for (int l = t; l < cnt; l += TEAM) {
    const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
    const double ns = nk + a.phat_bar[j], bs = bk + a.pbar[j];
    if (ns == 0.0 && bs == 0.0) continue;
    double xj[DIM], uj[DIM], d[DIM], du[DIM];
    load_vec<DIM>(v.pos, j, xj);
    load_vec<DIM>(v.vel, j, uj);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      d[q] = xj[q] - xk[q];
      du[q] = uj[q] - uk[q];
    }
    const double r2 = dot3<DIM>(d, d);
    if (!(r2 < v.re_n2)) continue;
    const double r = sqrt(r2);
    double w, dw, d2w;
    wdw2(v.kernel, r, v.re_n, &w, &dw, &d2w);
    const double g = dw / r, gpr = (d2w - dw / r) / (r * r), dd = dot3<DIM>(d, du);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      rb[q] -= ns * g * d[q] + bs * (g * du[q] + dd * gpr * d[q]);
      ub[q] -= bs * g * d[q];
    }
  }
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    rb[q] = team_sum(rb[q]);
    ub[q] = team_sum(ub[q]);
  }
  if (t == 0) {
    double r0[DIM], u0[DIM];
    load_vec<DIM>(a.pos_bar_in, k, r0);
    load_vec<DIM>(a.vel_bar_in, k, u0);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      r0[q] += rb[q];
      u0[q] += ub[q];
    }
    store_vec<DIM>(a.pos_bar_in, k, r0);
    store_vec<DIM>(a.vel_bar_in, k, u0);
  }
}

// (4) Reverse of the number density:
//   r*-bar_k += sum_m (n*-bar_k + n*-bar_m) w_n'(r)/r (r*_k - r*_m).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_density(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  if (v.type[k] == MPS_GHOST) return;
  double xk[DIM], rb[DIM];
  load_vec<DIM>(v.rs, k, xk);
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = 0.0;
  const double nk = a.nbar[k];
  const int cnt = v.nb_count[k];
  for (int l = t; l < cnt; l += TEAM) {
    const int32_t m = v.nb_list[sl_index(k, l, v.kpad)];
    double xm[DIM], d[DIM];
    load_vec<DIM>(v.rs, m, xm);
#pragma unroll
    for (int q = 0; q < DIM; ++q) d[q] = xk[q] - xm[q];
    const double r = sqrt(dot3<DIM>(d, d));
    if (!(r < v.re_n)) continue;
    double w, dw;
    wdw(v.kernel, r, v.re_n, &w, &dw);
    const double f = (nk + a.nbar[m]) * dw / r;
#pragma unroll
    for (int q = 0; q < DIM; ++q) rb[q] += f * d[q];
  }
#pragma unroll
  for (int q = 0; q < DIM; ++q) rb[q] = team_sum(rb[q]);
  if (t == 0) {
    double r0[DIM];
    load_vec<DIM>(a.rs_bar, k, r0);
#pragma unroll
    for (int q = 0; q < DIM; ++q) r0[q] += rb[q];
    store_vec<DIM>(a.rs_bar, k, r0);
  }
}

// (5a) Prediction, per fluid particle: u-tilde = u*-bar + dt r*-bar,
// a-bar = dt u-tilde, S-bar = nu C a-bar; partials of nu-bar = a-bar . C S
// and g-bar = a-bar (S recomputed at r^k).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_predict_a(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  double nub = 0.0, gb[3] = {0.0, 0.0, 0.0};
  const double clap = 2.0 * DIM / (v.lam_lap * v.n0_lap);
  if (k < v.n) {
    double ut[DIM], rsb[DIM], sb[DIM];
    load_vec<DIM>(a.ut, k, ut);
    load_vec<DIM>(a.rs_bar, k, rsb);
    const bool fl = v.type[k] == MPS_FLUID;
    const bool multi = v.rho_s != nullptr;
    double S[DIM];
#pragma unroll
    for (int q = 0; q < DIM; ++q) S[q] = 0.0;
    if (fl && !multi) {
      double xk[DIM], uk[DIM];
      load_vec<DIM>(v.pos, k, xk);
      load_vec<DIM>(v.vel, k, uk);
      const int cnt = v.nb_count[k];
      for (int l = t; l < cnt; l += TEAM) {
        const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
        double xj[DIM], uj[DIM], d[DIM];
        load_vec<DIM>(v.pos, j, xj);
        load_vec<DIM>(v.vel, j, uj);
#pragma unroll
        for (int q = 0; q < DIM; ++q) d[q] = xj[q] - xk[q];
        double w, dw;
        wdw(v.kernel, sqrt(dot3<DIM>(d, d)), v.re_lap, &w, &dw);
#pragma unroll
        for (int q = 0; q < DIM; ++q) S[q] += (uj[q] - uk[q]) * w;
      }
#pragma unroll
      for (int q = 0; q < DIM; ++q) S[q] = team_sum(S[q]);
    }
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      ut[q] = fl ? ut[q] + v.dt * rsb[q] : ut[q];
      const double ab = fl ? v.dt * ut[q] : 0.0;
      // two-phase: the pair factor mu_kj is applied in (5b), nu-bar there
      sb[q] = (multi ? clap / v.rho_s[k] : v.nu * clap) * ab;
      if (t == 0) {
        nub += ab * clap * S[q];
        gb[q] += ab;
      }
    }
    if (t == 0) {
      store_vec<DIM>(a.ut, k, ut);
      store_vec<DIM>(a.sbar, k, sb);
    }
  }
  // per-workgroup partials, fixed tree: shuffles then LDS
  double x[4] = {nub, gb[0], gb[1], gb[2]};
  __shared__ double sh[4][BLOCK / WAVE];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (int o = WAVE / 2; o > 0; o >>= 1) x[q] += __shfl_down(x[q], o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[q][threadIdx.x / WAVE] = x[q];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < BLOCK / WAVE; ++w) s += sh[threadIdx.x][w];
    a.part[(int64_t)xcd_block() * 4 + threadIdx.x] = s;
  }
}

// (5b) Cotangents of the step input, gathered per particle k:
//   u-bar_k = [fluid](u~_k - S-bar_k sum_j w_kj) + [other] u*-bar_k
//             + sum_{fluid i in L(k)} S-bar_i w_ik
//   r-bar_k = r*-bar_k + [fluid] sum_j -(S-bar_k . (u_j - u_k)) w'/r (r_j - r_k)
//             + sum_{fluid i} (S-bar_i . (u_k - u_i)) w'/r (r_k - r_i)
// Two-phase: every pair term carries mu_kj, and
//   mu-bar_k = sum_j w_kj dmu_kj/dmu_k ([fluid k] S-bar_k . (u_j - u_k)
//                                      + [fluid j] S-bar_j . (u_k - u_j)).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_predict_b(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  const bool fk = v.type[k] == MPS_FLUID;
  double xk[DIM], uk[DIM], sk[DIM], ub[DIM], rb[DIM];
  load_vec<DIM>(v.pos, k, xk);
  load_vec<DIM>(v.vel, k, uk);
  load_vec<DIM>(a.sbar, k, sk);
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    ub[q] = 0.0;
    rb[q] = 0.0;
  }
  double wsum = 0.0, mub = 0.0;
  const bool multi = v.rho_s != nullptr;
  const double mk = multi ? v.mu[k] : 0.0;
  if (v.type[k] != MPS_GHOST) {
    const int cnt = v.nb_count[k];
    for (int l = t; l < cnt; l += TEAM) {
      const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
      double xj[DIM], uj[DIM], d[DIM];
      load_vec<DIM>(v.pos, j, xj);
      load_vec<DIM>(v.vel, j, uj);
#pragma unroll
      for (int q = 0; q < DIM; ++q) d[q] = xj[q] - xk[q];  // r_j - r_k
      const double r = sqrt(dot3<DIM>(d, d));
      double w, dw;
      wdw(v.kernel, r, v.re_lap, &w, &dw);
      double mkj = 1.0, dmk = 0.0;
      if (multi) {
        const double mj = v.mu[j], ms = mk + mj;
        mkj = ms > 0.0 ? 2.0 * mk * mj / ms : 0.0;
        dmk = ms > 0.0 ? 2.0 * mj * mj / (ms * ms) : 0.0;
      }
      double pair = 0.0;  // S-bar . du of both ends, for mu-bar
      if (fk) {
        wsum += w * mkj;
        double du[DIM];
#pragma unroll
        for (int q = 0; q < DIM; ++q) du[q] = uj[q] - uk[q];
        const double sd = dot3<DIM>(sk, du);
        pair += sd;
        const double f = -sd * mkj * dw / r;
#pragma unroll
        for (int q = 0; q < DIM; ++q) rb[q] += f * d[q];
      }
      if (v.type[j] == MPS_FLUID) {
        double sj[DIM], du[DIM];
        load_vec<DIM>(a.sbar, j, sj);
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          ub[q] += sj[q] * w * mkj;
          du[q] = uk[q] - uj[q];
        }
        const double sd = dot3<DIM>(sj, du);
        pair += sd;
        const double f = sd * mkj * dw / r;
#pragma unroll
        for (int q = 0; q < DIM; ++q) rb[q] -= f * d[q];  // (r_k - r_j) = -d
      }
      mub += w * dmk * pair;
    }
    wsum = team_sum(wsum);
    if (multi) mub = team_sum(mub);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      ub[q] = team_sum(ub[q]);
      rb[q] = team_sum(rb[q]);
    }
  }
  if (t == 0) {
    double ut[DIM], rsb[DIM];
    load_vec<DIM>(a.ut, k, ut);
    load_vec<DIM>(a.rs_bar, k, rsb);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      ub[q] += fk ? ut[q] - sk[q] * wsum : ut[q];
      rb[q] += rsb[q];
    }
    store_vec<DIM>(a.vel_bar_in, k, ub);
    store_vec<DIM>(a.pos_bar_in, k, rb);
    if (multi) a.mubar[k] = v.type[k] == MPS_GHOST ? 0.0 : mub;
  }
}

// (6a, two-phase) nu_t-bar_k = <rho>_k mu-bar_k and, for a fluid particle
// with S:S > 0, V-bar_k = nu_t-bar_k d nu_t/dV = nu_t-bar 2 (Cs l0)^2 cg S/sqrt(2 S:S)
// with S = cg (V + V^T)/2, cg = d/n0, V recomputed in FP64 at r^k.  nu-bar
// (a common shift of the laminar viscosities): partials of sum <rho>_k mu-bar_k.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_smag_a(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  double nub = 0.0;
  if (k < v.n) {
    const int8_t tk = v.type[k];
    const double nutb = tk == MPS_GHOST ? 0.0 : v.rho_s[k] * a.mubar[k];
    nub = t == 0 ? nutb : 0.0;
    double G[DIM][DIM];
#pragma unroll
    for (int p = 0; p < DIM; ++p)
#pragma unroll
      for (int q = 0; q < DIM; ++q) G[p][q] = 0.0;
    if (tk == MPS_FLUID && v.smag_c2 > 0.0) {
      double xk[DIM], uk[DIM];
      load_vec<DIM>(v.pos, k, xk);
      load_vec<DIM>(v.vel, k, uk);
      const int cnt = v.nb_count[k];
      for (int l = t; l < cnt; l += TEAM) {
        const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
        double xj[DIM], uj[DIM], d[DIM];
        load_vec<DIM>(v.pos, j, xj);
        load_vec<DIM>(v.vel, j, uj);
#pragma unroll
        for (int q = 0; q < DIM; ++q) d[q] = xj[q] - xk[q];
        const double r = sqrt(dot3<DIM>(d, d));
        if (!(r < v.re_n)) continue;
        double h, dh;
        hdh(v.kernel, r, v.re_n, &h, &dh);
#pragma unroll
        for (int p = 0; p < DIM; ++p)
#pragma unroll
          for (int q = 0; q < DIM; ++q) G[p][q] += (uj[p] - uk[p]) * d[q] * h;
      }
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) G[p][q] = team_sum(G[p][q]);
      const double cg = (double)DIM / v.n0_n;
      double S[DIM][DIM], ss = 0.0;
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          S[p][q] = 0.5 * (G[p][q] + G[q][p]) * cg;
          ss += S[p][q] * S[p][q];
        }
      const double c = ss > 0.0 ? nutb * 2.0 * v.smag_c2 * cg / sqrt(2.0 * ss) : 0.0;
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) G[p][q] = c * S[p][q];
    }
    if (t == 0) {
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) a.gsm[k * 9 + p * DIM + q] = G[p][q];
    }
  }
  // nu-bar partial of this workgroup, added to the one of (5a)
  double x = nub;
  __shared__ double sh[BLOCK / WAVE];
  for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_down(x, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s2 = 0.0;
    for (int w = 0; w < BLOCK / WAVE; ++w) s2 += sh[w];
    a.part[(int64_t)xcd_block() * 4] += s2;
  }
}

// (6b, two-phase) V-bar gathered into u-bar and r-bar.  Pair (i, j), fluid
// i, r < re_n at r^k: V_i += (u_j - u_i) d^T h, d = r_j - r_i; with
// y = V-bar_i^T (u_j - u_i): u-bar_j += V-bar_i d h, u-bar_i -= V-bar_i d h,
// r-bar_j += y h + (d . y) h'/r d, r-bar_i -= the same.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_adj_smag_b(View v, AdjView a) {
  const int64_t k = arow();
  const int t = team_lane();
  if (k >= v.n) return;
  if (v.type[k] == MPS_GHOST || v.smag_c2 <= 0.0) return;
  const bool fk = v.type[k] == MPS_FLUID;
  double xk[DIM], uk[DIM], Gk[DIM][DIM], ub[DIM], rb[DIM];
  load_vec<DIM>(v.pos, k, xk);
  load_vec<DIM>(v.vel, k, uk);
#pragma unroll
  for (int p = 0; p < DIM; ++p) {
    ub[p] = 0.0;
    rb[p] = 0.0;
#pragma unroll
    for (int q = 0; q < DIM; ++q) Gk[p][q] = a.gsm[k * 9 + p * DIM + q];
  }
  const int cnt = v.nb_count[k];
  for (int l = t; l < cnt; l += TEAM) {
    const int32_t j = v.nb_list[sl_index(k, l, v.kpad)];
    double xj[DIM], uj[DIM], d[DIM];
    load_vec<DIM>(v.pos, j, xj);
    load_vec<DIM>(v.vel, j, uj);
#pragma unroll
    for (int q = 0; q < DIM; ++q) d[q] = xj[q] - xk[q];  // r_j - r_k
    const double r = sqrt(dot3<DIM>(d, d));
    if (!(r < v.re_n)) continue;
    double h, dh;
    hdh(v.kernel, r, v.re_n, &h, &dh);
    if (fk) {
      // k is the owner i of pair (k, j)
      double y[DIM], gd[DIM];
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        y[q] = 0.0;
        gd[q] = 0.0;
      }
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          y[q] += Gk[p][q] * (uj[p] - uk[p]);
          gd[p] += Gk[p][q] * d[q];
        }
      const double yd = dot3<DIM>(y, d);
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        ub[q] -= gd[q] * h;
        rb[q] -= y[q] * h + yd * dh / r * d[q];
      }
    }
    if (v.type[j] == MPS_FLUID) {
      // k is the neighbour in pair (j, k): e = r_k - r_j = -d
      double Gj[DIM][DIM], y[DIM], ge[DIM];
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) Gj[p][q] = a.gsm[(int64_t)j * 9 + p * DIM + q];
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        y[q] = 0.0;
        ge[q] = 0.0;
      }
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          y[q] += Gj[p][q] * (uk[p] - uj[p]);
          ge[p] -= Gj[p][q] * d[q];
        }
      const double ye = -dot3<DIM>(y, d);
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        ub[q] += ge[q] * h;
        rb[q] += y[q] * h - ye * dh / r * d[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    ub[q] = team_sum(ub[q]);
    rb[q] = team_sum(rb[q]);
  }
  if (t == 0) {
    double u0[DIM], r0[DIM];
    load_vec<DIM>(a.vel_bar_in, k, u0);
    load_vec<DIM>(a.pos_bar_in, k, r0);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      u0[q] += ub[q];
      r0[q] += rb[q];
    }
    store_vec<DIM>(a.vel_bar_in, k, u0);
    store_vec<DIM>(a.pos_bar_in, k, r0);
  }
}

static inline unsigned tb(int64_t n) { return (unsigned)((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK); }
static inline unsigned fb(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

int adj_partial_blocks(int64_t n) { return (int)tb(n); }

// Stages of the adjoint up to the point where the PPE model needs its
// transposed solve (x-bar is then in a.pbar).
int launch_adjoint_head(const View& v, const AdjView& a, int dim, int precision, int wc,
                        hipStream_t s) {
  const unsigned nt = tb(v.n), nf = fb(v.n);
  const bool mx = precision == MPS_MIXED;
  if (dim == 2) {
    if (mx) k_phat_arg<2, true><<<nt, BLOCK, 0, s>>>(v, a);
    else k_phat_arg<2, false><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_update<2><<<nf, BLOCK, 0, s>>>(v, a);
    k_adj_gradient<2><<<nt, BLOCK, 0, s>>>(v, a);
  } else {
    if (mx) k_phat_arg<3, true><<<nt, BLOCK, 0, s>>>(v, a);
    else k_phat_arg<3, false><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_update<3><<<nf, BLOCK, 0, s>>>(v, a);
    k_adj_gradient<3><<<nt, BLOCK, 0, s>>>(v, a);
  }
  k_adj_route<<<nt, BLOCK, 0, s>>>(v, a, wc);
  return 0;
}

int launch_adjoint_ppe(const View& v, const AdjView& a, int dim, hipStream_t s) {
  const bool ecs = v.source == MPS_SRC_HS_ECS;
  if (dim == 2) {
    k_adj_ppe<2><<<tb(v.n), BLOCK, 0, s>>>(v, a);
    if (ecs) k_adj_ecs_a<2><<<tb(v.n), BLOCK, 0, s>>>(v, a);
  } else {
    k_adj_ppe<3><<<tb(v.n), BLOCK, 0, s>>>(v, a);
    if (ecs) k_adj_ecs_a<3><<<tb(v.n), BLOCK, 0, s>>>(v, a);
  }
  return 0;
}

int launch_adjoint_tail(const View& v, const AdjView& a, int dim, hipStream_t s) {
  const unsigned nt = tb(v.n);
  const bool multi = v.rho_s != nullptr;
  if (dim == 2) {
    k_adj_density<2><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_predict_a<2><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_predict_b<2><<<nt, BLOCK, 0, s>>>(v, a);
    if (multi) {
      k_adj_smag_a<2><<<nt, BLOCK, 0, s>>>(v, a);
      k_adj_smag_b<2><<<nt, BLOCK, 0, s>>>(v, a);
    }
  } else {
    k_adj_density<3><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_predict_a<3><<<nt, BLOCK, 0, s>>>(v, a);
    k_adj_predict_b<3><<<nt, BLOCK, 0, s>>>(v, a);
    if (multi) {
      k_adj_smag_a<3><<<nt, BLOCK, 0, s>>>(v, a);
      k_adj_smag_b<3><<<nt, BLOCK, 0, s>>>(v, a);
    }
  }
  // the ECS terms at r^k, u^k go straight to the input cotangents (the
  // Dn/Dt sources exist only with the pressure equation)
  if (v.source == MPS_SRC_HS_ECS) {
    if (dim == 2) k_adj_ecs_b<2><<<nt, BLOCK, 0, s>>>(v, a);
    else k_adj_ecs_b<3><<<nt, BLOCK, 0, s>>>(v, a);
  }
  return 0;
}

}  // namespace mps
