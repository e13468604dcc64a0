// Kernel-weighted neighbour sums of one MPS step (arXiv 2105.01677,
// Section "The Moving Particle Semi-implicit Method"):
//   k_predict   viscous Laplacian (Eq. 7, radius re_lap) + body force, the
//               explicit prediction u* = u + dt a, r* = r + dt u* (fluid)
//   k_density   number density n* at r* (Eq. 5, radius re_n), free-surface
//               flag n* < beta n0 (Eq. 15); in the weakly-compressible model
//               also the equation of state (Eq. 16); writes the short lists
//               (the entries within re_n at r*)
//   k_gradient  p-hat, pressure gradient (standard MPS form or Eq. 18) and
//               the first-order Euler update, over the short lists
// Each particle is handled by a team of TEAM lanes that split its neighbour
// list (see mps_internal.h).  The precision template: FP64 throughout, or
// MIXED = FP32 distances and sums on positions stored relative to the lower
// corner of the particle's cell (so the FP32 values are at most one cell
// side and keep ~1e-7 relative accuracy in the separations), with FP64
// master state.
#include "mps_internal.h"

namespace mps {

// Position of a particle as seen by the sums: FP64 absolute, or FP32
// relative to its anchor cell with the packed cell coordinates.
template <int DIM, bool MIXED>
struct PosRef;

template <int DIM>
struct PosRef<DIM, false> {
  using R = double;
  double x[DIM];
  __device__ static PosRef load(const double* a, const float4*, int64_t i) {
    PosRef p;
    load_vec<DIM>(a, i, p.x);
    return p;
  }
  __device__ void diff(const PosRef& o, float, R (&d)[DIM]) const {
#pragma unroll
    for (int a = 0; a < DIM; ++a) d[a] = o.x[a] - x[a];
  }
};

template <int DIM>
struct PosRef<DIM, true> {
  using R = float;
  float4 f;
  __device__ static PosRef load(const double*, const float4* a, int64_t i) {
    PosRef p;
    p.f = a[i];
    return p;
  }
  __device__ int32_t pc() const { return __float_as_int(DIM == 2 ? f.z : f.w); }
  __device__ void diff(const PosRef& o, float cs, R (&d)[DIM]) const {
    const int32_t a = pc(), b = o.pc();
    d[0] = (o.f.x - f.x) + (float)(ucx(b) - ucx(a)) * cs;
    d[1] = (o.f.y - f.y) + (float)(ucy(b) - ucy(a)) * cs;
    if constexpr (DIM == 3) d[2] = (o.f.z - f.z) + (float)(ucz(b) - ucz(a)) * cs;
  }
};

// A particle at r^k as the viscous sums see it: position and velocity.
// Plain path: FP64 state.  Mixed path: the 32-byte FP32 record written by
// the cell sort (cell-relative position with the packed cell, then the FP32
// velocity), one contiguous gather per neighbour.
template <int DIM, bool MIXED>
struct KRec;

template <int DIM>
struct KRec<DIM, false> {
  PosRef<DIM, false> p;
  double u[DIM];
  __device__ static KRec load(const View& v, int64_t j) {
    KRec r;
    r.p = PosRef<DIM, false>::load(v.pos, nullptr, j);
    load_vec<DIM>(v.vel, j, r.u);
    return r;
  }
};

template <int DIM>
struct KRec<DIM, true> {
  PosRef<DIM, true> p;
  float u[DIM];
  __device__ static KRec load(const View& v, int64_t j) {
    KRec r;
    r.p.f = v.posf[2 * j];
    const float4 q = v.posf[2 * j + 1];
    r.u[0] = q.x;
    r.u[1] = q.y;
    if constexpr (DIM == 3) r.u[2] = q.z;
    return r;
  }
};

template <int DIM, class R>
__device__ inline R norm2(const R (&d)[DIM]) {
  R s = d[0] * d[0] + d[1] * d[1];
  if constexpr (DIM == 3) s += d[2] * d[2];
  return s;
}

// FP32 copy of an FP64 position relative to the lower corner of the
// particle's anchor cell (the cell it was binned in this step).
template <int DIM>
__device__ inline float4 to_rel(const View& v, const double (&x)[DIM], int32_t pc) {
  const int ci[3] = {ucx(pc), ucy(pc), ucz(pc)};
  float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < DIM; ++a) r[a] = (float)(x[a] - (v.lo[a] + ci[a] * v.cs));
  return DIM == 2 ? make_float4(r[0], r[1], __int_as_float(pc), 0.f)
                  : make_float4(r[0], r[1], r[2], __int_as_float(pc));
}

// Pressure as the gradient stage uses it: clamped at 0 when negative
// pressure is clamped (the solve's output is clamped on read here, and
// written back clamped by k_gradient; a reader that sees either value
// gets the same clamped number).
__device__ inline double p_eff(const View& v, double x) { return (v.clamp && x < 0.0) ? 0.0 : x; }

__device__ inline int64_t team_row() {
  return (int64_t)xcd_block() * ROWS_PER_BLOCK + threadIdx.x / TEAM;
}

// The list entries l = t, t + TEAM, ... < cnt of a row, U per lane and
// step, in two phases per step so that all gathers of a step are in flight
// together: load(j) issues the gathers of neighbour j (straight-line code),
// body(j, rec, ok) consumes them.  The list entries of the next step are
// loaded while this step's gathers are in flight (software pipelining:
// one exposed memory latency per step).  Slots past cnt (stale, but inside
// the row's kpad slots) are replaced by the row itself with ok = false; the
// body must then contribute nothing.  Slot indices past kpad are clamped to
// the row's first slot, so every load stays inside the row.
#ifndef SUM_U_PREDICT
#define SUM_U_PREDICT 2
#endif
#ifndef SUM_U_DENSITY
#define SUM_U_DENSITY 2
#endif
#ifndef SUM_U_VISC
#define SUM_U_VISC 2
#endif
#ifndef SUM_U_PHAT
#define SUM_U_PHAT 2
#endif
#ifndef SUM_U_GRAD
#define SUM_U_GRAD 2
#endif
template <int U, class LD, class F>
__device__ inline void for_list(const View& v, int64_t row, int cnt, int t, LD&& load,
                                F&& body) {
  const int64_t e0 = sl_index(row, t, v.kpad);
  const int ng = v.kpad / TEAM;  // slot groups of a row
  int32_t jn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) jn[u] = v.nb_list[e0 + (int64_t)(u < ng ? u : 0) * WAVE];
  for (int k0 = 0; t + k0 * TEAM < cnt; k0 += U) {
    int32_t j[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = t + (k0 + u) * TEAM < cnt;
      j[u] = ok[u] ? jn[u] : (int32_t)row;
    }
    decltype(load(j[0])) rec[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rec[u] = load(j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + U + u;
      jn[u] = v.nb_list[e0 + (int64_t)(k < ng ? k : 0) * WAVE];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) body(j[u], rec[u], ok[u]);
  }
}

// a3: u* = u + dt (nu 2d/(lambda n0) sum_j (u_j - u_i) w(r_ij) + g),
//     r* = r + dt u*  for fluid; other particles keep r and u.
template <int DIM, bool MIXED, bool MULTI>
__global__ __launch_bounds__(BLOCK) void k_predict(View v) {
  using P = PosRef<DIM, MIXED>;
  using R = typename P::R;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  // the row's own loads are issued together (no branch before the list)
  double ui[DIM], xi[DIM];
  load_vec<DIM>(v.vel, row, ui);
  load_vec<DIM>(v.pos, row, xi);
  const bool fluid = v.type[row] == MPS_FLUID;
  const int cnt_all = v.nb_count[row];
  using K = KRec<DIM, MIXED>;
  const K ri = K::load(v, row);
  const double mi = MULTI ? v.mu[row] : 0.0;
  const int cnt = fluid ? cnt_all : 0;
  double us[DIM], rs[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) { us[a] = ui[a]; rs[a] = xi[a]; }
  {
    const R re = (R)v.re_lap, re2 = (R)v.re_lap2;
    R acc[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc[a] = R(0);
    struct Rec {
      K k;
      double mj;
    };
    for_list<SUM_U_PREDICT>(
        v, row, cnt, t,
        [&](int32_t j) {
          Rec r;
          r.k = K::load(v, j);
          r.mj = MULTI ? v.mu[j] : 0.0;
          return r;
        },
        [&](int32_t, const Rec& rj, bool ok) {
          R d[DIM];
          ri.p.diff(rj.k.p, v.cs32, d);
          const R r2 = norm2<DIM, R>(d);
          const R wr = weight_r2<R>(v.kernel, r2, rsqrt_k(r2), re, re2);
          R w = ok ? wr : R(0);
          if constexpr (MULTI) {
            // two-phase: harmonic mean of the pair's dynamic viscosities
            const double ms = mi + rj.mj;
            w *= (R)(ms > 0.0 ? 2.0 * mi * rj.mj * rcp_k(ms) : 0.0);
          }
#pragma unroll
          for (int a = 0; a < DIM; ++a) acc[a] += (R)(rj.k.u[a] - ri.u[a]) * w;
        });
    if (fluid) {
      const double clap = 2.0 * DIM / (v.lam_lap * v.n0_lap);
      const double visc = MULTI ? clap / v.rho_s[row] : v.nu * clap;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double lap = (double)team_sum(acc[a]);
        us[a] = ui[a] + v.dt * (visc * lap + v.g[a]);
        rs[a] = xi[a] + v.dt * us[a];
      }
    }
  }
  if (t == 0) {
    store_vec<DIM>(v.us, row, us);
    store_vec<DIM>(v.rs, row, rs);
    if constexpr (MIXED) v.rsf[row] = to_rel<DIM>(v, rs, v.pcell[row]);
  }
}

// a2 + a3 with lists kept over steps (single phase): the prediction walks
// the superset list (radius re_lap + skin at the last build) and writes the
// exact list of this step -- the entries within re_lap at r, decided on
// dist2_exact of the FP64 positions in list order, with the same
// compaction, cap and flags as k_list_filter -- while it sums the viscous
// term over those entries.  On the mixed path the decision is taken on the
// FP32 cell-relative records the sum gathers anyway, except inside a band
// of +-KEEP_BAND re_lap^2 around the cut-off and for separations below
// KEEP_BAND re_lap^2 (coincidence), where the FP64 positions decide: the
// FP32 squared separation is within ~3e-6 re_lap^2 of the FP64 one (cell-
// relative coordinates of at most a cell side plus the skin, rounded once,
// subtracted, offset by whole FP32 cell sides), so outside the band both
// give the same answer.
#ifndef KEEP_BAND
#define KEEP_BAND 4e-5
#endif
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_predict_keep(View v) {
  using P = PosRef<DIM, MIXED>;
  using R = typename P::R;
  using K = KRec<DIM, MIXED>;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  double ui[DIM], xi[DIM];
  load_vec<DIM>(v.vel, row, ui);
  load_vec<DIM>(v.pos, row, xi);
  const bool fluid = v.type[row] == MPS_FLUID;
  const int cs = v.sk_count[row];
  const K ri = K::load(v, row);
  // the superset is walked; the exact list is written
  View vs = v;
  vs.nb_list = v.sk_list;
  vs.kpad = v.kpad_s;
  const int64_t e0 = sl_index(row, 0, v.kpad);
  const float lo = (float)(v.re_lap2 * (1.0 - KEEP_BAND)), hi = (float)(v.re_lap2 * (1.0 + KEEP_BAND)),
              tiny = (float)(v.re_lap2 * KEEP_BAND);
  int count = 0;
  bool coinc = false;
  double us[DIM], rs[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) { us[a] = ui[a]; rs[a] = xi[a]; }
  {
    const R re = (R)v.re_lap, re2 = (R)v.re_lap2;
    R acc[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc[a] = R(0);
    for_list<SUM_U_PREDICT>(
        vs, row, cs, t, [&](int32_t j) { return K::load(v, j); },
        [&](int32_t j, const K& rj, bool ok) {
          R d[DIM];
          ri.p.diff(rj.p, v.cs32, d);
          const R r2 = norm2<DIM, R>(d);
          bool hit;
          double d2 = 1.0;   // the FP64 separation, where it was computed
          if constexpr (MIXED) {
            if (r2 < tiny || (r2 >= lo && r2 < hi)) {
              double xj[DIM];
              load_vec<DIM>(v.pos, j, xj);
              d2 = dist2_exact<DIM>(xi, xj);
              hit = ok && d2 < v.re_lap2;
            } else {
              hit = ok && r2 < lo;
            }
          } else {
            d2 = dist2_exact<DIM>(xi, rj.p.x);
            hit = ok && d2 < v.re_lap2;
          }
          coinc = coinc || (hit && d2 == 0.0);
          const uint32_t m = team_ballot(hit);
          if (hit) {
            const unsigned q = (unsigned)(count + __popc(m & ((1u << t) - 1u)));
            if (q < (unsigned)v.max_neigh)
              v.nb_list[e0 + (int64_t)(q / TEAM) * WAVE + (q % TEAM)] = j;
          }
          count += __popc(m);
          const R wr = weight_r2<R>(v.kernel, r2, rsqrt_k(r2), re, re2);
          const R w = (fluid && hit) ? wr : R(0);
#pragma unroll
          for (int a = 0; a < DIM; ++a) acc[a] += (R)(rj.u[a] - ri.u[a]) * w;
        });
    if (fluid) {
      const double clap = 2.0 * DIM / (v.lam_lap * v.n0_lap);
      const double visc = v.nu * clap;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double lap = (double)team_sum(acc[a]);
        us[a] = ui[a] + v.dt * (visc * lap + v.g[a]);
        rs[a] = xi[a] + v.dt * us[a];
      }
    }
  }
  if (coinc) atomicOr(v.status, ST_COINCIDENT);
  if (count > v.max_neigh) {
    if (t == 0) atomicOr(v.status, ST_OVERFLOW);
    count = v.max_neigh;
  }
  if (t == 0) {
    v.nb_count[row] = count;
    store_vec<DIM>(v.us, row, us);
    store_vec<DIM>(v.rs, row, rs);
    if constexpr (MIXED) v.rsf[row] = to_rel<DIM>(v, rs, v.pcell[row]);
  }
}

// Integer power by multiplication (Eq. 16 uses gamma = 7).
__device__ inline double ipow(double x, int e) {
  double r = 1.0;
  for (int k = 0; k < e; ++k) r *= x;
  return r;
}

// a4 (+a7): n*_i = sum_j w(|r*_j - r*_i|) over the list within re_n; flags;
// equation of state p = rho c0^2/gamma ((n*/n0)^gamma - 1) for fluid and
// wall in the weakly-compressible model.
// Always FP64, also on the mixed path: the pressure source (n* - n0)/n0 of
// Eq. 13 and the EOS (Eq. 16) amplify the rounding of n*, and from rest
// n* - n0 is of the order of the FP32 rounding of n* itself.  In 2-D the
// FP64 position (double2) is as wide as the FP32 copy (float4), so this
// costs no extra bytes.
template <int DIM, int SRC>
__global__ __launch_bounds__(BLOCK) void k_density(View v, int wc) {
  using P = PosRef<DIM, false>;
  using R = typename P::R;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  // the row's own loads are issued together (no branch before the list)
  const int8_t ty = v.type[row];
  const int cnt_all = v.nb_count[row];
  const int32_t err = *v.status;
  const P pi = P::load(v.rs, v.rsf, row);
  double ui[DIM], xk[DIM], uk[DIM];
  if constexpr (SRC >= MPS_SRC_HS) load_vec<DIM>(v.us, row, ui);
  if constexpr (SRC == MPS_SRC_HS_ECS) {
    load_vec<DIM>(v.pos, row, xk);
    load_vec<DIM>(v.vel, row, uk);
  }
  const int cnt = ty != MPS_GHOST ? cnt_all : 0;
  // n* at r*; with a Dn/Dt source also Dn/Dt at r*, u* (Eq. 21) and, for
  // ECS, n and Dn/Dt at r^k, u^k (Eq. 24):
  //   Dn_i/Dt = sum_j w'(r_ij) ((r_j - r_i) . (u_j - u_i)) / r_ij
  R s = R(0);
  double dns = 0.0, nk = 0.0, dnk = 0.0;
  // the short list: entries within re_n at r* (widened by re_n2_keep),
  // appended in list order by a team ballot; nq is the same in every lane
  int nq = 0;
  const int64_t q0 = sl_index(row, 0, v.kpad);
  {
    const R re = (R)v.re_n, re2 = (R)v.re_n2;
    struct Rec {
      P p;
      double u[DIM], x[DIM], w[DIM];
    };
    for_list<SUM_U_DENSITY>(
        v, row, cnt, t,
        [&](int32_t j) {
          Rec r;
          r.p = P::load(v.rs, v.rsf, j);
          if constexpr (SRC >= MPS_SRC_HS) load_vec<DIM>(v.us, j, r.u);
          if constexpr (SRC == MPS_SRC_HS_ECS) {
            load_vec<DIM>(v.pos, j, r.x);
            load_vec<DIM>(v.vel, j, r.w);
          }
          return r;
        },
        [&](int32_t j, const Rec& rj, bool ok) {
          R d[DIM];
          pi.diff(rj.p, v.cs32, d);
          const R r2 = norm2<DIM, R>(d);
          const R ir = rsqrt_k(r2);
          const bool in = ok && r2 < re2;
          const bool keep = ok && r2 < v.re_n2_keep;
          const uint32_t km = team_ballot(keep);
          if (keep) {
            const unsigned q = (unsigned)(nq + __popc(km & ((1u << t) - 1u)));
            v.nbn_list[q0 + (int64_t)(q / TEAM) * WAVE + (q % TEAM)] = j;
          }
          nq += __popc(km);
          const R w = weight_r2<R>(v.kernel, r2, ir, re, re2);
          s += in ? w : R(0);
          if constexpr (SRC >= MPS_SRC_HS) {
            double dud = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) dud += d[a] * (rj.u[a] - ui[a]);
            const double f = dweight_r2<double>(v.kernel, r2, ir, re, re2) * dud * ir;
            dns += in ? f : 0.0;
          }
          if constexpr (SRC == MPS_SRC_HS_ECS) {
            double dk[DIM], dud = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
              dk[a] = rj.x[a] - xk[a];
              dud += dk[a] * (rj.w[a] - uk[a]);
            }
            const double rk2 = norm2<DIM, double>(dk);
            const double irk = rsqrt_k(rk2);
            const bool ink = ok && rk2 < v.re_n2;
            const double wk = weight_r2<double>(v.kernel, rk2, irk, v.re_n, v.re_n2);
            const double fk = dweight_r2<double>(v.kernel, rk2, irk, v.re_n, v.re_n2) * dud * irk;
            nk += ink ? wk : 0.0;
            dnk += ink ? fk : 0.0;
          }
        });
    s = team_sum(s);
    if constexpr (SRC >= MPS_SRC_HS) dns = team_sum(dns);
    if constexpr (SRC == MPS_SRC_HS_ECS) {
      nk = team_sum(nk);
      dnk = team_sum(dnk);
    }
  }
  if constexpr (SRC >= MPS_SRC_HS) {
    if (t == 0) {
      // b_i = ((Dn/Dt)*_i / n0 + ECS_i) / dt, ECS_i = |e| g + |g dt| e / dt
      // with e = (n_i - n0)/n0 and g = (Dn/Dt)_i / n0 at r^k, u^k
      double q = dns / v.n0_n;
      if constexpr (SRC == MPS_SRC_HS_ECS) {
        const double e = (nk - v.n0_n) / v.n0_n, g = dnk / v.n0_n;
        q += fabs(e) * g + fabs(g * v.dt) * e / v.dt;
      }
      v.src[row] = q / v.dt;
    }
  }
  if (t != 0) return;
  v.nbn_count[row] = nq;
  const double ns = (double)s;
  int8_t fl;
  if (ty == MPS_GHOST) fl = MPS_FLAG_GHOST;
  else if (ty == MPS_DUMMY) fl = MPS_FLAG_DUMMY;
  else fl = ns < v.beta * v.n0_n ? MPS_FLAG_SURFACE : MPS_FLAG_INNER;
  // no state is written after an error raised earlier in the call
  if (err) return;
  v.nstar[row] = ns;
  v.flags[row] = fl;
  if (wc) {
    double p = 0.0;
    if (ty == MPS_FLUID || ty == MPS_WALL) {
      const double B = (v.rho_s ? v.rho_s[row] : v.rho) * v.c0 * v.c0 / (double)v.gamma_i;
      p = B * (ipow(ns / v.n0_n, v.gamma_i) - 1.0);
      if (v.clamp && p < 0.0) p = 0.0;
    }
    v.p[row] = p;
  }
}

// Two-phase / turbulence: Smagorinsky eddy viscosity of fluid particles,
// nu_t = (Cs l0)^2 sqrt(2 S:S), S the symmetric part of the MPS velocity
// gradient d/n0 sum_j (u_j - u_i) (r_j - r_i)^T w(r)/r^2 (re_n, at r^k), and
// the dynamic viscosity mu_i = <rho>_i (nu_i + nu_t,i) of every particle.
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_viscosity(View v) {
  using P = PosRef<DIM, MIXED>;
  using R = typename P::R;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  const int8_t ty = v.type[row];
  double nut = 0.0;
  if (ty == MPS_FLUID && v.smag_c2 > 0.0) {
    using K = KRec<DIM, MIXED>;
    const K ri = K::load(v, row);
    R G[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = 0; b < DIM; ++b) G[a][b] = R(0);
    const R re = (R)v.re_n, re2 = (R)v.re_n2;
    const int cnt = v.nb_count[row];
    for_list<SUM_U_VISC>(v, row, cnt, t, [&](int32_t j) { return K::load(v, j); },
                         [&](int32_t, const K& rj, bool ok) {
      R d[DIM];
      ri.p.diff(rj.p, v.cs32, d);
      const R r2 = norm2<DIM, R>(d);
      const R ir = rsqrt_k(r2);
      const R fr = weight_r2<R>(v.kernel, r2, ir, re, re2) * ir * ir;
      const R f = (ok && r2 < re2) ? fr : R(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) G[a][b] += (R)(rj.u[a] - ri.u[a]) * d[b] * f;
    });
    double ss = 0.0;
    const double cg = (double)DIM / v.n0_n;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = 0; b < DIM; ++b) G[a][b] = team_sum(G[a][b]);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        const double sab = 0.5 * ((double)G[a][b] + (double)G[b][a]) * cg;
        ss += sab * sab;
      }
    nut = ss > 0.0 ? v.smag_c2 * sqrt(2.0 * ss) : 0.0;
  }
  if (t == 0) {
    v.nut[row] = nut;
    v.mu[row] = ty == MPS_GHOST ? 0.0 : v.rho_s[row] * (v.nu_l[row] + nut);
  }
}

// Smoothed density of the two-phase model, once before the run:
// <rho>_i = sum_j rho_j w / sum_j w over non-dummy neighbours within re_n
// (fluid); wall and dummy keep their own density.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_smooth_density(View v, const double* rho,
                                                          double* out) {
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  double sw = 0.0, srw = 0.0;
  if (v.type[row] == MPS_FLUID) {
    double xi[DIM];
    load_vec<DIM>(v.pos, row, xi);
    const int cnt = v.nb_count[row];
    for (int l = t; l < cnt; l += TEAM) {
      const int32_t j = v.nb_list[sl_index(row, l, v.kpad)];
      if (v.type[j] == MPS_DUMMY) continue;
      double xj[DIM];
      load_vec<DIM>(v.pos, j, xj);
      double r2 = 0.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a) r2 += (xj[a] - xi[a]) * (xj[a] - xi[a]);
      const double w = weight<double>(v.kernel, sqrt(r2), v.re_n);
      sw += w;
      srw += rho[j] * w;
    }
    sw = team_sum(sw);
    srw = team_sum(srw);
  }
  if (t == 0) out[row] = sw > 0.0 ? srw / sw : rho[row];
}

// p-hat of every fluid and wall particle (needed by Eq. 18 for both ends of
// a pair): minimum of p over i and its non-dummy neighbours within re_n.
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_phat(View v, double* phat) {
  using P = PosRef<DIM, MIXED>;
  using R = typename P::R;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  // the row's own loads are issued together (no branch before the list)
  const int8_t ty = v.type[row];
  double m = p_eff(v, v.p[row]);
  const int cnt_all = v.nb_count[row];
  const P pi = P::load(v.rs, v.rsf, row);
  const int cnt = ty == MPS_FLUID || ty == MPS_WALL ? cnt_all : 0;
  {
    const R re2 = (R)v.re_n2;
    struct Rec {
      P p;
      double pj;
      int8_t fj;
    };
    for_list<SUM_U_PHAT>(
        v, row, cnt, t,
        [&](int32_t j) {
          Rec r;
          r.p = P::load(v.rs, v.rsf, j);
          r.pj = p_eff(v, v.p[j]);
          r.fj = v.flags[j];
          return r;
        },
        [&](int32_t, const Rec& rj, bool ok) {
          R d[DIM];
          pi.diff(rj.p, v.cs32, d);
          // flags mark exactly the dummy particles MPS_FLAG_DUMMY
          if (ok && rj.fj != MPS_FLAG_DUMMY && norm2<DIM, R>(d) < re2) m = fmin(m, rj.pj);
        });
    m = team_min(m);
  }
  if (t == 0) phat[row] = m;
}

// a8: grad p_i = d/n0 sum_j num_ij / r^2 (r*_j - r*_i) w(r) over non-dummy j
// within re_n, num = p_j - phat_i (standard) or (p_i + p_j) - (phat_i +
// phat_j) (Eq. 18); u = u* - dt/rho grad p, r = r* + dt (u - u*).
// Standard form in one pass over the list: with f_ij = (r*_j - r*_i)
// w(r)/r^2, sum_j (p_j - phat_i) f_ij = A - phat_i B where A = sum_j p_j f_ij
// and B = sum_j f_ij are accumulated in FP64 together with the minimum that
// gives phat_i, so the cancellation in A - phat_i B costs no accuracy.
template <int DIM, bool MIXED, bool CMPS>
__global__ __launch_bounds__(BLOCK) void k_gradient(View v, const double* phat) {
  using P = PosRef<DIM, MIXED>;
  using R = typename P::R;
  const int64_t row = team_row();
  const int t = team_lane();
  if (row >= v.n) return;
  // the row's own loads are issued together (no branch before the list)
  const bool fluid = v.type[row] == MPS_FLUID;
  const P pi = P::load(v.rs, v.rsf, row);
  const R re = (R)v.re_n, re2 = (R)v.re_n2;
  const int cnt_all = v.nb_count[row];
  const double p_raw = v.p[row];
  const int32_t err = *v.status;
  const double p_i = p_eff(v, p_raw);
  double us[DIM], rs[DIM], un[DIM], xn[DIM];
  load_vec<DIM>(v.us, row, us);
  load_vec<DIM>(v.rs, row, rs);
  const double rho_i = v.rho_s ? v.rho_s[row] : v.rho;
  const int cnt = fluid ? cnt_all : 0;
  double gs[DIM], bs[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) gs[a] = bs[a] = 0.0;
  double m = p_i;
  const double ph_i = CMPS ? phat[row] : 0.0;
  struct Rec {
    P p;
    double pj, phj;
    int8_t fj;
  };
  for_list<SUM_U_GRAD>(
      v, row, cnt, t,
      [&](int32_t j) {
        Rec r;
        r.p = P::load(v.rs, v.rsf, j);
        r.pj = p_eff(v, v.p[j]);
        r.phj = CMPS ? phat[j] : 0.0;
        r.fj = v.flags[j];
        return r;
      },
      [&](int32_t, const Rec& rj, bool ok) {
    R d[DIM];
    pi.diff(rj.p, v.cs32, d);
    const R r2 = norm2<DIM, R>(d);
    const double pj = rj.pj;
    // flags mark exactly the dummy particles MPS_FLAG_DUMMY
    const bool in = ok && rj.fj != MPS_FLAG_DUMMY && r2 < re2;
    const R ir = rsqrt_k(r2);
    const R wr = weight_r2<R>(v.kernel, r2, ir, re, re2) * ir * ir;
    const R f = in ? wr : R(0);
    if constexpr (CMPS) {
      const double num = (p_i + pj) - (ph_i + rj.phj);
      const R fn = (R)num * f;
#pragma unroll
      for (int a = 0; a < DIM; ++a) gs[a] += (double)(fn * d[a]);
    } else {
      if (in) m = fmin(m, pj);
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double fd = (double)(f * d[a]);
        gs[a] += pj * fd;
        bs[a] += fd;
      }
    }
  });
  if constexpr (!CMPS) m = team_min(m);
  const double cg = (double)DIM / v.n0_n;
  bool finite = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    double sum = team_sum(gs[a]);
    if constexpr (!CMPS) sum -= m * team_sum(bs[a]);
    const double gp = cg * sum;
    un[a] = us[a] - v.dt / rho_i * gp;
    xn[a] = rs[a] + v.dt * (un[a] - us[a]);
    finite = finite && isfinite(un[a]) && isfinite(xn[a]);
  }
  // no state is written after an error raised earlier in the call
  if (err) return;
  if (t == 0 && p_i != p_raw) v.p[row] = p_i;
  if (fluid && t == 0) {
    store_vec<DIM>(v.vel_w, row, un);
    store_vec<DIM>(v.pos_w, row, xn);
    if (!finite) atomicOr(v.status, ST_NONFINITE);
  }
}

static inline unsigned team_blocks(int64_t n) {
  return (unsigned)((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
}

template <int DIM>
static void predict_t(const View& v, bool mx, bool keep, hipStream_t s) {
  const unsigned nb = team_blocks(v.n);
  const bool multi = v.rho_s != nullptr;
  if (keep && !multi) {
    if (mx) k_predict_keep<DIM, true><<<nb, BLOCK, 0, s>>>(v);
    else k_predict_keep<DIM, false><<<nb, BLOCK, 0, s>>>(v);
    return;
  }
  if (mx) {
    if (multi) k_predict<DIM, true, true><<<nb, BLOCK, 0, s>>>(v);
    else k_predict<DIM, true, false><<<nb, BLOCK, 0, s>>>(v);
  } else {
    if (multi) k_predict<DIM, false, true><<<nb, BLOCK, 0, s>>>(v);
    else k_predict<DIM, false, false><<<nb, BLOCK, 0, s>>>(v);
  }
}

int launch_predict(const View& v, int dim, int precision, bool filter_kept, hipStream_t s) {
  const bool mx = precision == MPS_MIXED;
  if (dim == 2) {
    predict_t<2>(v, mx, filter_kept, s);
  } else {
    predict_t<3>(v, mx, filter_kept, s);
  }
  return 0;
}

template <int DIM>
static void density_t(const View& v, unsigned nb, int wc, hipStream_t s) {
  if (v.source == MPS_SRC_HS) k_density<DIM, MPS_SRC_HS><<<nb, BLOCK, 0, s>>>(v, wc);
  else if (v.source == MPS_SRC_HS_ECS) k_density<DIM, MPS_SRC_HS_ECS><<<nb, BLOCK, 0, s>>>(v, wc);
  else k_density<DIM, MPS_SRC_STD><<<nb, BLOCK, 0, s>>>(v, wc);
}

int launch_density(const View& v, int dim, int precision, int pmode, hipStream_t s) {
  const unsigned nb = team_blocks(v.n);
  const bool mx = precision == MPS_MIXED;
  const int wc = pmode == MPS_WC_EOS;
  (void)mx;
  if (dim == 2) density_t<2>(v, nb, wc, s);
  else density_t<3>(v, nb, wc, s);
  return 0;
}

int launch_viscosity(const View& v, int dim, int precision, hipStream_t s) {
  const unsigned nb = team_blocks(v.n);
  const bool mx = precision == MPS_MIXED;
  if (dim == 2) {
    if (mx) k_viscosity<2, true><<<nb, BLOCK, 0, s>>>(v);
    else k_viscosity<2, false><<<nb, BLOCK, 0, s>>>(v);
  } else {
    if (mx) k_viscosity<3, true><<<nb, BLOCK, 0, s>>>(v);
    else k_viscosity<3, false><<<nb, BLOCK, 0, s>>>(v);
  }
  return 0;
}

int launch_smooth_density(const View& v, const double* rho_raw, double* rho_out, int dim,
                          hipStream_t s) {
  const unsigned nb = team_blocks(v.n);
  if (dim == 2) k_smooth_density<2><<<nb, BLOCK, 0, s>>>(v, rho_raw, rho_out);
  else k_smooth_density<3><<<nb, BLOCK, 0, s>>>(v, rho_raw, rho_out);
  return 0;
}

template <int DIM, bool MIXED>
static void gradient_dim(const View& v, hipStream_t s) {
  const unsigned nb = team_blocks(v.n);
  if (v.grad == MPS_GRAD_CMPS) {
    // the CG residual buffer is free at this point of the step
    double* phat = v.r;
    k_phat<DIM, MIXED><<<nb, BLOCK, 0, s>>>(v, phat);
    k_gradient<DIM, MIXED, true><<<nb, BLOCK, 0, s>>>(v, phat);
  } else {
    k_gradient<DIM, MIXED, false><<<nb, BLOCK, 0, s>>>(v, nullptr);
  }
}

int launch_gradient(const View& v0, int dim, int precision, hipStream_t s) {
  const bool mx = precision == MPS_MIXED;
  // p-hat and the gradient walk the short lists (within re_n at r*) that
  // the density kernel of the step wrote
  View v = v0;
  v.nb_list = v0.nbn_list;
  v.nb_count = v0.nbn_count;
  if (dim == 2) {
    if (mx) gradient_dim<2, true>(v, s);
    else gradient_dim<2, false>(v, s);
  } else {
    if (mx) gradient_dim<3, true>(v, s);
    else gradient_dim<3, false>(v, s);
  }
  return 0;
}

}  // namespace mps
