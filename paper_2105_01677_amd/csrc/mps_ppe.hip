// Pressure Poisson equation of the fully incompressible model (arXiv
// 2105.01677, Eq. 13 with the Laplacian model of Eq. 7, or Eq. 23 (HL) with
// c_ij = 2 r_e / (n0 rho r_ij^3)): assembly (a5) and Jacobi-preconditioned
// conjugate gradients (a6).
//
// Matrix.  Row-wise as in the listing "PPE assemble GPU code": for a
// pressure unknown i (fluid or wall, not on the free surface) and every
// listed non-dummy neighbour j with |r*_j - r*_i| < re_lap,
//     c_ij = 2d w(r*_ij) / (lambda n0 rho),
//     A_ii += c_ij,  A_ij = -c_ij if j is an unknown too,
// and A_ii += alpha/dt^2 (the listing's 1e-7/dt^2 term).  A free-surface
// neighbour (Dirichlet p = 0) keeps its c_ij on the diagonal only, so A is
// exactly symmetric and strictly diagonally dominant, hence SPD.
// Right-hand side b_i = (n*_i - n0)/(n0 dt^2).  Rows that are not unknowns
// are identity rows with b = 0.
//
// Storage.  Off-diagonal entries compacted per row in the sliced layout
// (mps_internal.h): FP32 values on the mixed path, FP64 otherwise; the
// diagonal is FP64 and, on the mixed path, the FP64 sum of the rounded FP32
// couplings, so each row of the stored matrix sums exactly like the FP64
// matrix built from the same FP32 couplings.
//
// Solver.  Two kernels per iteration, all scalars on the device:
//   k_cg_spmv    p = z + beta p_old (fused, computed on the fly for the
//                neighbours too), q = A p, (p, q); alpha = rz/(p, q)
//   k_cg_update  x += alpha p, r -= alpha q, z = r/diag, (r, z), (r, r);
//                beta, convergence flag
// FP64 dot products: wave64 shuffles, LDS across the workgroup, and the
// last workgroup to finish sums the per-workgroup partials in index order,
// so every reduction is deterministic.  Once converged, further launches
// return immediately, which lets the host enqueue iterations in batches and
// poll rarely.
#include "mps_internal.h"


// list entries per lane and step of the assembly (measured on MI355X: 2
// beats 1 by 13 % at 441,282 particles and 4 % at 44,832)
#ifndef ASM_UNROLL
#define ASM_UNROLL 2
#endif

namespace mps {

template <int DIM, bool MIXED>
struct PosRefP;

template <int DIM>
struct PosRefP<DIM, false> {
  using R = double;
  double x[DIM];
  __device__ static PosRefP load(const View& v, int64_t i) {
    PosRefP p;
    load_vec<DIM>(v.rs, i, p.x);
    return p;
  }
  __device__ void diff(const PosRefP& o, float, R (&d)[DIM]) const {
#pragma unroll
    for (int a = 0; a < DIM; ++a) d[a] = o.x[a] - x[a];
  }
};

template <int DIM>
struct PosRefP<DIM, true> {
  using R = float;
  float4 f;
  __device__ static PosRefP load(const View& v, int64_t i) {
    PosRefP p;
    p.f = v.rsf[i];
    return p;
  }
  __device__ int32_t pc() const { return __float_as_int(DIM == 2 ? f.z : f.w); }
  __device__ void diff(const PosRefP& o, float cs, R (&d)[DIM]) const {
    const int32_t a = pc(), b = o.pc();
    d[0] = (o.f.x - f.x) + (float)(ucx(b) - ucx(a)) * cs;
    d[1] = (o.f.y - f.y) + (float)(ucy(b) - ucy(a)) * cs;
    if constexpr (DIM == 3) d[2] = (o.f.z - f.z) + (float)(ucz(b) - ucz(a)) * cs;
  }
};

// Sum over the workgroup (NT threads) in a fixed order, valid in every
// thread: wavefront sums, then the NT / WAVE of them in order.  sh holds
// NV * NT / WAVE doubles; it is read after the barrier, so a second use of
// the same sh needs a barrier first.
template <int NV, int NT>
__device__ inline void block_sum_all(double (&x)[NV], double* sh) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (int k = 0; k < NV; ++k) x[k] = wave_sum_last(x[k]);
  if ((threadIdx.x & (WAVE - 1)) == WAVE - 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * NW + w] = x[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = sh[k * NW];
#pragma unroll
    for (int q = 1; q < NW; ++q) s += sh[k * NW + q];
    x[k] = s;
  }
}

// The same with a buffer of its own and a closing barrier (may be called
// again in the same kernel); result valid in every thread.
template <int NV, int NT = BLOCK>
__device__ inline void block_sum(double (&x)[NV]) {
  __shared__ double sh[NV * (NT / WAVE)];
  block_sum_all<NV, NT>(x, sh);
  __syncthreads();
}

// Sum of np per-workgroup partials (stride doubles apart) in a fixed order;
// every thread gets the result.  All workgroups that call this on the same
// data obtain the same bits.
template <int NV, int NT = BLOCK>
__device__ inline void sum_partials(const double* part, int np, int stride, double (&tot)[NV]) {
  __shared__ double sh[NV * (NT / WAVE)];
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = 0.0;
  for (int b = threadIdx.x; b < np; b += NT) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] += part[(int64_t)b * stride + k];
  }
  block_sum_all<NV, NT>(tot, sh);
}

// Contiguous chunk of row groups (rpb rows each) handled by this workgroup
// of a grid-capped team kernel.
struct Chunk {
  int64_t g0, g1;
  __device__ Chunk(int64_t n, int rpb = ROWS_PER_BLOCK) {
    const int64_t ng = (n + rpb - 1) / rpb;
    const int64_t per = (ng + gridDim.x - 1) / gridDim.x;
    g0 = (int64_t)xcd_block() * per;
    g1 = g0 + per < ng ? g0 + per : ng;
  }
};

// a5: assembly of row i by its team, plus the CG start:
// x0 = warm start (previous pressure) or 0, r0 = b - A x0, z0 = r0/diag,
// p_old = 0 so that the first SpMV forms p = z0.  Per-workgroup partials of
// (r0, z0), (r0, r0), (b, b) go to partA.
template <int DIM, bool MIXED, bool MULTI>
__global__ __launch_bounds__(BLOCK) void k_assemble(View v, const double* rhs, int zero_x0) {
  using P = PosRefP<DIM, MIXED>;
  using R = typename P::R;
  using VT = R;
  const int t = team_lane();
  double rz = 0.0, rr = 0.0, bb = 0.0;
  VT* aval = reinterpret_cast<VT*>(v.a_val);
  const Chunk ch(v.n);
  const int ng = v.kpad / TEAM;  // slot groups of a row
  for (int64_t g = ch.g0; g < ch.g1; ++g) {
    const int64_t row = g * ROWS_PER_BLOCK + threadIdx.x / TEAM;
    if (row >= v.n) continue;
    // the row's own loads and its first list entries are issued together
    // (no branch before the list)
    const bool inner = v.flags[row] == MPS_FLAG_INNER;
    const int cnt_all = v.nb_count[row];
    const P pi = P::load(v, row);
    const double rho_i = MULTI ? v.rho_s[row] : 0.0;
    const double p_row = v.p[row], ns_row = v.nstar[row];
    const double rhs_row = rhs ? rhs[row] : 0.0;
    const double src_row = v.source != MPS_SRC_STD ? v.src[row] : 0.0;
    const int cnt = inner ? cnt_all : 0;
    double dsum = 0.0, ax = 0.0;
    int nnz = 0;
    {
      const R re = (R)v.re_lap, re2 = (R)v.re_lap2;
      const R cpp = (R)(2.0 * DIM / (v.lam_lap * v.n0_lap * v.rho));
      // Eq. 23 (HL): c_ij = 2 r_e / (n0 rho r_ij^3)
      const R chl = (R)(2.0 * v.re_lap / (v.n0_lap * v.rho));
      const bool hl = v.laplacian == MPS_LAP_HL;
      // ASM_UNROLL list entries per lane and step: the gathers of a step in
      // flight together while the next step's list entries load (slot
      // indices past kpad clamped to the row's first slot), then the
      // ballots in list order
      constexpr int U = ASM_UNROLL;
      const int64_t e0 = sl_index(row, t, v.kpad);
      int32_t jn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) jn[u] = v.nb_list[e0 + (int64_t)(u < ng ? u : 0) * WAVE];
      for (int k0 = 0; k0 * TEAM < cnt; k0 += U) {
        int32_t j[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          ok[u] = t + (k0 + u) * TEAM < cnt;
          j[u] = ok[u] ? jn[u] : (int32_t)row;
        }
        int8_t fj[U];
        P pj_pos[U];
        double pj[U], rhoj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          fj[u] = v.flags[j[u]];
          pj_pos[u] = P::load(v, j[u]);
          pj[u] = v.p[j[u]];
          rhoj[u] = MULTI ? v.rho_s[j[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = k0 + U + u;
          jn[u] = v.nb_list[e0 + (int64_t)(k < ng ? k : 0) * WAVE];
        }
        R c[U];
        bool keep[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // this step's flags mark exactly the dummy particles MPS_FLAG_DUMMY
          R d[DIM];
          pi.diff(pj_pos[u], v.cs32, d);
          R r2 = d[0] * d[0] + d[1] * d[1];
          if constexpr (DIM == 3) r2 += d[2] * d[2];
          if (zero_x0) pj[u] = 0.0;
          const bool cand = ok[u] && fj[u] != MPS_FLAG_DUMMY;
          bool in = cand && r2 < re2;
          if constexpr (MIXED) {
            // the HL coupling does not vanish at r_e: a pair within the FP32
            // rounding of the cut-off is decided on the FP64 positions r*,
            // as the FP64 path decides it (rare: a thin shell)
            if (hl && cand && fabsf(r2 - re2) < 1e-5f * re2) {
              double a[DIM], b[DIM];
              load_vec<DIM>(v.rs, row, a);
              load_vec<DIM>(v.rs, j[u], b);
              double s2 = 0.0;
#pragma unroll
              for (int q = 0; q < DIM; ++q) s2 += (b[q] - a[q]) * (b[q] - a[q]);
              in = s2 < v.re_lap2;
            }
          }
          const R ir = rsqrt_k(r2);
          R cr = hl ? chl * (ir * ir * ir) : cpp * weight_r2<R>(v.kernel, r2, ir, re, re2);
          // two-phase: 1/rho -> 2/(<rho>_i + <rho>_j), symmetric
          if constexpr (MULTI) cr *= (R)(v.rho * 2.0 * rcp_k(rho_i + rhoj[u]));
          c[u] = in ? cr : R(0);
          dsum += (double)c[u];
          keep[u] = in && fj[u] == MPS_FLAG_INNER;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t m = team_ballot(keep[u]);
          if (keep[u]) {
            const int s = nnz + __popc(m & ((1u << t) - 1u));
            const int64_t e = sl_index(row, s, v.kpad);
            v.a_col[e] = j[u];
            aval[e] = -c[u];
            ax -= (double)c[u] * pj[u];
          }
          nnz += __popc(m);
        }
      }
      dsum = team_sum(dsum);
      ax = team_sum(ax);
    }
    if (t == 0) {
      double diag = 1.0, b = 0.0, x0 = 0.0;
      if (inner) {
        diag = dsum + v.alpha / (v.dt * v.dt);
        b = rhs ? rhs_row
                : v.source != MPS_SRC_STD ? src_row
                                          : (ns_row - v.n0_n) / (v.n0_n * v.dt * v.dt);
        x0 = zero_x0 ? 0.0 : p_row;
      }
      const double r0 = b - diag * x0 - ax;
      const double z0 = r0 / diag;
      v.a_nnz[row] = nnz;
      v.diag[row] = diag;
      v.b[row] = b;
      if (!inner || zero_x0) v.p[row] = x0;
      v.r[row] = r0;
      v.z[row] = z0;
      v.pd[0][row] = 0.0;
      rz += r0 * z0;
      rr += r0 * r0;
      bb += b * b;
    }
  }
  double x[3] = {rz, rr, bb};
  block_sum<3>(x);
  if (threadIdx.x == 0) {
    const int lb = xcd_block();
#pragma unroll
    for (int k = 0; k < 3; ++k) v.partA[(int64_t)lb * 4 + k] = x[k];
    if (blockIdx.x == 0) {
      CGScalars* sc = v.sc;
      sc->k_next = 0;
      sc->converged = 0;
      sc->iter = 0;
      sc->nasm = gridDim.x;
      sc->cg_bits = 0ull;
    }
  }
}

// a6, part 1 (iteration k): reduce the partials of the previous kernel into
// (r, z) and (r, r); stop if converged; beta = rz_k / rz_{k-1};
// p = z + beta p_old (formed on the fly for the neighbours as well),
// q = A p, per-workgroup (p, q).
template <class VT>
__global__ __launch_bounds__(BLOCK) void k_cg_spmv(View v) {
  CGScalars* sc = v.sc;
  if (sc->converged) return;
  const int k = sc->k_next;
  double tot[3];
  if (k == 0) {
    sum_partials<3>(v.partA, sc->nasm, 4, tot);
  } else {
    double t2[2];
    sum_partials<2>(v.partA, v.nupd, 4, t2);
    tot[0] = t2[0];
    tot[1] = t2[1];
    tot[2] = sc->bb;
  }
  const double rz = tot[0], rr = tot[1], bb = tot[2];
  const bool done = bb == 0.0 || rr <= v.cg_tol2 * bb;
  const Chunk ch(v.n);
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->rr = rr;
    sc->k_cur = k;
    sc->rzh[k & 1] = rz;
    if (k == 0) sc->bb = bb;
    if (done) {
      sc->converged = 1;
      sc->iter = k;
    }
  }
  if (done) {
    if (bb == 0.0) {  // b = 0: the solution is p = 0
      for (int64_t g = ch.g0; g < ch.g1; ++g) {
        const int64_t row = g * ROWS_PER_BLOCK + threadIdx.x / TEAM;
        if (row < v.n && team_lane() == 0) v.p[row] = 0.0;
      }
    }
    return;
  }
  const double beta = k == 0 ? 0.0 : rz / sc->rzh[(k - 1) & 1];
  const double* __restrict__ pold = v.pd[k & 1];
  double* __restrict__ pnew = v.pd[(k + 1) & 1];
  const VT* __restrict__ aval = reinterpret_cast<const VT*>(v.a_val);
  const int t = team_lane();
  double pq = 0.0;
  for (int64_t g = ch.g0; g < ch.g1; ++g) {
    const int64_t row = g * ROWS_PER_BLOCK + threadIdx.x / TEAM;
    if (row >= v.n) continue;
    const int nnz = v.a_nnz[row];
    const double* __restrict__ z = v.z;
    double s = row_dot<4>(v.a_col, aval, row, nnz, v.kpad, t,
                       [&](int32_t j) { return z[j] + beta * pold[j]; });
    s = team_sum(s);
    if (t == 0) {
      const double pi = v.z[row] + beta * pold[row];
      const double qi = v.diag[row] * pi + s;
      pnew[row] = pi;
      v.q[row] = qi;
      pq += pi * qi;
    }
  }
  double x[1] = {pq};
  block_sum<1>(x);
  if (threadIdx.x == 0) v.partB[xcd_block()] = x[0];
}

// a6, part 2 (iteration k): alpha = rz_k / (p, q) from the SpMV partials;
// x += alpha p, r -= alpha q, z = r/diag, per-workgroup (r, z), (r, r).
__global__ __launch_bounds__(BLOCK) void k_cg_update(View v) {
  CGScalars* sc = v.sc;
  if (sc->converged) return;
  const int k = sc->k_cur;
  double pq[1];
  sum_partials<1>(v.partB, v.nspmv, 1, pq);
  const double alpha = sc->rzh[k & 1] / pq[0];
  const double* __restrict__ pcur = v.pd[(k + 1) & 1];
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < v.n;
       i += (int64_t)gridDim.x * BLOCK) {
    v.p[i] += alpha * pcur[i];
    const double r = v.r[i] - alpha * v.q[i];
    const double z = r / v.diag[i];
    v.r[i] = r;
    v.z[i] = z;
    rz += r * z;
    rr += r * r;
  }
  double x[2] = {rz, rr};
  block_sum<2>(x);
  if (threadIdx.x == 0) {
    v.partA[(int64_t)blockIdx.x * 4 + 0] = x[0];
    v.partA[(int64_t)blockIdx.x * 4 + 1] = x[1];
    if (blockIdx.x == 0) {
      sc->k_next = k + 1;
      sc->iter = k + 1;
    }
  }
}

// ------------------------------------------------------- pipelined variant
// Preconditioned CG with one global reduction per iteration (Ghysels and
// Vanroose's pipelined CG), preconditioner M:
//   gamma = (r, u), delta = (w, u), m = M^-1 w, n = A m,
//   beta = gamma/gamma_old, alpha = gamma/(delta - beta gamma/alpha_old),
//   z = n + beta z, q = m + beta q, s = w + beta s, p = u + beta p,
//   x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z.
// With the Jacobi preconditioner M = D = diag(A) the recurrences u = D^-1 r
// and q = D^-1 s reduce to one division each, so u and q are not stored,
// and w = D m is not stored either: m is the one vector the SpMV gathers,
// double buffered because the neighbours' m of this iteration are read
// while the new m is written.  Per row an iteration loads D, m, z, s, p, r,
// x and stores m, z, s, p, r, x.  With block Jacobi (BJ, below) or the
// two-level M (TWO) u, q and w are stored as well.
// Every workgroup handles one group of PCG_ROWS rows and leaves one partial
// of the next iteration's dot products.  Two schedules:
//   fused  (grid <= pcg_fused_capacity(), all workgroups resident): one
//          kernel per iteration; every workgroup reduces all partials of
//          the previous iteration itself, in the same fixed order;
//   split  (larger grids): PCG_SPLIT_G workgroups first sum contiguous
//          slices of the partials (fixed order), then every workgroup of
//          the iteration kernel sums those slice sums itself.
// In both, every load that does not depend on the scalars (the row length,
// its first matrix entries, the gathers of m, the row's own vectors) is
// issued first, so their latencies overlap.
// Setup: w0 = A u0 with u0 = M^-1 r0 (Jacobi: D^-1 r0 from the assembly;
// block Jacobi: k_bj_start; two-level: plus the coarse correction), and
// m0 = M^-1 w0; gamma_old = inf and alpha_old = 1 make the first iteration
// beta = 0, alpha = gamma/delta.
// workgroup size of the two schedules (measured on MI355X: 512 fused, 256
// split)
template <bool FUSED>
constexpr int pcg_nt() { return FUSED ? PCG_BLOCK : PCG_SPLIT_BLOCK; }
constexpr int PCG_PK = (PCG_MAX_BLOCKS + PCG_BLOCK - 1) / PCG_BLOCK;

// Quantity k of workgroup b's partial of the pipelined iteration: the fused
// schedule keeps one array per quantity (PCG_PSTRIDE doubles each, zeros
// past npcg), the split schedule four doubles per workgroup.
template <bool FUSED>
__device__ inline int64_t part_at(int64_t b, int k) {
  return FUSED ? (int64_t)k * PCG_PSTRIDE + b : b * 4 + k;
}
// fused: each of six wavefronts loads PCG_FQ double2 per lane, one half of
// one quantity's array
constexpr int PCG_FQ = PCG_PSTRIDE / (2 * 2 * WAVE);
static_assert(PCG_FQ * 2 * 2 * WAVE == PCG_PSTRIDE, "whole double2 loads per lane");

// Fixed-order sum of np partials (double4 .x/.y/.z) by one workgroup of NT
// threads: thread i adds partials i, i + NT, ... in order (K loads in
// flight), then the workgroup tree.  Result valid in every thread.
template <int NT, int K>
__device__ inline void reduce_partials(const double* part, int np, double (&tot)[3]) {
  const double4* p4 = reinterpret_cast<const double4*>(part);
  double s[3] = {0.0, 0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < np; b0 += K * NT) {
    double4 q[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int b = b0 + k * NT;
      q[k] = b < np ? p4[b] : make_double4(0.0, 0.0, 0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s[0] += q[k].x;
      s[1] += q[k].y;
      s[2] += q[k].z;
    }
  }
  __shared__ double sh[3 * (NT / WAVE)];
  block_sum_all<3, NT>(s, sh);
  tot[0] = s[0];
  tot[1] = s[1];
  tot[2] = s[2];
}

// Start of the solve from the assembly partials: (r0, r0), (b, b), the
// convergence test, and the scalars that make iteration 0 take beta = 0.
__device__ inline bool pcg_start_scalars(const View& v, const double (&tot)[3], bool write) {
  CGScalars* sc = v.sc;
  const double rr = tot[1], bb = tot[2];
  const bool done = bb == 0.0 || rr <= v.cg_tol2 * bb;
  if (write && threadIdx.x == 0) {
    sc->bb = bb;
    sc->rr = rr;
    sc->iter = 0;
    sc->converged = done ? 1 : 0;
    sc->gam[1] = 0.0;  // 1 / (r,u) of a previous iteration: beta = 0
    sc->alp[1] = 1.0;
  }
  return done;
}

// split schedule: the assembly partials reduced once
__global__ __launch_bounds__(RED_BLOCK) void k_pcg_start(View v) {
  double tot[3];
  reduce_partials<RED_BLOCK, 2>(v.partA, v.sc->nasm, tot);
  pcg_start_scalars(v, tot, true);
}

// Block Jacobi (BJ): the diagonal blocks A_B of A over groups of BJ_ROWS
// consecutive rows, [BJ_ROWS g, BJ_ROWS (g + 1)), which are the rows of one
// workgroup of the fused schedule, approximated by one damped Neumann step:
//   M^-1 w = D^-1 (w - omega (A_B - D) D^-1 w),
// i.e. row i subtracts omega a_ij w_j / d_j over its entries j of the same
// group.  With N = D^-1/2 (A_B - D) D^-1/2 (zero diagonal, entries <= 0),
// M^-1 = D^-1/2 (I - omega N) D^-1/2 is symmetric, and positive definite
// while omega lambda_max(N) < 1.  lambda_max(N) is small because a group's
// neighbour graph is far from bipartite: measured 0.25 (2-D, kernel
// Laplacian) and 0.42 (2-D, Eq. 23 Laplacian) on the dam-break matrices,
// 0.10 and 0.18 in 3-D, so omega = 1.5 keeps M^-1 positive definite with
// margin (the undamped step, omega = 1, is definite for every weakly
// diagonally dominant A of this sign pattern).  CG iterations to 1e-9 on
// the 44,832-particle matrix: 89 Jacobi; omega 1, 1.5, 2: 69, 66, 65.
// A row's entries inside its group are the near ones of a cell-sorted
// order.
constexpr int BJ_ROWS = PCG_BLOCK / TEAM;
constexpr double BJ_OMEGA = 1.5;

// sum over the team's row entries j of its group of a_ij y[j - g0] (y in
// LDS, BJ_ROWS values), entries from slot l on
template <class VT>
__device__ inline double bj_row_sum(const View& v, const VT* __restrict__ aval, int64_t row,
                                    int nnz, int l, int32_t g0, const double* y) {
  return row_dot<4>(v.a_col, aval, row, nnz, v.kpad, l, [&](int32_t j) {
    const uint32_t k = (uint32_t)(j - g0);
    return k < (uint32_t)BJ_ROWS ? y[k] : 0.0;
  });
}

// u0 = M^-1 r0 of block Jacobi from z = D^-1 r0 (the assembly's), into
// pl_u; one team per row, one group per workgroup.
template <class VT>
__global__ __launch_bounds__(PCG_BLOCK) void k_bj_start(View v) {
  __shared__ double y[BJ_ROWS];
  const int lr = threadIdx.x / TEAM;
  const int64_t g0 = (int64_t)xcd_block() * BJ_ROWS;
  const int64_t row = g0 + lr;
  const int t = team_lane();
  const bool live = row < v.n;
  if (t == 0) y[lr] = live ? v.z[row] : 0.0;
  __syncthreads();
  if (!live) return;
  const VT* __restrict__ aval = reinterpret_cast<const VT*>(v.a_val);
  const double s = team_sum(bj_row_sum(v, aval, row, v.a_nnz[row], t, (int32_t)g0, y));
  if (t == 0) v.pl_u[row] = (v.r[row] - BJ_OMEGA * s) * (1.0 / v.diag[row]);
}

template <class VT, bool FUSED, bool TWO, bool BJ>
__global__ __launch_bounds__(pcg_nt<FUSED>()) void k_pcg_setup(View v) {
  constexpr int NT = pcg_nt<FUSED>();
  CGScalars* sc = v.sc;
  bool done;
  double bb;
  if constexpr (FUSED) {
    double tot[3];
    reduce_partials<NT, 1>(v.partA, sc->nasm, tot);
    done = pcg_start_scalars(v, tot, blockIdx.x == 0);
    bb = tot[2];
  } else {
    done = sc->converged != 0;
    bb = sc->bb;
  }
  const int64_t row = (int64_t)xcd_block() * (NT / TEAM) + threadIdx.x / TEAM;
  const int t = team_lane();
  if (done) {
    if (bb == 0.0 && row < v.n && t == 0) v.p[row] = 0.0;
    return;
  }
  static_assert(!BJ || (FUSED && TWO), "block Jacobi: fused schedule, u/q/w recurrences");
  const VT* __restrict__ aval = reinterpret_cast<const VT*>(v.a_val);
  // u0 = M^-1 r0: D^-1 r0 written by the assembly (plus, two-level, the
  // coarse correction added before this kernel; block Jacobi: k_bj_start's)
  const double* __restrict__ u0 = BJ ? v.pl_u : v.z;
  double gam = 0.0, del = 0.0, rr2 = 0.0;
  const bool live = row < v.n;
  double w = 0.0, dg = 1.0;
  if (live) {
    const int nnz = v.a_nnz[row];
    double s = row_dot<4>(v.a_col, aval, row, nnz, v.kpad, t,
                          [&](int32_t j) { return u0[j]; });
    s = team_sum(s);
    dg = v.diag[row];
    const double u = u0[row];
    w = dg * u + s;
    if (t == 0) {
      const double r = v.r[row];
      // m0 = D^-1 w0 (two-level: its coarse part is added after this kernel;
      // block Jacobi: written below)
      if constexpr (!BJ) v.pl_m[0][row] = w / dg;
      v.pl_z[row] = 0.0;
      v.pl_s[row] = 0.0;
      v.pd[0][row] = 0.0;
      if constexpr (TWO) {
        if constexpr (!BJ) v.pl_u[row] = u;  // block Jacobi: already there
        v.pl_q[row] = 0.0;
        v.pl_w[row] = w;
      }
      gam = r * u;
      del = w * u;
      rr2 = r * r;
    }
  }
  if constexpr (BJ) {
    // m0 = M^-1 w0 over the workgroup's group of rows
    __shared__ double y[BJ_ROWS];
    const int lr = threadIdx.x / TEAM;
    const int64_t g0 = row - lr;
    // (1 / d as in the iteration kernel)
    const double id = 1.0 / dg;
    if (t == 0) y[lr] = live ? w * id : 0.0;
    __syncthreads();
    if (live) {
      const double a = team_sum(bj_row_sum(v, aval, row, v.a_nnz[row], t, (int32_t)g0, y));
      if (t == 0) v.pl_m[0][row] = (w - BJ_OMEGA * a) * id;
    }
  }
  double x[3] = {gam, del, rr2};
  block_sum<3, NT>(x);
  if (threadIdx.x == 0) {
    const int lb = xcd_block();
#pragma unroll
    for (int k = 0; k < 3; ++k) v.pl_part[0][part_at<FUSED>(lb, k)] = x[k];
  }
}

// Scalars of iteration k from (r,u), (w,u), (r,r) of its partials: the
// convergence test, beta and alpha; workgroup 0 of the iteration kernel
// records them.
__device__ inline bool pcg_scalars(const View& v, const double (&tot)[3], int par,
                                   double igam_old, double alp_old, double bb, bool write,
                                   double& alpha, double& beta) {
  CGScalars* sc = v.sc;
  const double gam = tot[0], del = tot[1], rr = tot[2];
  const bool done = rr <= v.cg_tol2 * bb;
  // beta = gam / gam_old from the stored 1 / gam_old; alpha = gam / (del -
  // beta gam / alpha_old), with one division
  beta = gam * igam_old;
  alpha = gam * alp_old / (del * alp_old - beta * gam);
  if (write && threadIdx.x == 0) {
    sc->rr = rr;
    if (done) {
      sc->converged = 1;
    } else {
      sc->gam[par] = 1.0 / gam;
      sc->alp[par] = alpha;
      sc->iter += 1;
    }
  }
  return done;
}

// split schedule: workgroup g sums slice g of iteration k's partials (a
// contiguous range, fixed order) into pl_part2; the iteration kernel sums
// the npcg2 slice sums
template <int PAR>
__global__ __launch_bounds__(RED2_BLOCK) void k_pcg_reduce(View v) {
  if (v.sc->converged) return;
  const int per = (v.npcg + v.npcg2 - 1) / v.npcg2;
  const int b0 = blockIdx.x * per;
  const int nb = min(per, v.npcg - b0);
  double tot[3];
  reduce_partials<RED2_BLOCK, 4>(v.pl_part[PAR] + (int64_t)b0 * 4, nb > 0 ? nb : 0, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v.pl_part2[PAR][(int64_t)blockIdx.x * 4 + k] = tot[k];
  }
}

// PRED: slots past the row length are neither loaded nor gathered (the
// loads then wait for the row length).  Without it every lane loads its
// first U slots whatever the row length, which keeps the load chain short
// but reads padding for rows with few or no entries (dummy particles).
// Block Jacobi keeps three workgroups per CU resident (six waves per SIMD,
// at most 80 VGPRs), as the Jacobi and two-level kernels do by themselves,
// so that the systems of the fused schedule stay within it.
template <class VT, int PAR, bool FUSED, bool PRED, bool TWO, bool BJ>
__global__ __launch_bounds__(pcg_nt<FUSED>()) __attribute__((amdgpu_waves_per_eu(BJ ? 6 : 1)))
void k_pcg_iter(View v) {
  constexpr int U = CG_UNROLL;
  constexpr int NT = pcg_nt<FUSED>();
  static_assert(!BJ || (FUSED && TWO), "block Jacobi: fused schedule, u/q/w recurrences");
  static_assert(PCG_PK * PCG_BLOCK >= PCG_MAX_BLOCKS, "one partial load per slot");
  static_assert(PCG_SPLIT_G <= PCG_SPLIT_BLOCK, "one slice sum per thread");
  static_assert(!(FUSED && PRED), "the small fused systems are latency-bound");
  __shared__ double sh_in[3 * (NT / WAVE)], sh_lead[3][NT / TEAM];
  CGScalars* sc = v.sc;
  const int t = team_lane();

  // -- loads that do not need this iteration's scalars, all issued before
  //    the first wait: the previous partials, the row length, the first U
  //    entries per lane, the row's own vectors (every lane: clamped row) --
  // fused: every partial of the previous iteration, one quantity per
  // wavefront: wavefronts k and 4 + k (k < 3) load the first and the second
  // half of quantity k's array, wavefronts 3 and 7 none; split: wavefront k
  // (k < 3) loads quantity k of the slice sums, one per lane
  // the wavefront index, uniform (a scalar register)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), wk = wv & 3;
  double2 qf[FUSED ? PCG_FQ : 1];
  double qs = 0.0;
  if constexpr (FUSED) {
    static_assert(NT == 8 * WAVE, "two wavefronts per quantity");
    if (wk < 3) {
      const double2* p2 = reinterpret_cast<const double2*>(
                              v.pl_part[PAR] + part_at<true>((wv >> 2) * (PCG_PSTRIDE / 2), wk)) +
                          (threadIdx.x & (WAVE - 1));
#pragma unroll
      for (int j = 0; j < PCG_FQ; ++j) qf[j] = p2[j * WAVE];
    }
  } else {
    static_assert(PCG_SPLIT_G <= WAVE && NT / WAVE >= 3, "one slice sum per lane");
    const int l = threadIdx.x & (WAVE - 1);
    if (wk < 3) qs = l < v.npcg2 ? v.pl_part2[PAR][l * 4 + wk] : 0.0;
  }
  const double* __restrict__ M = v.pl_m[PAR];
  double* __restrict__ Mn = v.pl_m[PAR ^ 1];
  const VT* __restrict__ aval = reinterpret_cast<const VT*>(v.a_val);
  const int conv = sc->converged;
  const double igam_old = sc->gam[PAR ^ 1], alp_old = sc->alp[PAR ^ 1], bb = sc->bb;
  double alpha = 0.0, beta = 0.0;
  const int64_t row = (int64_t)xcd_block() * (NT / TEAM) + threadIdx.x / TEAM;
  const bool live = row < v.n;
  const int64_t rc = live ? row : v.n - 1;
  const int64_t e0 = sl_index(rc, t, v.kpad);
  int nnz = v.a_nnz[rc];
  int32_t jj[U];
  VT aa[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // slot u of the row exists (the context's row capacity kpad is at least
    // U * TEAM); stale slots past the row length are masked below
    const int64_t e = e0 + u * WAVE;
    if constexpr (PRED) {
      const bool in = t + u * TEAM < nnz;
      jj[u] = in ? v.a_col[e] : 0;
      aa[u] = in ? aval[e] : VT(0);
    } else {
      jj[u] = v.a_col[e];
      aa[u] = aval[e];
    }
  }
  // the row's own seven values, one per team lane (one load instruction;
  // moved to lane 0 below)
  const double* optr = t == 0 ? v.diag : t == 1 ? M : t == 2 ? v.pl_z : t == 3 ? v.pl_s
                       : t == 4 ? v.pd[0] : t == 5 ? v.r : v.p;
  const double ov = optr[rc];
  // non-diagonal M: u = M^-1 r, q = M^-1 s and w are recurrences of their
  // own, loaded the same way (u, q, w in team lanes 0, 1, 2)
  double ov2 = 0.0;
  if constexpr (TWO) ov2 = (t == 0 ? v.pl_u : t == 1 ? v.pl_q : v.pl_w)[rc];
  // a launch after convergence ends here, without waiting for the loads
  if (conv) return;
  // every load above is issued before any of them is waited for: without
  // this fence the compiler sinks slot loads behind the wait for the row
  // length, or consumes the partials before issuing the rest (one more
  // memory latency in the chain either way)
#pragma unroll
  for (int u = 0; u < U; ++u) asm volatile("" : "+v"(jj[u]), "+v"(aa[u])::"memory");
  if (!live) nnz = 0;
  double xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool in = t + u * TEAM < nnz;
    if constexpr (PRED) xv[u] = in ? M[jj[u]] : 0.0;
    else xv[u] = M[in ? jj[u] : (int32_t)rc];
    if (!in) {
      xv[u] = 0.0;
      aa[u] = VT(0);
    }
  }
  // block Jacobi: each of the lane's first U entries that lies in the
  // workgroup's group of rows, as (position in the group, value), the rest
  // as (BJ_ROWS, 0); parked in LDS by the lane itself (one byte per slot),
  // so that they are not held in registers over the reductions
  __shared__ uint2 sh_k[BJ ? NT : 1];
  __shared__ VT sh_a[BJ ? U : 1][BJ ? NT : 1];
  if constexpr (BJ) {
    static_assert(U <= 8 && BJ_ROWS < 256, "one byte per slot");
    const int32_t g0 = xcd_block() * BJ_ROWS;
    uint32_t kp[2] = {0u, 0u};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t k = (uint32_t)(jj[u] - g0);
      const bool ing = t + u * TEAM < nnz && k < (uint32_t)BJ_ROWS;
      kp[u / 4] |= (ing ? k : (uint32_t)BJ_ROWS) << (8 * (u % 4));
      sh_a[u][threadIdx.x] = ing ? aa[u] : VT(0);
    }
    sh_k[threadIdx.x] = make_uint2(kp[0], kp[1]);
  }

  // lane 0 of the team takes lane k's value (DPP row_shl:k)
  const double o_d = ov, o_m = dpp_move<DPP_SHL1>(ov), o_z = dpp_move<DPP_SHL2>(ov),
               o_s = dpp_move<DPP_SHL3>(ov), o_p = dpp_move<DPP_SHL4>(ov),
               o_r = dpp_move<DPP_SHL5>(ov), o_x = dpp_move<DPP_SHL6>(ov);
  const double o_u = ov2, o_q = dpp_move<DPP_SHL1>(ov2), o_w = dpp_move<DPP_SHL2>(ov2);

  // -- the scalars (every workgroup alike; workgroup 0 records them) --
  {
    double tot[3];
    if constexpr (FUSED) {
      if (wk < 3) {
        double ps = qf[0].x + qf[0].y;
#pragma unroll
        for (int j = 1; j < PCG_FQ; ++j) ps += qf[j].x + qf[j].y;
        ps = wave_sum_last(ps);
        if ((threadIdx.x & (WAVE - 1)) == WAVE - 1) sh_in[2 * wk + (wv >> 2)] = ps;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 3; ++k) tot[k] = sh_in[2 * k] + sh_in[2 * k + 1];
    } else {
      if (wk < 3) {
        const double ps = wave_sum_last(qs);
        if ((threadIdx.x & (WAVE - 1)) == WAVE - 1) sh_in[wk] = ps;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 3; ++k) tot[k] = sh_in[k];
    }
    if (pcg_scalars(v, tot, PAR, igam_old, alp_old, bb, blockIdx.x == 0, alpha, beta)) return;
  }
  // block Jacobi: 1 / d, while the gathers of m are waited for
  const double o_id = BJ ? 1.0 / o_d : 0.0;

  double s = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) s += (double)aa[u] * xv[u];
  // entries beyond the first U per lane (measured: cheaper here than
  // before the reduction; block Jacobi: two loads in flight per step, which
  // keeps its registers within three workgroups per CU)
  s += row_dot<BJ ? 2 : 4>(v.a_col, aval, rc, nnz, v.kpad, t + U * TEAM,
                           [&](int32_t j) { return M[j]; });
  s = team_sum(s);
  const bool lead = live && t == 0;
  double r, wn, un;
  if constexpr (TWO) {
    // n = A m, z = n + beta z, q = m + beta q, s = w + beta s,
    // p = u + beta p; x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z
    const double z = (o_d * o_m + s) + beta * o_z;
    const double qv = o_m + beta * o_q;
    const double sv = o_w + beta * o_s;
    const double pv = o_u + beta * o_p;
    r = o_r - alpha * sv;
    un = o_u - alpha * qv;
    wn = o_w - alpha * z;
    if (lead) {
      v.p[row] = o_x + alpha * pv;
      v.pl_z[row] = z;
      v.pl_s[row] = sv;
      v.pd[0][row] = pv;
      v.r[row] = r;
      v.pl_u[row] = un;
      v.pl_q[row] = qv;
      v.pl_w[row] = wn;
      // the coarse part is added after this kernel
      if constexpr (!BJ) Mn[row] = wn / o_d;
    }
  } else {
    const double w = o_d * o_m;
    const double z = (w + s) + beta * o_z;
    const double sv = w + beta * o_s;
    const double pv = o_r / o_d + beta * o_p;
    r = o_r - alpha * sv;
    wn = w - alpha * z;
    un = r / o_d;
    // the stores go out before the reduction (its barrier waits for LDS
    // only), so their latency overlaps it
    if (lead) {
      v.p[row] = o_x + alpha * pv;
      v.pl_z[row] = z;
      v.pl_s[row] = sv;
      v.pd[0][row] = pv;
      v.r[row] = r;
      Mn[row] = wn / o_d;
    }
  }
  // the workgroup's partial: one value per row, from the team leads
  if (t == 0) {
    const int i = threadIdx.x / TEAM;
    sh_lead[0][i] = live ? r * un : 0.0;
    sh_lead[1][i] = live ? wn * un : 0.0;
    sh_lead[2][i] = live ? r * r : 0.0;
  }
  // block Jacobi: D^-1 w of the group's rows into LDS before the
  // barrier below, read after it; the lane's parked entries are read
  // back before it (its own data; FP64 values after it, for registers)
  __shared__ double y[BJ ? BJ_ROWS + 1 : 1];
  constexpr bool KA_EARLY = sizeof(VT) == 4;
  uint2 kq;
  VT ka[BJ ? U : 1];
  if constexpr (BJ) {
    if (t == 0) y[threadIdx.x / TEAM] = live ? wn * o_id : 0.0;
    if (threadIdx.x == 0) y[BJ_ROWS] = 0.0;
    kq = sh_k[threadIdx.x];
    if constexpr (KA_EARLY) {
#pragma unroll
      for (int u = 0; u < U; ++u) ka[u] = sh_a[u][threadIdx.x];
    }
  }
  __syncthreads();
  // the last three wavefronts each sum one quantity's row values (one per
  // lane) into the partial
  {
    static_assert(NT / TEAM <= WAVE && NT / WAVE >= 3, "one row per lane");
    const int k = NT / WAVE - 1 - wv, l = threadIdx.x & (WAVE - 1);
    if (k < 3) {
      double x = l < NT / TEAM ? sh_lead[k][l] : 0.0;
      x = wave_sum_last(x);
      if (l == WAVE - 1) v.pl_part[PAR ^ 1][part_at<FUSED>(xcd_block(), k)] = x;
    }
  }
  if constexpr (BJ) {
    // m = M^-1 w: the first U entries per lane parked, the rest reloaded
    if constexpr (!KA_EARLY) {
#pragma unroll
      for (int u = 0; u < U; ++u) ka[u] = sh_a[u][threadIdx.x];
    }
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t kk = ((u < 4 ? kq.x : kq.y) >> (8 * (u % 4))) & 0xffu;
      a += (double)ka[u] * y[kk];
    }
    a += bj_row_sum(v, aval, rc, nnz, t + U * TEAM, xcd_block() * BJ_ROWS, y);
    a = team_sum(a);
    if (lead) Mn[row] = (wn - BJ_OMEGA * a) * o_id;
  }
}

// ------------------------------------------------- two-level preconditioner
// M^-1 = D^-1 + P C P^T.  Aggregates: the cells of the background grid (side
// >= re_lap); P sums the pressure unknowns (flags inner) of a cell, whose
// rows are contiguous in the sorted order ([cell_start[a], cell_start[a+1]);
// with lists kept over steps, the cells of the last build, which the order
// follows).  Every matrix entry couples cells at most one apart, so the cell
// operator A_c = P^T A P is a 3^DIM-point stencil on the grid.  C: CHEB_K
// steps of the Chebyshev iteration for A_c, preconditioned by its diagonal,
// on [G/10, G], G the largest Gershgorin bound of D_c^-1 A_c (so the
// polynomial is positive on the spectrum and M is symmetric positive
// definite).  All sums in a fixed order.
#ifndef CHEB_K
#define CHEB_K 3
#endif
template <int DIM>
constexpr int nsten() { return DIM == 3 ? 27 : 9; }

__device__ inline int cell_lin(const View& v, int32_t pc) {
  return ucx(pc) + v.nx * (ucy(pc) + v.ny * ucz(pc));
}

// Stencil slot of cell b seen from cell a (both packed, at most one apart).
template <int DIM>
__device__ inline int sten_slot(int32_t pa, int32_t pb) {
  const int dx = ucx(pb) - ucx(pa) + 1, dy = ucy(pb) - ucy(pa) + 1;
  if constexpr (DIM == 3) return dx + 3 * dy + 9 * (ucz(pb) - ucz(pa) + 1);
  return dx + 3 * dy;
}

// A_c, stored slot-major (ac[o * ncell + cell]), in three kernels:
// k_coarse_rows: one team per row (32 rows per workgroup, like the
//   assembly): each lane adds every 8th matrix entry of its row into the
//   bin of the neighbour cell's stencil slot (COARSE_U entries per step,
//   their loads issued together; bins in registers, selected without
//   indexing), the team sums its bins; the workgroup then sums its rows by
//   runs of equal cell (rows are sorted by cell) in row order.  A run whose
//   cell lies wholly in the workgroup's rows is written to A_c; a cell that
//   crosses the workgroup's first or last row leaves its partial in head /
//   tail slots of the workgroup.
// k_coarse_join: every cell that spans workgroups b0 < b1 sums tail[b0],
//   head[b] of the workgroups between and head[b1], in that order.
// k_coarse_bound: the Gershgorin bound of every cell row, one maximum per
//   workgroup, and k_coarse_gmax the largest of those.
#ifndef COARSE_U
#define COARSE_U 4
#endif
constexpr int CROWS = ROWS_PER_BLOCK;   // rows per workgroup of k_coarse_rows

template <int DIM, class VT>
__global__ __launch_bounds__(BLOCK) void k_coarse_rows(View v, double* head, double* tail) {
  constexpr int NS = nsten<DIM>();
  constexpr int CEN = NS / 2;
  constexpr int U = COARSE_U;
  __shared__ double rows[CROWS][NS];
  __shared__ int32_t rcell[CROWS];
  const int lr = threadIdx.x / TEAM;
  const int64_t row = (int64_t)blockIdx.x * CROWS + lr;
  const int t = team_lane();
  const VT* __restrict__ aval = reinterpret_cast<const VT*>(v.a_val);
  double bin[NS];
#pragma unroll
  for (int o = 0; o < NS; ++o) bin[o] = 0.0;
  int32_t pi = GHOST_CELL;
  bool inner = false;
  if (row < v.n) {
    inner = v.flags[row] == MPS_FLAG_INNER;
    pi = v.pcell[row];
  }
  if (inner) {
    if (t == 0) bin[CEN] = v.diag[row];
    const int nnz = v.a_nnz[row];
    for (int l0 = t; l0 < nnz; l0 += U * TEAM) {
      int32_t jj[U];
      double aa[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = l0 + u * TEAM;
        // past the row: slot l0 again (an entry of the row), weight 0
        const int64_t e = sl_index(row, l < nnz ? l : l0, v.kpad);
        jj[u] = v.a_col[e];
        aa[u] = l < nnz ? (double)aval[e] : 0.0;
      }
      int32_t pj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pj[u] = v.pcell[jj[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int slot = sten_slot<DIM>(pi, pj[u]);
#pragma unroll
        for (int o = 0; o < NS; ++o) bin[o] += slot == o ? aa[u] : 0.0;
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NS; ++o) {
    const double x = team_sum(bin[o]);
    if (t == 0) rows[lr][o] = x;
  }
  if (t == 0) rcell[lr] = (row < v.n && pi != GHOST_CELL) ? cell_lin(v, pi) : -1;
  __syncthreads();
  // runs of equal cell among the workgroup's rows: thread k < NS sums slot
  // k of every run in row order
  const int64_t r0 = (int64_t)blockIdx.x * CROWS;
  const int nr = (int)min<int64_t>(CROWS, v.n - r0);
  if (threadIdx.x < NS) {
    const int o = threadIdx.x;
    int k = 0;
    while (k < nr) {
      const int c = rcell[k];
      int e = k;
      double sum = 0.0;
      while (e < nr && rcell[e] == c) sum += rows[e++][o];
      if (c >= 0) {
        const bool starts = v.cell_start[c] >= r0, ends = v.cell_start[c + 1] <= r0 + nr;
        if (starts && ends) v.ac[(int64_t)o * v.ncell + c] = sum;
        else {
          if (k == 0) head[(int64_t)blockIdx.x * NS + o] = sum;
          if (e == nr) tail[(int64_t)blockIdx.x * NS + o] = sum;
        }
      }
      k = e;
    }
  }
}

// Cells whose rows span workgroups: the partials in workgroup order.
// Cells without rows get a zero centre slot.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_coarse_join(View v, const double* head,
                                                       const double* tail) {
  constexpr int NS = nsten<DIM>();
  const int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= v.ncell) return;
  const int cs = v.cell_start[c], ce = v.cell_start[c + 1];
  if (cs == ce) {
    // only the cell's own row reads its slots, and a zero centre marks it
    // empty (the other slots keep stale values nobody uses)
    v.ac[(int64_t)(NS / 2) * v.ncell + c] = 0.0;
    return;
  }
  const int64_t b0 = cs / CROWS, b1 = (ce - 1) / CROWS;
  if (b0 == b1) return;  // written whole by its workgroup
  for (int o = 0; o < NS; ++o) {
    double sum = tail[b0 * NS + o];
    for (int64_t b = b0 + 1; b <= b1; ++b) sum += head[b * NS + o];
    v.ac[(int64_t)o * v.ncell + c] = sum;
  }
}

// Gershgorin bound of D_c^-1 A_c per cell row; one maximum per workgroup.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_coarse_bound(View v) {
  constexpr int NS = nsten<DIM>();
  const int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  double g = 0.0;
  if (c < v.ncell) {
    double row[NS];
#pragma unroll
    for (int o = 0; o < NS; ++o) row[o] = v.ac[(int64_t)o * v.ncell + c];
    double sum_abs = 0.0;
#pragma unroll
    for (int o = 0; o < NS; ++o) sum_abs += fabs(row[o]);
    if (row[NS / 2] > 0.0) g = sum_abs / row[NS / 2];
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, WAVE));
  __shared__ double shg[BLOCK / WAVE];
  if ((threadIdx.x & (WAVE - 1)) == 0) shg[threadIdx.x / WAVE] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = shg[0];
    for (int k = 1; k < BLOCK / WAVE; ++k) m = fmax(m, shg[k]);
    v.red_blk[blockIdx.x] = m;
  }
}

// G = the largest of the workgroup maxima (one workgroup).
constexpr int GMAX_NT = 1024;
__global__ __launch_bounds__(GMAX_NT) void k_coarse_gmax(View v, int nblk) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += GMAX_NT) m = fmax(m, v.red_blk[b]);
  for (int o = WAVE / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
  __shared__ double sh[GMAX_NT / WAVE];
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < GMAX_NT / WAVE; ++k) m = fmax(m, sh[k]);
  v.sc->cg_bits = (unsigned long long)__double_as_longlong(m);
}

// Chebyshev constants of [G/10, G]: theta, delta and rho_k.
__device__ inline void cheb_consts(const View& v, double& th, double& de) {
  const double G = __longlong_as_double((long long)v.sc->cg_bits);
  th = 0.55 * G;
  de = 0.45 * G;
}
__device__ inline double cheb_rho(double sig, int k) {
  double rho = 1.0 / sig;
  for (int q = 1; q <= k; ++q) rho = 1.0 / (2.0 * sig - rho);
  return rho;
}

// Restriction and the first Chebyshev step, one team per cell:
// r_c = sum of src over the cell's unknowns, d = D_c^-1 r_c / theta, x = d.
__global__ __launch_bounds__(BLOCK) void k_coarse_start(View v, const double* src, int ns) {
  if (v.sc->converged) return;
  const int64_t cell = (int64_t)xcd_block() * ROWS_PER_BLOCK + threadIdx.x / TEAM;
  const int t = team_lane();
  if (cell >= v.ncell) return;
  const int b0 = v.cell_start[cell], b1 = v.cell_start[cell + 1];
  double sum = 0.0;
  for (int i = b0 + t; i < b1; i += TEAM)
    sum += v.flags[i] == MPS_FLAG_INNER ? src[i] : 0.0;
  sum = team_sum(sum);
  if (t == 0) {
    double th, de;
    cheb_consts(v, th, de);
    const double cen = v.ac[(int64_t)(ns / 2) * v.ncell + cell];
    const double d = cen > 0.0 && th > 0.0 ? sum / (cen * th) : 0.0;
    v.rc[cell] = sum;
    v.dc[0][cell] = d;
    v.xc[cell] = d;
  }
}

// Chebyshev step k >= 1, one thread per cell: r_c -= A_c d_(k-1),
// d_k = rho_k rho_(k-1) d_(k-1) + 2 rho_k / delta D_c^-1 r_c, x += d_k.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_coarse_step(View v, int k) {
  constexpr int NS = nsten<DIM>();
  if (v.sc->converged) return;
  const int64_t cell = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= v.ncell) return;
  const double* __restrict__ dold = v.dc[(k - 1) & 1];
  const double* a = v.ac + cell;  // slot o at a[o * ncell]
  const double cen = a[(int64_t)(NS / 2) * v.ncell];
  if (!(cen > 0.0)) {
    // a cell without unknowns: its direction stays 0
    v.dc[k & 1][cell] = 0.0;
    return;
  }
  const int cx = (int)(cell % v.nx), cy = (int)((cell / v.nx) % v.ny),
            cz = (int)(cell / ((int64_t)v.nx * v.ny));
  // every load first (indices of neighbours outside the grid clamped to the
  // cell itself, their products dropped), then the sum
  double av[NS], dv[NS];
  bool in[NS];
#pragma unroll
  for (int o = 0; o < NS; ++o) {
    const int x = cx + o % 3 - 1, y = cy + (o / 3) % 3 - 1, z = DIM == 3 ? cz + o / 9 - 1 : 0;
    in[o] = x >= 0 && x < v.nx && y >= 0 && y < v.ny && z >= 0 && z < v.nz;
    const int64_t nb = in[o] ? x + (int64_t)v.nx * (y + (int64_t)v.ny * z) : cell;
    av[o] = a[(int64_t)o * v.ncell];
    dv[o] = dold[nb];
  }
  double q = 0.0;
#pragma unroll
  for (int o = 0; o < NS; ++o) q += in[o] ? av[o] * dv[o] : 0.0;
  double th, de;
  cheb_consts(v, th, de);
  const double r = v.rc[cell] - q;
  double d = 0.0;
  if (de > 0.0) {
    const double sig = th / de;
    const double rk = cheb_rho(sig, k), rk1 = cheb_rho(sig, k - 1);
    d = rk * rk1 * dv[NS / 2] + 2.0 * rk / de * (r / cen);
  }
  v.rc[cell] = r;
  v.dc[k & 1][cell] = d;
  v.xc[cell] += d;
}

// Prolongation: target_i += x_c(cell of i) for the unknowns.
__global__ __launch_bounds__(BLOCK) void k_coarse_prolong(View v, double* target) {
  if (v.sc->converged) return;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= v.n || v.flags[i] != MPS_FLAG_INNER) return;
  target[i] += v.xc[cell_lin(v, v.pcell[i])];
}

// Export of the assembled system in original order.
template <class VT>
__global__ __launch_bounds__(BLOCK) void k_export_ppe(View v, double* diag, double* b,
                                                      int32_t* nnz, int32_t* cols,
                                                      double* vals) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= v.n) return;
  const int64_t o = v.id[k];
  const int m = v.a_nnz[k];
  if (diag) diag[o] = v.diag[k];
  if (b) b[o] = v.b[k];
  if (nnz) nnz[o] = m;
  const VT* aval = reinterpret_cast<const VT*>(v.a_val);
  for (int l = 0; l < v.max_neigh; ++l) {
    const bool in = l < m;
    const int64_t e = in ? sl_index(k, l, v.kpad) : 0;
    if (cols) cols[o * v.max_neigh + l] = in ? v.id[v.a_col[e]] : -1;
    if (vals) vals[o * v.max_neigh + l] = in ? (double)aval[e] : 0.0;
  }
}

// Reorder between the caller's original order and the sorted order.
__global__ __launch_bounds__(BLOCK) void k_to_orig(View v, const double* src, double* dst,
                                                   int comps, int stride) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= v.n) return;
  const int64_t o = v.id[k];
  for (int a = 0; a < comps; ++a) dst[o * comps + a] = src[k * stride + a];
}
__global__ __launch_bounds__(BLOCK) void k_from_orig(View v, const double* src, double* dst,
                                                     int comps, int stride) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= v.n) return;
  const int64_t o = v.id[k];
  for (int a = 0; a < comps; ++a) dst[k * stride + a] = src[o * comps + a];
  for (int a = comps; a < stride; ++a) dst[k * stride + a] = 0.0;
}

static inline unsigned nb_team(int64_t n) {
  return (unsigned)((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
}
static inline unsigned nb_flat(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

int cg_spmv_blocks(int64_t n) {
  const int64_t a = nb_team(n);
  return (int)(a < CG_SPMV_BLOCKS ? a : CG_SPMV_BLOCKS);
}
// The pipelined solve reduces the assembly partials once per solve, so the
// assembly takes one 32-row group per workgroup (the hardware balances dense
// and sparse regions); the textbook SpMV re-reduces them in every
// workgroup and keeps the capped grid.
#ifndef ASM_GRID_FULL
#define ASM_GRID_FULL 1
#endif
int assemble_blocks(int64_t n, bool pipelined) {
  return pipelined && ASM_GRID_FULL ? (int)nb_team(n) : cg_spmv_blocks(n);
}
int cg_update_blocks(int64_t n) {
  const int64_t a = nb_flat(n);
  return (int)(a < CG_UPD_BLOCKS ? a : CG_UPD_BLOCKS);
}

template <int DIM>
static void assemble_t(const View& v, bool mx, unsigned nb, const double* rhs, int zx,
                       hipStream_t s) {
  const bool multi = v.rho_s != nullptr;
  if (mx) {
    if (multi) k_assemble<DIM, true, true><<<nb, BLOCK, 0, s>>>(v, rhs, zx);
    else k_assemble<DIM, true, false><<<nb, BLOCK, 0, s>>>(v, rhs, zx);
  } else {
    if (multi) k_assemble<DIM, false, true><<<nb, BLOCK, 0, s>>>(v, rhs, zx);
    else k_assemble<DIM, false, false><<<nb, BLOCK, 0, s>>>(v, rhs, zx);
  }
}

int launch_assemble(const View& v, int dim, int precision, const double* rhs, bool zero_x0,
                    hipStream_t s) {
  const unsigned nb = (unsigned)v.nasmb;
  const int zx = zero_x0 ? 1 : 0;
  const bool mx = precision == MPS_MIXED;
  if (dim == 2) {
    assemble_t<2>(v, mx, nb, rhs, zx, s);
  } else {
    assemble_t<3>(v, mx, nb, rhs, zx, s);
  }
  return 0;
}

int launch_cg_spmv(const View& v, int precision, hipStream_t s) {
  const unsigned nt = (unsigned)v.nspmv;
  if (precision == MPS_MIXED) launch_k(k_cg_spmv<float>, nt, BLOCK, s, v);
  else launch_k(k_cg_spmv<double>, nt, BLOCK, s, v);
  return 0;
}

int pcg_blocks(int64_t n, bool fused) {
  const int rows = (fused ? PCG_BLOCK : PCG_SPLIT_BLOCK) / TEAM;
  return (int)((n + rows - 1) / rows);
}

// Largest grid of the fused iteration kernel: what the device holds
// resident at once (a second wave of workgroups would double the latency of
// an iteration), and at most PCG_MAX_BLOCKS partials per reduction.  The
// workgroups never wait for each other, so this is a matter of speed only.
int pcg_fused_capacity(int precond) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  int worst = 1 << 30;
  const void* ks[2];
  if (precond == MPS_PC_TWO_LEVEL) {
    ks[0] = (const void*)k_pcg_iter<float, 0, true, false, true, false>;
    ks[1] = (const void*)k_pcg_iter<double, 0, true, false, true, false>;
  } else if (precond == MPS_PC_BLOCK) {
    ks[0] = (const void*)k_pcg_iter<float, 0, true, false, true, true>;
    ks[1] = (const void*)k_pcg_iter<double, 0, true, false, true, true>;
  } else {
    ks[0] = (const void*)k_pcg_iter<float, 0, true, false, false, false>;
    ks[1] = (const void*)k_pcg_iter<double, 0, true, false, false, false>;
  }
  for (const void* k : ks) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, PCG_BLOCK, 0) != hipSuccess) return 0;
    worst = per < worst ? per : worst;
  }
  const int cap = worst * cus;
  return cap < PCG_MAX_BLOCKS ? cap : PCG_MAX_BLOCKS;
}

template <bool TWO, bool BJ>
static void pcg_setup_t(const View& v, bool mx, int dim, hipStream_t s) {
  const unsigned nb = (unsigned)v.npcg;
  if (v.pcg_fused) {
    if constexpr (TWO && !BJ) launch_coarse_correct(v, dim, v.r, v.z, s);
    if constexpr (BJ) {
      if (mx) k_bj_start<float><<<nb, PCG_BLOCK, 0, s>>>(v);
      else k_bj_start<double><<<nb, PCG_BLOCK, 0, s>>>(v);
    }
    if (mx) k_pcg_setup<float, true, TWO, BJ><<<nb, PCG_BLOCK, 0, s>>>(v);
    else k_pcg_setup<double, true, TWO, BJ><<<nb, PCG_BLOCK, 0, s>>>(v);
  } else if constexpr (!BJ) {
    k_pcg_start<<<1, RED_BLOCK, 0, s>>>(v);
    if constexpr (TWO) launch_coarse_correct(v, dim, v.r, v.z, s);
    if (mx) k_pcg_setup<float, false, TWO, false><<<nb, PCG_SPLIT_BLOCK, 0, s>>>(v);
    else k_pcg_setup<double, false, TWO, false><<<nb, PCG_SPLIT_BLOCK, 0, s>>>(v);
  }
  if constexpr (TWO && !BJ) launch_coarse_correct(v, dim, v.pl_w, v.pl_m[0], s);
}

int launch_pcg_setup(const View& v, int precision, int dim, hipStream_t s) {
  const bool mx = precision == MPS_MIXED;
  if (v.pc_block) {
    // block Jacobi runs on the fused schedule only (checked at set-up)
    if (!v.pcg_fused) return 1;
    pcg_setup_t<true, true>(v, mx, dim, s);
  } else if (v.ac) {
    pcg_setup_t<true, false>(v, mx, dim, s);
  } else {
    pcg_setup_t<false, false>(v, mx, dim, s);
  }
  return 0;
}

int launch_pcg_reduce(const View& v, int parity, hipStream_t s) {
  const unsigned g = (unsigned)v.npcg2;
  if (parity) launch_k(k_pcg_reduce<1>, g, RED2_BLOCK, s, v);
  else launch_k(k_pcg_reduce<0>, g, RED2_BLOCK, s, v);
  return 0;
}

template <class VT, bool FUSED, bool PRED, bool TWO, bool BJ>
static void pcg_iter_t(const View& v, int parity, hipStream_t s) {
  const unsigned nb = (unsigned)v.npcg;
  const unsigned nt = FUSED ? PCG_BLOCK : PCG_SPLIT_BLOCK;
  launch_k(parity ? k_pcg_iter<VT, 1, FUSED, PRED, TWO, BJ>
                  : k_pcg_iter<VT, 0, FUSED, PRED, TWO, BJ>,
           nb, nt, s, v);
}

template <class VT, bool TWO>
static void pcg_iter_s(const View& v, int parity, hipStream_t s) {
  if (v.pcg_fused) pcg_iter_t<VT, true, false, TWO, false>(v, parity, s);
  else if (v.pcg_pred) pcg_iter_t<VT, false, true, TWO, false>(v, parity, s);
  else pcg_iter_t<VT, false, false, TWO, false>(v, parity, s);
}

int launch_pcg_iter(const View& v, int precision, int parity, hipStream_t s) {
  const bool mx = precision == MPS_MIXED;
  if (v.pc_block) {
    if (!v.pcg_fused) return 1;
    if (mx) pcg_iter_t<float, true, false, true, true>(v, parity, s);
    else pcg_iter_t<double, true, false, true, true>(v, parity, s);
  } else if (v.ac) {
    if (mx) pcg_iter_s<float, true>(v, parity, s);
    else pcg_iter_s<double, true>(v, parity, s);
  } else {
    if (mx) pcg_iter_s<float, false>(v, parity, s);
    else pcg_iter_s<double, false>(v, parity, s);
  }
  return 0;
}

int launch_coarse_assemble(const View& v, int dim, int precision, hipStream_t s) {
  const unsigned nr = (unsigned)((v.n + CROWS - 1) / CROWS);
  const unsigned nc = (unsigned)((v.ncell + BLOCK - 1) / BLOCK);
  const int ns = dim == 3 ? 27 : 9;
  double* head = v.cwork;
  double* tail = v.cwork + (int64_t)nr * ns;
  const bool mx = precision == MPS_MIXED;
  if (dim == 2) {
    if (mx) k_coarse_rows<2, float><<<nr, BLOCK, 0, s>>>(v, head, tail);
    else k_coarse_rows<2, double><<<nr, BLOCK, 0, s>>>(v, head, tail);
    k_coarse_join<2><<<nc, BLOCK, 0, s>>>(v, head, tail);
    k_coarse_bound<2><<<nc, BLOCK, 0, s>>>(v);
  } else {
    if (mx) k_coarse_rows<3, float><<<nr, BLOCK, 0, s>>>(v, head, tail);
    else k_coarse_rows<3, double><<<nr, BLOCK, 0, s>>>(v, head, tail);
    k_coarse_join<3><<<nc, BLOCK, 0, s>>>(v, head, tail);
    k_coarse_bound<3><<<nc, BLOCK, 0, s>>>(v);
  }
  k_coarse_gmax<<<1, GMAX_NT, 0, s>>>(v, (int)nc);
  return 0;
}

int launch_coarse_correct(const View& v, int dim, const double* src, double* target,
                          hipStream_t s) {
  const int ns = dim == 3 ? 27 : 9;
  k_coarse_start<<<(unsigned)((v.ncell + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK), BLOCK, 0, s>>>(
      v, src, ns);
  const unsigned nc = (unsigned)((v.ncell + BLOCK - 1) / BLOCK);
  for (int k = 1; k < CHEB_K; ++k) {
    if (dim == 2) k_coarse_step<2><<<nc, BLOCK, 0, s>>>(v, k);
    else k_coarse_step<3><<<nc, BLOCK, 0, s>>>(v, k);
  }
  k_coarse_prolong<<<nb_flat(v.n), BLOCK, 0, s>>>(v, target);
  return 0;
}

int launch_cg_update(const View& v, hipStream_t s) {
  launch_k(k_cg_update, (unsigned)v.nupd, BLOCK, s, v);
  return 0;
}

int launch_export_ppe(const View& v, int precision, double* diag, double* b, int32_t* nnz,
                      int32_t* cols, double* vals, hipStream_t s) {
  if (precision == MPS_MIXED)
    k_export_ppe<float><<<nb_flat(v.n), BLOCK, 0, s>>>(v, diag, b, nnz, cols, vals);
  else
    k_export_ppe<double><<<nb_flat(v.n), BLOCK, 0, s>>>(v, diag, b, nnz, cols, vals);
  return 0;
}

int launch_scatter_orig(const View& v, const double* src, double* dst, int comps, int stride,
                        hipStream_t s) {
  k_to_orig<<<nb_flat(v.n), BLOCK, 0, s>>>(v, src, dst, comps, stride);
  return 0;
}
int launch_gather_orig(const View& v, const double* src, double* dst, int comps, int stride,
                       hipStream_t s) {
  k_from_orig<<<nb_flat(v.n), BLOCK, 0, s>>>(v, src, dst, comps, stride);
  return 0;
}

}  // namespace mps
