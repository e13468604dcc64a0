// C ABI (include/mps.h) and the step pipeline of the MPS library.
//
// The context keeps the particle state in cell-sorted order on the device
// (double-buffered so the per-step re-sort is a gather) and all per-step
// work arrays, allocated once.  One step enqueues, on the context's stream:
//   bin -> scan -> scatter -> in-cell order -> permute        (a1)
//   neighbour lists                                         (a2)
//   viscous prediction                                      (a3)
//   number density, flags (+ equation of state)             (a4, a7)
//   PPE assembly + CG iterations + clamp   [PPE model]      (a5, a6)
//   pressure gradient + Euler update                        (a8)
// The only host synchronisations are the CG convergence polls (batches of
// iterations, sized from the previous step's count) and one status read at
// the end of each call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mps_internal.h"

using namespace mps;

struct mps_ctx {
  mps_params P;
  int64_t n = 0;
  int dim = 2;
  int ps = 2;          // doubles per stored vector
  int kpad = 0;
  int64_t slots = 0;
  int ncell = 0;
  hipStream_t s = nullptr;
  double n0_n = 0, n0_lap = 0, lam_lap = 0;
  // state buffers: a step reads buffer cur and writes the next one of a ring
  // of NBUF (three, so that a step's input survives while the step after
  // it is already enqueued)
  static constexpr int NBUF = 3;
  int cur = 0;
  // state, double-buffered
  double* pos[NBUF] = {};
  double* vel[NBUF] = {};
  double* pres[NBUF] = {};
  int8_t* type[NBUF] = {};
  int32_t* id[NBUF] = {};
  // per-step
  int32_t* pcell = nullptr;
  float4* posf = nullptr;
  float4* rsf = nullptr;
  double* us = nullptr;
  double* rs = nullptr;
  double* nstar = nullptr;
  double* src = nullptr;  // PPE source from Dn/Dt (source != MPS_SRC_STD)
  int8_t* flags = nullptr;
  int32_t *cellid = nullptr, *slot = nullptr, *cell_count = nullptr, *cell_start = nullptr,
          *cell_local = nullptr, *tile_sum = nullptr, *perm = nullptr;
  int32_t *nb_count = nullptr, *nb_list = nullptr;
  int32_t *nbn_count = nullptr, *nbn_list = nullptr;  // short lists (re_n at r*)
  // lists kept over steps (skin > 0): superset lists, positions at the
  // build, the device record of the decisions
  int32_t *sk_count = nullptr, *sk_list = nullptr;
  double* r_build = nullptr;
  ListState* ls = nullptr;
  double* red_blk = nullptr;   // per-workgroup maxima (list check, coarse bound)
  int kpad_s = 0, cap_s = 0;
  int64_t slots_s = 0;
  int32_t *a_nnz = nullptr, *a_col = nullptr;
  void* a_val = nullptr;
  double *diag = nullptr, *b = nullptr;
  double *r = nullptr, *z = nullptr, *pd[2] = {nullptr, nullptr}, *q = nullptr;
  double* p_save = nullptr;
  // two-phase / turbulence
  bool multi = false;
  double* rho_s[NBUF] = {};
  double* nu_l[NBUF] = {};
  double* rho_o = nullptr;  // <rho> and nu in the caller's order (tape reloads)
  double* nu_o = nullptr;
  double* nut = nullptr;
  double* mu = nullptr;
  double* partA = nullptr;
  double* partB = nullptr;
  // two-level preconditioner: cell operator and cell vectors, u, q, w
  double *ac = nullptr, *rc = nullptr, *xc = nullptr, *dc[2] = {nullptr, nullptr};
  double* cwork = nullptr;
  double *pl_u = nullptr, *pl_q = nullptr, *pl_w = nullptr;
  double *pl_z = nullptr, *pl_s = nullptr, *pl_m[2] = {nullptr, nullptr},
         *pl_part[2] = {nullptr, nullptr}, *pl_part2[2] = {nullptr, nullptr};
  int nspmv = 0, nupd = 0, nasmb = 0, npcg = 0, pcg_fused = 0, pcg_pred = 0, pc_block = 0;
  CGScalars* sc = nullptr;
  int32_t* status = nullptr;
  int32_t* step_count = nullptr;   // steps of a call begun with a clean status
  int64_t* counts = nullptr;   // surface, ghost, list entries, matrix nnz,
                                // short-list entries
  // pinned host mirrors
  CGScalars* h_sc = nullptr;
  int32_t* h_status = nullptr;
  // status word at the end of the whole-step graph from buffer b ([b]) and
  // of a polled step ([NBUF]); [NBUF + 1]: the step counter
  int32_t* h_step_status = nullptr;
  int64_t* h_counts = nullptr;
  // profiling: event pairs around launches of the selected kernel classes
  static constexpr int kPool = 2048;
  uint32_t prof_mask = 0;
  hipEvent_t ev_a[kPool] = {};
  hipEvent_t ev_b[kPool] = {};
  int ev_cls[kPool] = {};
  int nev = 0;
  bool ev_created = false;
  double prof_ms[MPS_KC_COUNT] = {};
  int64_t prof_n[MPS_KC_COUNT] = {};
  // HIP graphs of the step stages, one per parity of the double-buffered
  // state (pre: a1-a5 or a1-a4+a7; cg: CG_BATCH iterations; post: clamp +
  // a8; wc2: two whole weakly-compressible steps)
  static constexpr int CG_BATCH = 4;   // smallest CG graph; also 4x and 16x
  bool graphs_built = false;
  hipGraphExec_t g_pre[NBUF] = {}, g_cg[NBUF][3] = {}, g_post[NBUF] = {}, g_wc2[NBUF] = {};
  // whole PPE steps as one graph each (pre, a fixed number of CG iterations,
  // the CG scalars to the host, post), per buffer parity and iteration
  // count; a few are kept, least recently used replaced
  struct StepGraph {
    int ncg = 0;
    uint64_t used = 0;
    hipGraphExec_t g = nullptr;
  };
  static constexpr int kStepGraphs = 12;
  StepGraph g_step[NBUF][kStepGraphs];
  hipEvent_t ev_step[NBUF] = {};  // end of the whole-step graph from buffer b
  bool ev_step_created = false;
  uint64_t step_clock = 0;
  // checkpoint tape: per slot the sorted state (pos, vel, p, type, id)
  struct Slot {
    double *pos = nullptr, *vel = nullptr, *p = nullptr;
    int8_t* type = nullptr;
    int32_t* id = nullptr;
    bool valid = false;
  };
  Slot* tape = nullptr;
  int ntape = 0;
  // adjoint work arrays (allocated with the tape)
  AdjView adj = {};
  double* h_part = nullptr;
  // bookkeeping
  int64_t bytes = 0;       // device memory held by the context (state, work)
  int64_t tape_bytes = 0;  // device memory of the tape and adjoint arrays
  bool poisoned = false;
  bool ppe_valid = false;
  int last_iters = 0;
  // margin of the speculative CG count (spec_ncg)
  static constexpr int CG_MARGIN_MIN = 3, CG_MARGIN_MAX = 9;
  int cg_margin = CG_MARGIN_MIN;
  int cg_quiet = 0;    // accepted speculative steps since the last change
  int32_t steps_ok = 0;    // steps of the running mps_step call completed
  char err[256] = {0};
};

namespace {

mps_status fail(mps_ctx* c, mps_status st, const char* msg) {
  if (c) std::snprintf(c->err, sizeof(c->err), "%s", msg);
  return st;
}

mps_status hip_fail(mps_ctx* c, hipError_t e, const char* where) {
  if (c) std::snprintf(c->err, sizeof(c->err), "%s: %s", where, hipGetErrorString(e));
  return MPS_E_DEVICE;
}

#define HIPCHK(c, expr)                                 \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
  } while (0)

// Lattice constants of an interior particle of the square/cubic lattice of
// spacing l0: n0 = sum w (Eq. 5) and lambda = sum r^2 w / sum w (the weighted
// mean of r^2 of Eq. 7).
void lattice(int dim, double l0, double re, int kernel, double* n0, double* lam) {
  const int m = (int)std::ceil(re / l0) + 1;
  double sw = 0.0, s2 = 0.0;
  const int kz = dim == 3 ? m : 0;
  for (int k = -kz; k <= kz; ++k)
    for (int jy = -m; jy <= m; ++jy)
      for (int ix = -m; ix <= m; ++ix) {
        if (ix == 0 && jy == 0 && k == 0) continue;
        const double x = ix * l0, y = jy * l0, z = k * l0;
        double r2 = x * x + y * y;
        if (dim == 3) r2 = r2 + z * z;
        if (!(r2 < re * re)) continue;
        const double r = std::sqrt(r2);
        const double w = kernel == MPS_K_KOSHIZUKA ? re / r - 1.0
                                                   : (1.0 - r / re) * (1.0 - r / re) * (1.0 - r / re);
        sw += w;
        s2 += r2 * w;
      }
  *n0 = sw;
  *lam = s2 / sw;
}

// Device allocations of all contexts go through here; the running total of
// each context is kept by the callers (mps_ctx::bytes).
thread_local int64_t* g_bytes = nullptr;
template <class T>
hipError_t dalloc(T** p, size_t count) {
  const size_t b = count * sizeof(T) + 256;
  hipError_t e = hipMalloc((void**)p, b);
  if (e == hipSuccess && g_bytes) *g_bytes += (int64_t)b;
  return e;
}

// Doubles in each partial buffer of the pipelined CG: four per workgroup
// (split schedule) or three arrays of PCG_PSTRIDE (fused).
inline size_t pl_part_len(const mps_ctx* c) {
  return std::max((size_t)c->npcg * 4, (size_t)3 * PCG_PSTRIDE);
}

// The buffer a step from buffer cur writes.
inline int nxt(const mps_ctx* c) { return (c->cur + 1) % mps_ctx::NBUF; }

View make_view(const mps_ctx* c) {
  View v;
  std::memset(&v, 0, sizeof(v));
  const mps_params& P = c->P;
  v.n = c->n;
  v.kpad = c->kpad;
  v.max_neigh = P.max_neigh;
  v.nx = P.grid_n[0];
  v.ny = P.grid_n[1];
  v.nz = c->dim == 3 ? P.grid_n[2] : 1;
  v.ncell = c->ncell;
  for (int a = 0; a < 3; ++a) {
    v.lo[a] = a < c->dim ? P.grid_lo[a] : 0.0;
    v.g[a] = a < c->dim ? P.g[a] : 0.0;
  }
  v.cs = P.cell_size;
  v.inv_cs = 1.0 / P.cell_size;
  v.cs32 = (float)P.cell_size;
  v.re_n = P.re_n;
  v.re_lap = P.re_lap;
  v.re_n2 = P.re_n * P.re_n;
  v.re_lap2 = P.re_lap * P.re_lap;
  v.re_n_f = (float)P.re_n;
  v.re_lap_f = (float)P.re_lap;
  v.n0_n = c->n0_n;
  v.n0_lap = c->n0_lap;
  v.lam_lap = c->lam_lap;
  v.nu = P.nu;
  v.rho = P.rho;
  v.dt = P.dt;
  v.beta = P.beta;
  v.c0 = P.c0;
  v.alpha = P.alpha;
  v.cg_tol2 = P.cg_tol * P.cg_tol;
  v.gamma_i = (int)P.gamma;
  v.kernel = P.kernel;
  v.grad = P.grad;
  v.clamp = P.clamp_negative_p;
  const int a = c->cur, o = nxt(c);
  v.pos = c->pos[a];
  v.pos_w = c->pos[o];
  v.vel = c->vel[a];
  v.vel_w = c->vel[o];
  v.type = c->type[a];
  v.type_w = c->type[o];
  v.id = c->id[a];
  v.id_w = c->id[o];
  v.p_in = c->pres[a];
  v.p_w = c->pres[o];
  v.pcell = c->pcell;
  v.posf = c->posf;
  v.rsf = c->rsf;
  v.us = c->us;
  v.rs = c->rs;
  v.nstar = c->nstar;
  v.src = c->src;
  v.source = P.source;
  v.laplacian = P.laplacian;
  if (P.skin > 0.0) {
    v.ls = c->ls;
    v.half_skin2 = 0.25 * P.skin * P.skin;
    v.re_s2 = (P.re_lap + P.skin) * (P.re_lap + P.skin);
    v.kpad_s = c->kpad_s;
    v.cap_s = c->cap_s;
    v.sk_list = c->sk_list;
    v.sk_count = c->sk_count;
    v.r_build = c->r_build;
  }
  v.red_blk = c->red_blk;
  v.flags = c->flags;
  v.cellid = c->cellid;
  v.slot = c->slot;
  v.cell_count = c->cell_count;
  v.cell_local = c->cell_local;
  v.tile_sum = c->tile_sum;
  v.ntile = scan_tiles(c->ncell);
  v.cell_start = c->cell_start;
  v.perm = c->perm;
  v.nb_count = c->nb_count;
  v.nb_list = c->nb_list;
  v.nbn_count = c->nbn_count;
  v.nbn_list = c->nbn_list;
  v.re_n2_keep = v.re_n2 * (1.0 + 1e-4);
  v.a_nnz = c->a_nnz;
  v.a_col = c->a_col;
  v.a_val = c->a_val;
  v.diag = c->diag;
  v.b = c->b;
  v.p = c->pres[a];
  v.r = c->r;
  v.z = c->z;
  v.pd[0] = c->pd[0];
  v.pd[1] = c->pd[1];
  v.q = c->q;
  v.partA = c->partA;
  v.partB = c->partB;
  v.pl_z = c->pl_z;
  v.pl_s = c->pl_s;
  v.pl_m[0] = c->pl_m[0];
  v.pl_m[1] = c->pl_m[1];
  v.pl_part[0] = c->pl_part[0];
  v.pl_part[1] = c->pl_part[1];
  v.pl_part2[0] = c->pl_part2[0];
  v.pl_part2[1] = c->pl_part2[1];
  v.npcg2 = std::min(c->npcg, PCG_SPLIT_G);
  v.ac = c->ac;
  v.cwork = c->cwork;
  v.rc = c->rc;
  v.xc = c->xc;
  v.dc[0] = c->dc[0];
  v.dc[1] = c->dc[1];
  v.pl_u = c->pl_u;
  v.pl_q = c->pl_q;
  v.pl_w = c->pl_w;
  v.nspmv = c->nspmv;
  v.nasmb = c->nasmb;
  v.nupd = c->nupd;
  v.npcg = c->npcg;
  v.pcg_fused = c->pcg_fused;
  v.pcg_pred = c->pcg_pred;
  v.pc_block = c->pc_block;
  v.sc = c->sc;
  v.status = c->status;
  if (c->multi) {
    v.rho_s = c->rho_s[a];
    v.rho_s_w = c->rho_s[o];
    v.nu_l = c->nu_l[a];
    v.nu_l_w = c->nu_l[o];
    v.nut = c->nut;
    v.mu = c->mu;
    v.smag_c2 = (P.smagorinsky_cs * P.l0) * (P.smagorinsky_cs * P.l0);
  }
  return v;
}

// In-place variant: the gradient kernel writes the current buffers.
View make_view_inplace(const mps_ctx* c) {
  View v = make_view(c);
  v.pos_w = c->pos[c->cur];
  v.vel_w = c->vel[c->cur];
  return v;
}

}  // namespace

namespace mps {
mps_status check_params(const mps_params* P, int64_t n) {
  if (!P || n < 1 || n > (int64_t)INT32_MAX / 2) return MPS_E_ARG;
  if (P->dim != 2 && P->dim != 3) return MPS_E_ARG;
  if (!(P->l0 > 0) || !(P->re_n > 0) || !(P->re_lap > 0)) return MPS_E_ARG;
  if (!(P->cell_size >= P->re_lap) || !(P->cell_size >= P->re_n)) return MPS_E_ARG;
  if (!(P->dt > 0) || !(P->rho > 0) || !(P->nu >= 0)) return MPS_E_ARG;
  if (P->max_neigh < 1 || P->max_neigh > 1024) return MPS_E_ARG;
  if (P->pmode != MPS_PPE_CG && P->pmode != MPS_WC_EOS) return MPS_E_ARG;
  if (P->kernel != MPS_K_KOSHIZUKA && P->kernel != MPS_K_CUBIC) return MPS_E_ARG;
  if (P->precision != MPS_FP64 && P->precision != MPS_MIXED) return MPS_E_ARG;
  if (P->grad != MPS_GRAD_STD && P->grad != MPS_GRAD_CMPS) return MPS_E_ARG;
  if (P->gamma < 1 || P->gamma > 16 || P->gamma != std::floor(P->gamma)) return MPS_E_ARG;
  if (P->cg_maxit < 1 || !(P->cg_tol > 0)) return MPS_E_ARG;
  if (P->cg_pipelined != 0 && P->cg_pipelined != 1) return MPS_E_ARG;
  if (!(P->smagorinsky_cs >= 0.0) || P->smagorinsky_cs > 1.0) return MPS_E_ARG;
  if (P->source < MPS_SRC_STD || P->source > MPS_SRC_HS_ECS) return MPS_E_ARG;
  if (P->source != MPS_SRC_STD && P->pmode != MPS_PPE_CG) return MPS_E_ARG;
  if (P->laplacian != MPS_LAP_STD && P->laplacian != MPS_LAP_HL) return MPS_E_ARG;
  if (P->laplacian != MPS_LAP_STD && P->pmode != MPS_PPE_CG) return MPS_E_ARG;
  if (!(P->skin >= 0.0) || !(P->skin < P->re_lap)) return MPS_E_ARG;
  if (P->precond != MPS_PC_JACOBI && P->precond != MPS_PC_TWO_LEVEL &&
      P->precond != MPS_PC_BLOCK)
    return MPS_E_ARG;
  if (P->precond != MPS_PC_JACOBI && (P->cg_pipelined != 1 || P->pmode != MPS_PPE_CG))
    return MPS_E_ARG;
  if (P->skin > 0.0 && !(P->cell_size >= P->re_lap + P->skin)) return MPS_E_ARG;
  int64_t nc = 1;
  for (int a = 0; a < P->dim; ++a) {
    if (P->grid_n[a] < 1 || P->grid_n[a] > 1023) return MPS_E_ARG;
    nc *= P->grid_n[a];
  }
  if (nc > (int64_t)1 << 28) return MPS_E_ARG;
  return MPS_OK;
}
}  // namespace mps

namespace {

// Element type scatter/gather for int8 state.
__global__ void k_i8_to_orig(int64_t n, const int32_t* id, const int8_t* src, int8_t* dst) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) dst[id[k]] = src[k];
}
__global__ void k_i8_from_orig(int64_t n, const int32_t* id, const int8_t* src, int8_t* dst) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) dst[k] = src[id[k]];
}
__global__ void k_fill(int64_t n, double* a, double x) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) a[k] = x;
}
__global__ void k_iota(int64_t n, int32_t* id) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) id[k] = (int32_t)k;
}
// Input types are FLUID/WALL/DUMMY; anything else is rejected by a status bit.
__global__ void k_check_types(int64_t n, const int8_t* t, int32_t* status) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n && (t[k] < MPS_FLUID || t[k] > MPS_GHOST)) atomicOr(status, ST_BADTYPE);
}
constexpr int NCOUNTS = 5;
__global__ __launch_bounds__(256) void k_count_flags(int64_t n, const int8_t* flags,
                                                     const int32_t* nb_count,
                                                     const int32_t* nbn_count,
                                                     const int32_t* a_nnz, int ppe,
                                                     int64_t* counts) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long c[NCOUNTS] = {0, 0, 0, 0, 0};
  if (k < n) {
    const int8_t f = flags[k];
    c[0] = f == MPS_FLAG_SURFACE;
    c[1] = f == MPS_FLAG_GHOST;
    c[2] = (unsigned long long)nb_count[k];
    c[3] = ppe ? (unsigned long long)a_nnz[k] : 0ull;
    c[4] = (unsigned long long)nbn_count[k];
  }
  __shared__ unsigned long long sh[NCOUNTS][4];
#pragma unroll
  for (int q = 0; q < NCOUNTS; ++q) {
    for (int o = 32; o > 0; o >>= 1) c[q] += __shfl_down(c[q], o, 64);
    if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x / 64] = c[q];
  }
  __syncthreads();
  // integer atomics, one per workgroup: the totals do not depend on the order
  if (threadIdx.x < NCOUNTS) {
    const unsigned long long t = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] +
                                 sh[threadIdx.x][3];
    if (t) atomicAdd((unsigned long long*)&counts[threadIdx.x], t);
  }
}

unsigned flat_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

void prof_flush(mps_ctx* c);

// The error of a raised status word st (!= 0): the device word is cleared
// and the context poisoned.
mps_status status_error(mps_ctx* c, int32_t st) {
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(int32_t), c->s));
  c->poisoned = true;
  if (st & ST_OVERFLOW) return fail(c, MPS_E_NEIGH_OVERFLOW, "more than max_neigh neighbours");
  if (st & ST_COINCIDENT) return fail(c, MPS_E_COINCIDENT, "two particles at distance 0");
  if (st & ST_NONFINITE) return fail(c, MPS_E_NONFINITE, "non-finite position or velocity");
  return fail(c, MPS_E_ARG, "invalid particle type");
}

mps_status read_status(mps_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  prof_flush(c);
  const int32_t st = *c->h_status;
  if (st == 0) return MPS_OK;
  return status_error(c, st);
}

// Counts a step begun with a clean status word and, for a whole-step graph,
// keeps a copy of that word from before the step (one thread).
__global__ void k_step_begin(const int32_t* status, int32_t* count, int32_t* snap) {
  if (threadIdx.x == 0) {
    const int32_t st = *status;
    if (snap) *snap = st;
    if (st == 0) *count += 1;
  }
}

// End of a whole-step graph: the CG scalars and the status word into their
// pinned host copies, which the host reads once the step's event has
// completed (one wavefront, a word per lane; one kernel instead of two
// copies in the graph).
__global__ void k_step_end(const CGScalars* sc, const int32_t* status, CGScalars* h_sc,
                           int32_t* h_status) {
  constexpr int NW = (int)(sizeof(CGScalars) / sizeof(int32_t));
  static_assert(sizeof(CGScalars) % sizeof(int32_t) == 0 && NW <= 64, "a word per lane");
  const int i = threadIdx.x;
  if (i < NW) reinterpret_cast<int32_t*>(h_sc)[i] = reinterpret_cast<const int32_t*>(sc)[i];
  if (i == 0) *h_status = *status;
}

// Accumulate the recorded event pairs (the stream must be synchronised).
void prof_flush(mps_ctx* c) {
  for (int k = 0; k < c->nev; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_a[k], c->ev_b[k]) == hipSuccess) {
      c->prof_ms[c->ev_cls[k]] += ms;
      c->prof_n[c->ev_cls[k]] += 1;
    }
  }
  c->nev = 0;
}

}  // namespace

namespace mps {
thread_local ExtTiming* g_ext_timing = nullptr;
}

namespace {

// Bracket a group of launches of one kernel class with events.  With
// single = true the scope holds exactly one launch made through launch_k,
// which records the events from its own dispatch (kernel execution only).
struct Prof {
  mps_ctx* c;
  int cls;
  bool on;
  bool single;
  ExtTiming et;
  Prof(mps_ctx* c_, int cls_, bool single_ = false)
      : c(c_), cls(cls_), on((c_->prof_mask >> cls_) & 1u), single(single_) {
    if (!on) return;
    if (c->nev == mps_ctx::kPool) {
      (void)hipStreamSynchronize(c->s);
      prof_flush(c);
    }
    if (single) {
      et.start = c->ev_a[c->nev];
      et.stop = c->ev_b[c->nev];
      g_ext_timing = &et;
    } else {
      (void)hipEventRecord(c->ev_a[c->nev], c->s);
    }
  }
  ~Prof() {
    if (!on) return;
    if (single) {
      g_ext_timing = nullptr;
      if (!et.used) return;  // nothing was launched
    } else {
      (void)hipEventRecord(c->ev_b[c->nev], c->s);
    }
    c->ev_cls[c->nev] = cls;
    c->nev += 1;
  }
};

// a1 + a2 at the current state; leaves the context in the new sorted order.
// With a skin the step first decides on the device whether to build: if so
// the cell sort and a search at radius re_lap + skin write the superset
// lists, if not the state is copied in its order; then the superset is
// filtered to the exact lists at the step's positions.
// fold: the caller's prediction filters kept lists (single phase), so the
// separate filter is not launched.
mps_status search(mps_ctx* c, bool fold = false) {
  c->ppe_valid = false;
  const bool keep = c->P.skin > 0.0;
  View v = make_view(c);
  if (keep) {
    Prof pr(c, MPS_KC_NEIGH);
    launch_list_check(v, c->dim, c->s);
  }
  {
    Prof pr(c, MPS_KC_SORT);
    launch_bin(v, c->dim, c->s);
    launch_permute(v, c->dim, c->P.precision, c->s);
  }
  c->cur = nxt(c);
  v = make_view(c);
  {
    Prof pr(c, MPS_KC_NEIGH);
    if (keep) {
      View vs = v;
      vs.nb_list = c->sk_list;
      vs.nb_count = c->sk_count;
      vs.kpad = c->kpad_s;
      vs.max_neigh = c->cap_s;
      vs.re_lap2 = vs.re_s2;
      launch_neighbors(vs, c->dim, c->P.precision, c->s);
      if (!fold) launch_list_filter(v, c->dim, c->s);
    } else {
      launch_neighbors(v, c->dim, c->P.precision, c->s);
    }
  }
  return MPS_OK;
}

// The next step builds its lists afresh (the state or its order changed
// other than by a step).
void force_build(mps_ctx* c) {
  if (c->ls) launch_list_force(make_view(c), c->s);
}

// --------------------------------------------------------------- stages
// PPE assembly and the start of the CG (pipelined: its setup SpMV).
void enqueue_assemble(mps_ctx* c, const View& v, const double* rhs, bool zero_x0) {
  {
    Prof pr(c, MPS_KC_ASSEMBLE);
    launch_assemble(v, c->dim, c->P.precision, rhs, zero_x0, c->s);
  }
  if (c->P.cg_pipelined) {
    // the CG start (w0 = A u0 and its dot products; two-level: the cell
    // operator and the coarse corrections of r0 and w0) is timed with the
    // assembly
    Prof pr(c, MPS_KC_ASSEMBLE);
    if (c->ac) launch_coarse_assemble(v, c->dim, c->P.precision, c->s);
    launch_pcg_setup(v, c->P.precision, c->dim, c->s);
  }
}

// Stages before the pressure solve: a1-a5 (PPE) or a1-a4 + a7 (EOS).
// Leaves the context in the new sorted order (flips cur).
void enqueue_pre(mps_ctx* c, int32_t* status_snap = nullptr) {
  k_step_begin<<<1, 64, 0, c->s>>>(c->status, c->step_count, status_snap);
  // kept lists, single phase: the prediction filters the superset
  const bool fold = c->P.skin > 0.0 && !c->multi;
  search(c, fold);
  View v = make_view(c);
  if (c->multi) {
    Prof pr(c, MPS_KC_PREDICT);
    launch_viscosity(v, c->dim, c->P.precision, c->s);
  }
  {
    Prof pr(c, MPS_KC_PREDICT);
    launch_predict(v, c->dim, c->P.precision, fold, c->s);
  }
  {
    Prof pr(c, MPS_KC_DENSITY);
    launch_density(v, c->dim, c->P.precision, c->P.pmode, c->s);
  }
  if (c->P.pmode == MPS_PPE_CG) enqueue_assemble(c, v, nullptr, false);
}

// CG iterations; the pipelined variant alternates buffer parities, and
// every batch has an even length so each starts at parity 0.
void enqueue_cg(mps_ctx* c, int iters) {
  View v = make_view(c);
  if (c->P.cg_pipelined) {
    for (int it = 0; it < iters; ++it) {
      if (!c->pcg_fused) {
        Prof pr(c, MPS_KC_CG_UPDATE, true);
        launch_pcg_reduce(v, it & 1, c->s);
      }
      {
        Prof pr(c, MPS_KC_CG_SPMV, true);
        launch_pcg_iter(v, c->P.precision, it & 1, c->s);
      }
      if (c->ac) {
        // two-level: the coarse part of m = M^-1 w for the next iteration
        Prof pr(c, MPS_KC_CG_UPDATE);
        launch_coarse_correct(v, c->dim, c->pl_w, c->pl_m[(it & 1) ^ 1], c->s);
      }
    }
    return;
  }
  for (int it = 0; it < iters; ++it) {
    {
      Prof pr(c, MPS_KC_CG_SPMV, true);
      launch_cg_spmv(v, c->P.precision, c->s);
    }
    Prof pr(c, MPS_KC_CG_UPDATE, true);
    launch_cg_update(v, c->s);
  }
}

// Stages after the pressure: a8 (the gradient kernels clamp negative
// pressure on read and write it back clamped).
void enqueue_post(mps_ctx* c) {
  Prof pr(c, MPS_KC_GRADIENT);
  launch_gradient(make_view_inplace(c), c->dim, c->P.precision, c->s);
}

template <class F>
mps_status capture(mps_ctx* c, hipGraphExec_t* out, F&& body) {
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
  body();
  HIPCHK(c, hipStreamEndCapture(c->s, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  return MPS_OK;
}

// Graphs are used on a non-default stream with profiling off (event timing
// needs the direct launches).
bool use_graphs(const mps_ctx* c) { return c->s != nullptr && c->prof_mask == 0; }

mps_status build_graphs(mps_ctx* c) {
  if (c->graphs_built) return MPS_OK;
  const int cur0 = c->cur;
  for (int par = 0; par < mps_ctx::NBUF; ++par) {
    c->cur = par;
    mps_status st = capture(c, &c->g_pre[par], [&] { enqueue_pre(c); });
    if (st != MPS_OK) return st;
    c->cur = par;
    st = capture(c, &c->g_post[par], [&] { enqueue_post(c); });
    if (st != MPS_OK) return st;
    if (c->P.pmode == MPS_PPE_CG) {
      for (int q = 0; q < 3 && st == MPS_OK; ++q)
        st = capture(c, &c->g_cg[par][q], [&] { enqueue_cg(c, mps_ctx::CG_BATCH << (2 * q)); });
    } else {
      st = capture(c, &c->g_wc2[par], [&] {
        enqueue_pre(c);
        enqueue_post(c);
        enqueue_pre(c);
        enqueue_post(c);
      });
    }
    if (st != MPS_OK) return st;
  }
  c->cur = cur0;
  c->graphs_built = true;
  return MPS_OK;
}

// CG from the state left by the assembly.  Iterations are enqueued in
// batches (graphs of CG_BATCH iterations when available) sized from the
// previous step's count, then the device scalars are polled.
mps_status solve(mps_ctx* c, int* iters, double* relres, bool graphs) {
  int launched = 0;
  const int maxit = c->P.cg_maxit;
  const int B = mps_ctx::CG_BATCH;
  int batch = c->last_iters > 0 ? c->last_iters + 1 : 16;
  for (;;) {
    int k = std::min(batch, maxit - launched);
    if (k > 0) {
      if (graphs) {
        // greedy cover of k iterations by graphs of 64, 16 and 4 iterations:
        // few host launches (hipGraphLaunch dominates the host cost)
        int left = ((k + B - 1) / B) * B, done = 0;
        for (int q = 2; q >= 0; --q) {
          const int size = B << (2 * q);
          while (left >= size) {
            HIPCHK(c, hipGraphLaunch(c->g_cg[c->cur][q], c->s));
            left -= size;
            done += size;
          }
        }
        k = done;
      } else {
        k += k & 1;
        enqueue_cg(c, k);
      }
      launched += k;
    }
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->sc, sizeof(CGScalars), hipMemcpyDeviceToHost, c->s));
    HIPCHK(c, hipStreamSynchronize(c->s));
    prof_flush(c);
    if (c->h_sc->converged || launched >= maxit) break;
    batch = std::max(B, c->h_sc->iter / 8);
  }
  const CGScalars h = *c->h_sc;
  *iters = h.converged ? h.iter : std::min(launched, maxit);
  *relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  if (!h.converged) return fail(c, MPS_E_CG_NOCONV, "CG reached cg_maxit");
  return MPS_OK;
}

// nsteps steps of the weakly-compressible model: no host synchronisation.
mps_status steps_wc(mps_ctx* c, int nsteps) {
  const bool graphs = use_graphs(c);
  if (graphs) {
    mps_status st = build_graphs(c);
    if (st != MPS_OK) return st;
  }
  int k = 0;
  if (graphs) {
    for (; k + 2 <= nsteps; k += 2) {
      HIPCHK(c, hipGraphLaunch(c->g_wc2[c->cur], c->s));
      c->cur = (c->cur + 2) % mps_ctx::NBUF;
    }
  }
  for (; k < nsteps; ++k) {
    if (graphs) {
      HIPCHK(c, hipGraphLaunch(c->g_pre[c->cur], c->s));
      c->cur = nxt(c);
      HIPCHK(c, hipGraphLaunch(c->g_post[c->cur], c->s));
    } else {
      enqueue_pre(c);
      enqueue_post(c);
    }
  }
  return MPS_OK;
}

// The graph of a whole PPE step from buffer parity par with ncg CG
// iterations (built on first use).
mps_status step_graph(mps_ctx* c, int par, int ncg, hipGraphExec_t* out) {
  mps_ctx::StepGraph* slot = nullptr;
  for (auto& sg : c->g_step[par]) {
    if (sg.g && sg.ncg == ncg) {
      sg.used = ++c->step_clock;
      *out = sg.g;
      return MPS_OK;
    }
    if (!slot || !sg.g || (slot->g && sg.used < slot->used)) slot = &sg;
  }
  if (slot->g) (void)hipGraphExecDestroy(slot->g);
  slot->g = nullptr;
  const int cur0 = c->cur;
  c->cur = par;
  mps_status st = capture(c, &slot->g, [&] {
    enqueue_pre(c, c->status + 1 + par);
    enqueue_cg(c, ncg);
    enqueue_post(c);
    k_step_end<<<1, 64, 0, c->s>>>(c->sc, c->status, c->h_sc + 1 + par, c->h_step_status + par);
  });
  c->cur = cur0;
  if (st != MPS_OK) {
    slot->g = nullptr;
    return st;
  }
  slot->ncg = ncg;
  slot->used = ++c->step_clock;
  *out = slot->g;
  return MPS_OK;
}

void record_cg(mps_ctx* c, mps_step_stats* st, int it, double rel) {
  c->last_iters = it;
  c->steps_ok += 1;
  if (st) {
    st->cg_iters_last = it;
    st->cg_iters_total += it;
    st->cg_relres_last = rel;
  }
}

// A step that raised the status word st: wait for everything enqueued
// (a step enqueued behind it writes no state, see k_rank_permute), go back
// to its input buffer b and report the error.
mps_status fail_step(mps_ctx* c, int b, int32_t st) {
  HIPCHK(c, hipStreamSynchronize(c->s));
  c->cur = b;
  return status_error(c, st);
}

mps_status one_step_polled(mps_ctx* c, mps_step_stats* st) {
  const int b_in = c->cur;
  const bool graphs = use_graphs(c);
  if (graphs) {
    mps_status s0 = build_graphs(c);
    if (s0 != MPS_OK) return s0;
    HIPCHK(c, hipGraphLaunch(c->g_pre[c->cur], c->s));
    c->cur = nxt(c);
    c->ppe_valid = true;
  } else {
    enqueue_pre(c);
  }
  c->ppe_valid = true;
  int it = 0;
  double rel = 0;
  mps_status res = solve(c, &it, &rel, graphs);
  if (res != MPS_OK && res != MPS_E_CG_NOCONV) return res;
  if (graphs) HIPCHK(c, hipGraphLaunch(c->g_post[c->cur], c->s));
  else enqueue_post(c);
  // the step's own status, before the next step is enqueued
  int32_t* hs = c->h_step_status + mps_ctx::NBUF;
  HIPCHK(c, hipMemcpyAsync(hs, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  prof_flush(c);
  if (*hs) return fail_step(c, b_in, *hs);
  record_cg(c, st, it, rel);
  return res;
}

// CG iterations of a speculative whole step: the last accepted step's
// count plus a margin, rounded up to even (launches after convergence
// return at once; a step that needs more is redone, which costs about two
// steps).  The margin starts at 3, grows by 3 (to at most 9) at every redo
// and shrinks by 1 after 50 accepted steps without one.  With two steps in
// flight the count comes from two steps back; on the 2-D dam break it
// rises by at most 3 over two steps with the kernel Laplacian, by more
// with the Eq. 23 Laplacian (one redo in 240 steps under this rule,
// against 5 with a fixed margin of 3).
int spec_ncg(const mps_ctx* c) {
  const int B = 2;
  return std::min(((c->last_iters + c->cg_margin + B - 1) / B) * B,
                  ((c->P.cg_maxit + B - 1) / B) * B);
}

void margin_after(mps_ctx* c, bool redone) {
  if (redone) {
    c->cg_margin = std::min(mps_ctx::CG_MARGIN_MAX, c->cg_margin + 3);
    c->cg_quiet = 0;
  } else if (++c->cg_quiet >= 50 && c->cg_margin > mps_ctx::CG_MARGIN_MIN) {
    c->cg_margin -= 1;
    c->cg_quiet = 0;
  }
}

// Spin on an event (the host's next decision waits for it: a blocking
// wait wakes up later).
mps_status spin_wait(mps_ctx* c, hipEvent_t ev) {
  hipError_t q;
  while ((q = hipEventQuery(ev)) == hipErrorNotReady) {
  }
  if (q != hipSuccess) return hip_fail(c, q, "hipEventQuery");
  return MPS_OK;
}

mps_status launch_step_graph(mps_ctx* c, int b, int ncg) {
  hipGraphExec_t g = nullptr;
  mps_status s0 = step_graph(c, b, ncg, &g);
  if (s0 != MPS_OK) return s0;
  if (!c->ev_step_created) {
    for (int k = 0; k < mps_ctx::NBUF; ++k)
      HIPCHK(c, hipEventCreateWithFlags(&c->ev_step[k], hipEventDisableTiming));
    c->ev_step_created = true;
  }
  HIPCHK(c, hipGraphLaunch(g, c->s));
  HIPCHK(c, hipEventRecord(c->ev_step[b], c->s));
  return MPS_OK;
}

// A step whose whole-step graph did not converge: wait for everything
// enqueued, restore the error flags from before it, and take it again
// from its input buffer b (untouched: the buffers after it are the only
// ones written since) with polled CG batches.
mps_status redo_step(mps_ctx* c, int b, mps_step_stats* st) {
  HIPCHK(c, hipStreamSynchronize(c->s));
  HIPCHK(c, hipMemcpyAsync(c->status, c->status + 1 + b, sizeof(int32_t),
                           hipMemcpyDeviceToDevice, c->s));
  c->cur = b;
  // the discarded steps may have rebuilt the lists in another order
  force_build(c);
  margin_after(c, true);
  if (st) st->cg_redone += 1;
  return one_step_polled(c, st);
}

// Accepts step results from the CG scalars and the status word the
// whole-step graph from buffer b left in pinned memory: 1 accepted, 0 the
// solve did not converge in it, -1 the step raised an error.
int accept_step(mps_ctx* c, int b, mps_step_stats* st) {
  if (c->h_step_status[b]) return -1;
  const CGScalars h = c->h_sc[1 + b];
  if (!h.converged) return 0;
  c->cur = (b + 1) % mps_ctx::NBUF;
  c->ppe_valid = true;
  record_cg(c, st, h.iter, h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0);
  margin_after(c, false);
  return 1;
}

mps_status one_step_ppe(mps_ctx* c, mps_step_stats* st) {
  if (use_graphs(c) && c->last_iters > 0) {
    // speculative whole step; if the solve did not converge within it, the
    // step is discarded and redone with polled batches
    const int b = c->cur;
    mps_status s0 = launch_step_graph(c, b, spec_ncg(c));
    if (s0 != MPS_OK) return s0;
    s0 = spin_wait(c, c->ev_step[b]);
    if (s0 != MPS_OK) return s0;
    const int a = accept_step(c, b, st);
    if (a > 0) return MPS_OK;
    if (a < 0) return fail_step(c, b, c->h_step_status[b]);
    return redo_step(c, b, st);
  }
  return one_step_polled(c, st);
}

// nsteps PPE steps with up to two whole-step graphs in flight: step k + 1
// is enqueued before step k's CG result is read, so the device never waits
// for the host between steps; the three-buffer ring keeps step k's input
// until then.  A step found unconverged is redone from its input and the
// step after it, already run, discarded.
mps_status steps_ppe(mps_ctx* c, int nsteps, mps_step_stats* st) {
  mps_status res = MPS_OK;
  int k = 0;
  while (k < nsteps) {
    if (!use_graphs(c) || c->last_iters == 0 || nsteps - k == 1) {
      mps_status r = one_step_ppe(c, st);
      if (r == MPS_E_CG_NOCONV) res = r;
      else if (r != MPS_OK) return r;
      ++k;
      continue;
    }
    int b = c->cur, inflight = 1;
    mps_status r = launch_step_graph(c, b, spec_ncg(c));
    if (r != MPS_OK) return r;
    for (;;) {
      if (inflight == 1 && k + 1 < nsteps) {
        r = launch_step_graph(c, (b + 1) % mps_ctx::NBUF, spec_ncg(c));
        if (r != MPS_OK) return r;
        inflight = 2;
      }
      r = spin_wait(c, c->ev_step[b]);
      if (r != MPS_OK) return r;
      const int a = accept_step(c, b, st);
      if (a < 0) return fail_step(c, b, c->h_step_status[b]);
      if (a == 0) {
        r = redo_step(c, b, st);
        if (r == MPS_E_CG_NOCONV) res = r;
        else if (r != MPS_OK) return r;
        ++k;
        break;
      }
      ++k;
      --inflight;
      b = (b + 1) % mps_ctx::NBUF;
      if (inflight == 0) break;
    }
  }
  return res;
}

void free_tape(mps_ctx* c) {
  for (int k = 0; k < c->ntape; ++k) {
    mps_ctx::Slot& t = c->tape[k];
    void* ps[] = {t.pos, t.vel, t.p, t.type, t.id};
    for (void* q : ps)
      if (q) (void)hipFree(q);
  }
  delete[] c->tape;
  c->tape = nullptr;
  c->ntape = 0;
  AdjView& a = c->adj;
  void* as[] = {(void*)a.pos_bar, (void*)a.vel_bar, a.gbar, a.phat_bar, a.pbar, a.nbar,
                a.rs_bar, a.ut, a.sbar, a.pos_bar_in, a.vel_bar_in, a.arg, a.lam, a.part,
                a.mubar, a.gsm};
  for (void* q : as)
    if (q) (void)hipFree(q);
  c->adj = AdjView{};
  if (c->h_part) (void)hipHostFree(c->h_part);
  c->h_part = nullptr;
}

}  // namespace

extern "C" {

mps_status mps_init(const mps_params* params, int64_t n, const double* pos, const double* vel,
                    const int8_t* type, const double* rho_i, const double* nu_i,
                    void* hip_stream, mps_ctx** out) {
  if (!out) return MPS_E_ARG;
  *out = nullptr;
  if (check_params(params, n) != MPS_OK || !pos || !vel || !type) return MPS_E_ARG;
  mps_ctx* c = new (std::nothrow) mps_ctx();
  if (!c) return MPS_E_NOMEM;
  c->P = *params;
  c->n = n;
  c->dim = params->dim;
  c->ps = c->dim == 2 ? 2 : 4;
  // row capacity: max_neigh in whole team steps, and at least the CG
  // iteration's first-pass slots (CG_UNROLL per lane, loaded unchecked)
  c->kpad = std::max((params->max_neigh + TEAM - 1) / TEAM * TEAM, CG_UNROLL * TEAM);
  c->slots = ((n + SLICE - 1) / SLICE) * (int64_t)c->kpad * SLICE;
  c->ncell = params->grid_n[0] * params->grid_n[1] * (c->dim == 3 ? params->grid_n[2] : 1);
  c->s = (hipStream_t)hip_stream;
  c->multi = rho_i || nu_i || params->smagorinsky_cs > 0.0;
  double lam_n;
  lattice(c->dim, params->l0, params->re_n, params->kernel, &c->n0_n, &lam_n);
  lattice(c->dim, params->l0, params->re_lap, params->kernel, &c->n0_lap, &c->lam_lap);

  const size_t nv = (size_t)n * c->ps;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  g_bytes = &c->bytes;
  for (int k = 0; k < mps_ctx::NBUF; ++k) {
    A(dalloc(&c->pos[k], nv));
    A(dalloc(&c->vel[k], nv));
    A(dalloc(&c->pres[k], n));
    A(dalloc(&c->type[k], n));
    A(dalloc(&c->id[k], n));
  }
  for (int k = 0; k < 2; ++k) A(dalloc(&c->pd[k], n));
  A(dalloc(&c->pcell, n));
  A(dalloc(&c->posf, 2 * n));
  A(dalloc(&c->rsf, n));
  A(dalloc(&c->us, nv));
  A(dalloc(&c->rs, nv));
  A(dalloc(&c->nstar, n));
  if (params->source != MPS_SRC_STD) A(dalloc(&c->src, n));
  A(dalloc(&c->flags, n));
  A(dalloc(&c->cellid, n));
  A(dalloc(&c->slot, n));
  A(dalloc(&c->perm, n));
  A(dalloc(&c->cell_count, scan_cells_padded(c->ncell)));
  A(dalloc(&c->cell_start, scan_cells_padded(c->ncell)));
  A(dalloc(&c->cell_local, scan_cells_padded(c->ncell)));
  A(dalloc(&c->tile_sum, scan_tiles(c->ncell)));
  A(dalloc(&c->nb_count, n));
  A(dalloc(&c->nb_list, c->slots));
  A(dalloc(&c->nbn_count, n));
  A(dalloc(&c->nbn_list, c->slots));
  if (params->skin > 0.0) {
    // superset capacity: the cap scaled by the volume of the larger ball,
    // with a fifth more for density fluctuations
    const double f = std::pow((params->re_lap + params->skin) / params->re_lap, c->dim);
    c->cap_s = (int)std::ceil(1.2 * f * params->max_neigh);
    c->kpad_s = (c->cap_s + TEAM - 1) / TEAM * TEAM;
    c->slots_s = ((n + SLICE - 1) / SLICE) * (int64_t)c->kpad_s * SLICE;
    A(dalloc(&c->sk_count, n));
    A(dalloc(&c->sk_list, c->slots_s));
    A(dalloc(&c->r_build, nv));
    A(dalloc(&c->ls, 1));
  }
  A(dalloc(&c->a_nnz, n));
  A(dalloc(&c->a_col, c->slots));
  {
    const size_t b = c->slots * (params->precision == MPS_MIXED ? 4 : 8) + 256;
    A(hipMalloc(&c->a_val, b));
    c->bytes += (int64_t)b;
  }
  A(dalloc(&c->diag, n));
  A(dalloc(&c->b, n));
  A(dalloc(&c->r, n));
  A(dalloc(&c->z, n));
  A(dalloc(&c->q, n));
  A(dalloc(&c->p_save, n));
  if (c->multi) {
    for (int k = 0; k < mps_ctx::NBUF; ++k) {
      A(dalloc(&c->rho_s[k], n));
      A(dalloc(&c->nu_l[k], n));
    }
    A(dalloc(&c->nut, n));
    A(dalloc(&c->rho_o, n));
    A(dalloc(&c->nu_o, n));
    A(dalloc(&c->mu, n));
  }
  c->nspmv = cg_spmv_blocks(n);
  c->nasmb = assemble_blocks(n, params->cg_pipelined != 0);
  c->nupd = cg_update_blocks(n);
  A(dalloc(&c->partA, (size_t)std::max({c->nspmv, c->nupd, c->nasmb}) * 4));
  A(dalloc(&c->partB, (size_t)c->nspmv));
  c->pcg_fused = pcg_blocks(n, true) <= pcg_fused_capacity(params->precond) ? 1 : 0;
  c->npcg = pcg_blocks(n, c->pcg_fused != 0);
  c->pc_block = params->precond == MPS_PC_BLOCK ? 1 : 0;
  if (params->skin > 0.0 || params->precond == MPS_PC_TWO_LEVEL)
    A(dalloc(&c->red_blk, std::max<int64_t>((n + BLOCK - 1) / BLOCK,
                                            (c->ncell + BLOCK - 1) / BLOCK)));
  if (params->precond == MPS_PC_TWO_LEVEL) {
    const int ns = c->dim == 3 ? 27 : 9;
    A(dalloc(&c->ac, (size_t)c->ncell * ns));
    A(dalloc(&c->cwork, (size_t)2 * ((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK) * ns));
    A(dalloc(&c->rc, c->ncell));
    A(dalloc(&c->xc, c->ncell));
    A(dalloc(&c->dc[0], c->ncell));
    A(dalloc(&c->dc[1], c->ncell));
  }
  if (params->precond != MPS_PC_JACOBI) {
    A(dalloc(&c->pl_u, n));
    A(dalloc(&c->pl_q, n));
    A(dalloc(&c->pl_w, n));
  }
  if (params->cg_pipelined) {
    A(dalloc(&c->pl_z, n));
    A(dalloc(&c->pl_s, n));
    for (int k = 0; k < 2; ++k) {
      A(dalloc(&c->pl_m[k], n));
      A(dalloc(&c->pl_part[k], pl_part_len(c)));
      A(dalloc(&c->pl_part2[k], (size_t)PCG_SPLIT_G * 4));
    }
  }
  A(dalloc(&c->sc, 1));
  // [1 + b]: copy taken before a whole-step graph from buffer b
  A(dalloc(&c->status, 1 + mps_ctx::NBUF));
  A(dalloc(&c->step_count, 1));
  A(dalloc(&c->counts, NCOUNTS));
  g_bytes = nullptr;
  // [0]: polled solves; [1 + b]: the whole-step graph from buffer b
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->h_sc, (1 + mps_ctx::NBUF) * sizeof(CGScalars),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_status, sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->h_step_status, (mps_ctx::NBUF + 2) * sizeof(int32_t),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_counts, NCOUNTS * sizeof(int64_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    mps_free(c);
    return e == hipErrorOutOfMemory ? MPS_E_NOMEM : MPS_E_DEVICE;
  }
  // initial state: identity order
  hipStream_t s = c->s;
  A(hipMemsetAsync(c->cell_count, 0, scan_cells_padded(c->ncell) * sizeof(int32_t), s));
  A(hipMemsetAsync(c->status, 0, sizeof(int32_t), s));
  A(hipMemsetAsync(c->step_count, 0, sizeof(int32_t), s));
  A(hipMemsetAsync(c->sc, 0, sizeof(CGScalars), s));
  // the fused iteration sums every slot of its partial arrays: zeros past
  // npcg, which no kernel writes
  for (int k = 0; k < 2; ++k)
    if (c->pl_part[k]) A(hipMemsetAsync(c->pl_part[k], 0, pl_part_len(c) * sizeof(double), s));
  A(hipMemsetAsync(c->nb_count, 0, n * sizeof(int32_t), s));
  A(hipMemsetAsync(c->nbn_count, 0, n * sizeof(int32_t), s));
  if (c->ls) {
    A(hipMemsetAsync(c->ls, 0, sizeof(ListState), s));
    A(hipMemsetAsync(c->sk_count, 0, n * sizeof(int32_t), s));
    A(hipMemsetAsync(c->r_build, 0, nv * sizeof(double), s));
    force_build(c);
  }
  A(hipMemsetAsync(c->a_nnz, 0, n * sizeof(int32_t), s));
  A(hipMemsetAsync(c->nstar, 0, n * sizeof(double), s));
  A(hipMemsetAsync(c->flags, 0, n, s));
  A(hipMemsetAsync(c->pres[0], 0, n * sizeof(double), s));
  k_iota<<<flat_blocks(n), 256, 0, s>>>(n, c->id[0]);
  View v = make_view(c);
  launch_gather_orig(v, pos, c->pos[0], c->dim, c->ps, s);
  launch_gather_orig(v, vel, c->vel[0], c->dim, c->ps, s);
  A(hipMemcpyAsync(c->type[0], type, n, hipMemcpyDeviceToDevice, s));
  k_check_types<<<flat_blocks(n), 256, 0, s>>>(n, c->type[0], c->status);
  if (c->multi) {
    if (rho_i) launch_gather_orig(v, rho_i, c->rho_s[0], 1, 1, s);
    else k_fill<<<flat_blocks(n), 256, 0, s>>>(n, c->rho_s[0], params->rho);
    if (nu_i) launch_gather_orig(v, nu_i, c->nu_l[0], 1, 1, s);
    else k_fill<<<flat_blocks(n), 256, 0, s>>>(n, c->nu_l[0], params->nu);
    A(hipMemsetAsync(c->nut, 0, n * sizeof(double), s));
    // the smoothed density is fixed before the run, from the initial lists
    search(c);
    View w = make_view(c);
    launch_smooth_density(w, c->rho_s[c->cur], c->rho_s[nxt(c)], c->dim, s);
    A(hipMemcpyAsync(c->rho_s[c->cur], c->rho_s[nxt(c)], n * sizeof(double),
                     hipMemcpyDeviceToDevice, s));
    launch_scatter_orig(w, c->rho_s[c->cur], c->rho_o, 1, 1, s);
    launch_scatter_orig(w, c->nu_l[c->cur], c->nu_o, 1, 1, s);
  }
  A(hipGetLastError());
  A(hipStreamSynchronize(s));
  if (e != hipSuccess) {
    mps_free(c);
    return MPS_E_DEVICE;
  }
  mps_status st = read_status(c);
  // block Jacobi is applied inside the one-kernel iteration only
  if (st != MPS_OK || (c->pc_block && !c->pcg_fused)) {
    mps_free(c);
    return MPS_E_ARG;
  }
  if (!c->pcg_fused) {
    // Dummy particles are never unknowns and their rows hold no entries.
    // Where they are one row in five or more (the 3-D tanks with two dummy
    // layers), the split iteration kernel loads only the slots a row holds;
    // with fewer, loading the first slots unconditionally is faster.
    std::vector<int8_t> ht((size_t)n);
    if (hipMemcpy(ht.data(), c->type[0], (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
      mps_free(c);
      return MPS_E_DEVICE;
    }
    const int64_t nd = std::count(ht.begin(), ht.end(), (int8_t)MPS_DUMMY);
    c->pcg_pred = nd * 5 >= n ? 1 : 0;
  }
  *out = c;
  return MPS_OK;
}

namespace {
void free_tape(mps_ctx* c);
}

mps_status mps_free(mps_ctx* c) {
  if (!c) return MPS_OK;
  if (c->s) (void)hipStreamSynchronize(c->s);
  for (int k = 0; k < mps_ctx::NBUF; ++k) {
    void* st[] = {c->pos[k], c->vel[k], c->pres[k], c->type[k], c->id[k], c->rho_s[k],
                  c->nu_l[k]};
    for (void* p : st)
      if (p) (void)hipFree(p);
  }
  void* ptrs[] = {c->pd[0], c->pd[1],
                  c->pcell, c->posf, c->rsf, c->us, c->rs, c->nstar, c->src, c->flags,
                  c->cellid, c->slot, c->perm, c->cell_count, c->cell_start,
                  c->cell_local, c->tile_sum,
                  c->nb_count,
                  c->nb_list, c->nbn_count, c->nbn_list, c->a_nnz, c->a_col, c->a_val, c->diag, c->b, c->r, c->z,
                  c->q, c->p_save, c->partA, c->partB, c->sc, c->status, c->step_count,
                  c->sk_count, c->sk_list, c->r_build, c->ls, c->red_blk,
                  c->ac, c->cwork, c->rc, c->xc, c->dc[0], c->dc[1], c->pl_u, c->pl_q,
                  c->pl_w,
                  c->counts,
                  c->nut, c->mu,
                  c->rho_o, c->nu_o,
                  c->pl_z, c->pl_s, c->pl_m[0], c->pl_m[1], c->pl_part[0], c->pl_part[1],
                  c->pl_part2[0], c->pl_part2[1]};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < mps_ctx::NBUF; ++k) {
    hipGraphExec_t gs[] = {c->g_pre[k], c->g_cg[k][0], c->g_cg[k][1], c->g_cg[k][2],
                           c->g_post[k], c->g_wc2[k]};
    for (hipGraphExec_t g : gs)
      if (g) (void)hipGraphExecDestroy(g);
    for (auto& sg : c->g_step[k])
      if (sg.g) (void)hipGraphExecDestroy(sg.g);
  }
  if (c->ev_created)
    for (int k = 0; k < mps_ctx::kPool; ++k) {
      (void)hipEventDestroy(c->ev_a[k]);
      (void)hipEventDestroy(c->ev_b[k]);
    }
  if (c->ev_step_created)
    for (hipEvent_t ev : c->ev_step) (void)hipEventDestroy(ev);
  free_tape(c);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_step_status) (void)hipHostFree(c->h_step_status);
  if (c->h_counts) (void)hipHostFree(c->h_counts);
  delete c;
  return MPS_OK;
}

const char* mps_last_error(const mps_ctx* c) { return c ? c->err : mps::noctx_error(); }

mps_status mps_device_bytes(const mps_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return MPS_E_ARG;
  *bytes = c->bytes + c->tape_bytes;
  return MPS_OK;
}

mps_status mps_constants(const mps_ctx* c, double* n0_n, double* n0_lap, double* lambda_lap) {
  if (!c) return MPS_E_ARG;
  if (n0_n) *n0_n = c->n0_n;
  if (n0_lap) *n0_lap = c->n0_lap;
  if (lambda_lap) *lambda_lap = c->lam_lap;
  return MPS_OK;
}

mps_status mps_neighbors(mps_ctx* c, int32_t* cell_id, int32_t* count, int32_t* list) {
  if (!c) return MPS_E_ARG;
  if (c->poisoned) return fail(c, MPS_E_POISONED, "context poisoned; call mps_set_state");
  search(c);
  View v = make_view(c);
  launch_export_lists(v, cell_id, count, list, c->dim, c->s);
  HIPCHK(c, hipGetLastError());
  return read_status(c);
}

mps_status mps_step(mps_ctx* c, int32_t nsteps, mps_step_stats* stats) {
  if (!c || nsteps < 0) return MPS_E_ARG;
  if (c->poisoned) return fail(c, MPS_E_POISONED, "context poisoned; call mps_set_state");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  mps_status res = MPS_OK;
  c->steps_ok = 0;
  if (c->ls)
    HIPCHK(c, hipMemsetAsync(&c->ls->builds, 0, sizeof(int32_t), c->s));
  if (c->P.pmode == MPS_WC_EOS) {
    // no host synchronisation between the steps: each step counts itself
    // on the device when it begins with a clean status, and once a step has
    // raised an error the steps behind it write no state, so the failing
    // step's input is the buffer after (count - 1) steps
    const int cur0 = c->cur;
    HIPCHK(c, hipMemsetAsync(c->step_count, 0, sizeof(int32_t), c->s));
    res = steps_wc(c, nsteps);
    if (res != MPS_OK) return res;
    HIPCHK(c, hipGetLastError());
    int32_t* hs = c->h_step_status;
    HIPCHK(c, hipMemcpyAsync(hs, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, c->s));
    HIPCHK(c, hipMemcpyAsync(hs + mps_ctx::NBUF + 1, c->step_count, sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->s));
    HIPCHK(c, hipStreamSynchronize(c->s));
    prof_flush(c);
    if (hs[0]) {
      const int begun = std::max(1, (int)hs[mps_ctx::NBUF + 1]);
      c->cur = (cur0 + begun - 1) % mps_ctx::NBUF;
      if (stats) stats->steps = begun - 1;
      return status_error(c, hs[0]);
    }
    c->steps_ok = nsteps;
  } else {
    res = steps_ppe(c, nsteps, stats);
    if (stats) stats->steps = c->steps_ok;
    if (res != MPS_OK && res != MPS_E_CG_NOCONV) return res;
  }
  HIPCHK(c, hipGetLastError());
  mps_status st = read_status(c);
  if (st != MPS_OK) return st;
  if (stats) {
    stats->steps = c->steps_ok;
    HIPCHK(c, hipMemsetAsync(c->counts, 0, NCOUNTS * sizeof(int64_t), c->s));
    k_count_flags<<<flat_blocks(c->n), 256, 0, c->s>>>(c->n, c->flags, c->nb_count,
                                                       c->nbn_count, c->a_nnz,
                                                       c->P.pmode == MPS_PPE_CG, c->counts);
    HIPCHK(c, hipMemcpyAsync(c->h_counts, c->counts, NCOUNTS * sizeof(int64_t),
                             hipMemcpyDeviceToHost, c->s));
    HIPCHK(c, hipStreamSynchronize(c->s));
    stats->n_surface = c->h_counts[0];
    stats->n_ghost = c->h_counts[1];
    stats->list_entries = c->h_counts[2];
    stats->ppe_nnz = c->h_counts[3];
    stats->short_entries = c->h_counts[4];
    stats->list_builds = nsteps;
    if (c->ls) {
      int32_t* hb = c->h_step_status + mps_ctx::NBUF + 1;
      HIPCHK(c, hipMemcpyAsync(hb, &c->ls->builds, sizeof(int32_t), hipMemcpyDeviceToHost, c->s));
      HIPCHK(c, hipStreamSynchronize(c->s));
      stats->list_builds = *hb;
    }
  }
  return res;
}

mps_status mps_pressure_solve(mps_ctx* c, const double* rhs, double* p, int32_t* iters,
                              double* relres) {
  if (!c || !p) return MPS_E_ARG;
  if (c->poisoned) return fail(c, MPS_E_POISONED, "context poisoned; call mps_set_state");
  const bool fold = c->P.skin > 0.0 && !c->multi;
  search(c, fold);
  View v = make_view(c);
  HIPCHK(c, hipMemcpyAsync(c->p_save, c->pres[c->cur], c->n * sizeof(double),
                           hipMemcpyDeviceToDevice, c->s));
  launch_predict(v, c->dim, c->P.precision, fold, c->s);
  launch_density(v, c->dim, c->P.precision, MPS_PPE_CG, c->s);
  const double* rhs_sorted = nullptr;
  if (rhs) {
    // q is free until the CG starts
    launch_gather_orig(v, rhs, c->q, 1, 1, c->s);
    rhs_sorted = c->q;
  }
  enqueue_assemble(c, v, rhs_sorted, true);
  c->ppe_valid = true;
  int it = 0;
  double rel = 0.0;
  const int saved_last = c->last_iters;
  c->last_iters = 0;
  mps_status res = solve(c, &it, &rel, false);
  c->last_iters = saved_last;
  if (res != MPS_OK && res != MPS_E_CG_NOCONV) return res;
  launch_scatter_orig(v, c->pres[c->cur], p, 1, 1, c->s);
  HIPCHK(c, hipMemcpyAsync(c->pres[c->cur], c->p_save, c->n * sizeof(double),
                           hipMemcpyDeviceToDevice, c->s));
  if (iters) *iters = it;
  if (relres) *relres = rel;
  HIPCHK(c, hipGetLastError());
  mps_status st = read_status(c);
  return st != MPS_OK ? st : res;
}

mps_status mps_get_ppe(mps_ctx* c, double* diag, double* b, int32_t* nnz, int32_t* cols,
                       double* vals) {
  if (!c) return MPS_E_ARG;
  if (!c->ppe_valid) return fail(c, MPS_E_ARG, "no assembled system");
  View v = make_view(c);
  launch_export_ppe(v, c->P.precision, diag, b, nnz, cols, vals, c->s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->s));
  return MPS_OK;
}

mps_status mps_get_state(mps_ctx* c, double* pos, double* vel, double* p, double* n_star,
                         int8_t* flags, int8_t* type) {
  if (!c) return MPS_E_ARG;
  View v = make_view(c);
  if (pos) launch_scatter_orig(v, c->pos[c->cur], pos, c->dim, c->ps, c->s);
  if (vel) launch_scatter_orig(v, c->vel[c->cur], vel, c->dim, c->ps, c->s);
  if (p) launch_scatter_orig(v, c->pres[c->cur], p, 1, 1, c->s);
  if (n_star) launch_scatter_orig(v, c->nstar, n_star, 1, 1, c->s);
  const unsigned nb = flat_blocks(c->n);
  if (flags) k_i8_to_orig<<<nb, 256, 0, c->s>>>(c->n, c->id[c->cur], c->flags, flags);
  if (type) k_i8_to_orig<<<nb, 256, 0, c->s>>>(c->n, c->id[c->cur], c->type[c->cur], type);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->s));
  return MPS_OK;
}

mps_status mps_set_state(mps_ctx* c, const double* pos, const double* vel, const int8_t* type) {
  if (!c || !pos || !vel) return MPS_E_ARG;
  View v = make_view(c);
  launch_gather_orig(v, pos, c->pos[c->cur], c->dim, c->ps, c->s);
  launch_gather_orig(v, vel, c->vel[c->cur], c->dim, c->ps, c->s);
  if (type) {
    k_i8_from_orig<<<flat_blocks(c->n), 256, 0, c->s>>>(c->n, c->id[c->cur], type,
                                                        c->type[c->cur]);
    k_check_types<<<flat_blocks(c->n), 256, 0, c->s>>>(c->n, c->type[c->cur], c->status);
  }
  HIPCHK(c, hipMemsetAsync(c->pres[c->cur], 0, c->n * sizeof(double), c->s));
  force_build(c);
  HIPCHK(c, hipGetLastError());
  c->poisoned = false;
  c->ppe_valid = false;
  c->last_iters = 0;
  mps_status st = read_status(c);
  if (st != MPS_OK) {
    c->poisoned = true;
    return st;
  }
  return MPS_OK;
}

mps_status mps_profile(mps_ctx* c, uint32_t mask) {
  if (!c) return MPS_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->s));
  if (mask && !c->ev_created) {
    for (int k = 0; k < mps_ctx::kPool; ++k) {
      HIPCHK(c, hipEventCreate(&c->ev_a[k]));
      HIPCHK(c, hipEventCreate(&c->ev_b[k]));
    }
    c->ev_created = true;
  }
  prof_flush(c);
  c->prof_mask = mask;
  for (int k = 0; k < MPS_KC_COUNT; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return MPS_OK;
}

mps_status mps_profile_read(mps_ctx* c, double* ms, int64_t* launches) {
  if (!c) return MPS_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->s));
  prof_flush(c);
  for (int k = 0; k < MPS_KC_COUNT; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (launches) launches[k] = c->prof_n[k];
  }
  return MPS_OK;
}

mps_status mps_get_phase(mps_ctx* c, double* rho_s, double* nu_t) {
  if (!c) return MPS_E_ARG;
  if (!c->multi) return fail(c, MPS_E_ARG, "single-phase context");
  View v = make_view(c);
  if (rho_s) launch_scatter_orig(v, c->rho_s[c->cur], rho_s, 1, 1, c->s);
  if (nu_t) launch_scatter_orig(v, c->nut, nu_t, 1, 1, c->s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->s));
  return MPS_OK;
}

mps_status mps_tape_alloc(mps_ctx* c, int32_t nslots) {
  if (!c || nslots < 1) return MPS_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->s));
  free_tape(c);
  const int64_t n = c->n;
  const size_t nv = (size_t)n * c->ps;
  c->tape = new (std::nothrow) mps_ctx::Slot[nslots];
  if (!c->tape) return fail(c, MPS_E_NOMEM, "tape");
  c->ntape = nslots;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  const int64_t before = c->bytes;
  c->tape_bytes = 0;
  g_bytes = &c->tape_bytes;
  for (int k = 0; k < nslots; ++k) {
    mps_ctx::Slot& t = c->tape[k];
    A(dalloc(&t.pos, nv));
    A(dalloc(&t.vel, nv));
    A(dalloc(&t.p, n));
    A(dalloc(&t.type, n));
    A(dalloc(&t.id, n));
  }
  AdjView& a = c->adj;
  double *pb = nullptr, *vb = nullptr;
  A(dalloc(&pb, nv));
  A(dalloc(&vb, nv));
  a.pos_bar = pb;
  a.vel_bar = vb;
  A(dalloc(&a.gbar, nv));
  A(dalloc(&a.phat_bar, n));
  A(dalloc(&a.pbar, n));
  A(dalloc(&a.nbar, n));
  A(dalloc(&a.rs_bar, nv));
  A(dalloc(&a.ut, nv));
  A(dalloc(&a.sbar, nv));
  A(dalloc(&a.pos_bar_in, nv));
  A(dalloc(&a.vel_bar_in, nv));
  A(dalloc(&a.arg, n));
  A(dalloc(&a.lam, n));
  const int nb = adj_partial_blocks(n);
  A(dalloc(&a.part, (size_t)nb * 4));
  if (c->multi) {
    A(dalloc(&a.mubar, n));
    A(dalloc(&a.gsm, (size_t)n * 9));
  }
  g_bytes = nullptr;
  (void)before;
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_part, (size_t)nb * 4 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    free_tape(c);
    return e == hipErrorOutOfMemory ? fail(c, MPS_E_NOMEM, "tape allocation")
                                    : hip_fail(c, e, "tape allocation");
  }
  return MPS_OK;
}

mps_status mps_tape_save(mps_ctx* c, int32_t slot) {
  if (!c || slot < 0 || slot >= c->ntape) return MPS_E_ARG;
  mps_ctx::Slot& t = c->tape[slot];
  const int64_t n = c->n;
  const size_t nv = (size_t)n * c->ps * sizeof(double);
  const int a = c->cur;
  HIPCHK(c, hipMemcpyAsync(t.pos, c->pos[a], nv, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(t.vel, c->vel[a], nv, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(t.p, c->pres[a], n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(t.type, c->type[a], n, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(t.id, c->id[a], n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->s));
  t.valid = true;
  return MPS_OK;
}

mps_status mps_tape_load(mps_ctx* c, int32_t slot) {
  if (!c || slot < 0 || slot >= c->ntape || !c->tape[slot].valid) return MPS_E_ARG;
  mps_ctx::Slot& t = c->tape[slot];
  const int64_t n = c->n;
  const size_t nv = (size_t)n * c->ps * sizeof(double);
  const int a = c->cur;
  HIPCHK(c, hipMemcpyAsync(c->pos[a], t.pos, nv, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(c->vel[a], t.vel, nv, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(c->pres[a], t.p, n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(c->type[a], t.type, n, hipMemcpyDeviceToDevice, c->s));
  HIPCHK(c, hipMemcpyAsync(c->id[a], t.id, n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->s));
  if (c->multi) {
    // the per-particle phase data follow the slot's particle order
    View v = make_view(c);
    launch_gather_orig(v, c->rho_o, c->rho_s[a], 1, 1, c->s);
    launch_gather_orig(v, c->nu_o, c->nu_l[a], 1, 1, c->s);
  }
  force_build(c);
  c->ppe_valid = false;
  return MPS_OK;
}

mps_status mps_step_adjoint(mps_ctx* c, const double* pos_bar, const double* vel_bar,
                            double* pos_bar_prev, double* vel_bar_prev, double* nu_bar,
                            double* g_bar) {
  if (!c || !pos_bar || !vel_bar || !pos_bar_prev || !vel_bar_prev) return MPS_E_ARG;
  if (!c->tape) return fail(c, MPS_E_ARG, "call mps_tape_alloc first");
  if (c->P.skin > 0.0) return fail(c, MPS_E_ARG, "adjoint needs lists built every step (skin 0)");
  if (c->poisoned) return fail(c, MPS_E_POISONED, "context poisoned; call mps_set_state");
  const bool wc = c->P.pmode == MPS_WC_EOS;
  // forward recompute of the step's stages from the current (taped) state
  enqueue_pre(c);
  mps_status res = MPS_OK;
  if (!wc) {
    int it = 0;
    double rel = 0.0;
    res = solve(c, &it, &rel, false);
    if (res != MPS_OK && res != MPS_E_CG_NOCONV) return res;
    c->last_iters = it;
  }
  View v = make_view(c);
  AdjView a = c->adj;
  launch_gather_orig(v, pos_bar, const_cast<double*>(a.pos_bar), c->dim, c->ps, c->s);
  launch_gather_orig(v, vel_bar, const_cast<double*>(a.vel_bar), c->dim, c->ps, c->s);
  launch_adjoint_head(v, a, c->dim, c->P.precision, wc ? 1 : 0, c->s);
  if (!wc) {
    // transposed solve A lambda = x-bar (A is symmetric): same matrix, same
    // CG kernels, from lambda = 0; the forward pressure is kept aside
    HIPCHK(c, hipMemcpyAsync(c->p_save, c->pres[c->cur], c->n * sizeof(double),
                             hipMemcpyDeviceToDevice, c->s));
    enqueue_assemble(c, v, a.pbar, true);
    int it = 0;
    double rel = 0.0;
    const int saved = c->last_iters;
    mps_status r2 = solve(c, &it, &rel, false);
    c->last_iters = saved;
    if (r2 != MPS_OK && r2 != MPS_E_CG_NOCONV) return r2;
    if (r2 == MPS_E_CG_NOCONV) res = r2;
    HIPCHK(c, hipMemcpyAsync(a.lam, c->pres[c->cur], c->n * sizeof(double),
                             hipMemcpyDeviceToDevice, c->s));
    HIPCHK(c, hipMemcpyAsync(c->pres[c->cur], c->p_save, c->n * sizeof(double),
                             hipMemcpyDeviceToDevice, c->s));
    launch_adjoint_ppe(v, a, c->dim, c->s);
  }
  launch_adjoint_tail(v, a, c->dim, c->s);
  launch_scatter_orig(v, a.pos_bar_in, pos_bar_prev, c->dim, c->ps, c->s);
  launch_scatter_orig(v, a.vel_bar_in, vel_bar_prev, c->dim, c->ps, c->s);
  const int nb = adj_partial_blocks(c->n);
  HIPCHK(c, hipMemcpyAsync(c->h_part, a.part, (size_t)nb * 4 * sizeof(double),
                           hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipGetLastError());
  mps_status st = read_status(c);
  if (st != MPS_OK) return st;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b)
    for (int q = 0; q < 4; ++q) s4[q] += c->h_part[(size_t)b * 4 + q];
  if (nu_bar) *nu_bar = s4[0];
  if (g_bar)
    for (int q = 0; q < c->dim; ++q) g_bar[q] = s4[1 + q];
  return res;
}

}  // extern "C"
