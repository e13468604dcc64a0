// Internal definitions shared by the HIP translation units of the MPS
// library (gfx950).  Not part of the public ABI (include/mps.h).
//
// Execution model
//   Every per-particle kernel assigns a TEAM of 8 lanes to one particle: a
//   64-lane wavefront covers 8 consecutive cell-sorted particles, a 256-lane
//   workgroup 32.  The lanes of a team split the particle's neighbour (or
//   matrix-row) entries and combine their partial sums with cross-lane
//   shuffles in a fixed tree, so every sum is bitwise reproducible.  Eight
//   lanes per particle keep several wavefronts per SIMD busy already at a
//   few ten thousand particles, where one thread per particle would leave
//   most of the 1024 SIMDs of the chip idle.
//
// Sliced layout of per-neighbour arrays (lists, matrix columns and values)
//   Rows are grouped in slices of H = 8 consecutive particles (one
//   wavefront).  Inside a slice, entry l of row r lives at
//     (l / TEAM) * 64 + r * TEAM + (l % TEAM)
//   so one load instruction of a wavefront reads 64 consecutive words: a
//   fully coalesced 256 B (int32/float) or 512 B (double) segment.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mps.h"

namespace mps {

constexpr int TEAM = 8;
constexpr int WAVE = 64;
constexpr int SLICE = WAVE / TEAM;        // rows per wavefront
constexpr int BLOCK = 256;
constexpr int ROWS_PER_BLOCK = BLOCK / TEAM;
// cell-count scan: tiles of SCAN_TILE cells, one workgroup of SCAN_NT
// threads (SCAN_PER cells each) per tile
constexpr int SCAN_NT = 256, SCAN_PER = 16, SCAN_TILE = SCAN_NT * SCAN_PER;
// cells allocated for the counts and starts (ncell + 2, in whole tiles)
inline int64_t scan_cells_padded(int ncell) {
  return ((int64_t)ncell + 2 + SCAN_TILE - 1) / SCAN_TILE * SCAN_TILE;
}
inline int scan_tiles(int ncell) { return (int)(scan_cells_padded(ncell) / SCAN_TILE); }

// Status bits raised by kernels (one int32 word on the device).
enum : int32_t {
  ST_OVERFLOW = 1,
  ST_COINCIDENT = 2,
  ST_NONFINITE = 4,
  ST_BADTYPE = 8,
};

__host__ __device__ inline int64_t sl_index(int64_t row, int l, int kpad) {
  return (row / SLICE) * ((int64_t)kpad * SLICE) + (int64_t)(l / TEAM) * WAVE +
         (row % SLICE) * TEAM + (l % TEAM);
}

// Conjugate-gradient scalars, kept on the device so that no iteration
// needs the host.  Each field has exactly one writer kernel and is only read
// by later kernels (or by other workgroups of the writer that never read
// it), so no fence or atomic is needed inside a kernel.
struct CGScalars {
  double rzh[2];     // (r, z) of iterate k, slot k & 1 (written by SpMV k)
  double bb;         // (b, b) (written by SpMV 0)
  double rr;         // (r, r) of the last iterate checked (written by SpMV k)
  int32_t k_next;    // index of the next SpMV (written by assembly / update)
  int32_t k_cur;     // index of the running iteration (written by SpMV)
  int32_t converged; // 1 once ||r|| <= tol ||b|| (written by SpMV)
  int32_t iter;      // iterations completed
  int32_t nasm;      // number of assembly partials (written by assembly)
  int32_t pad;
  // pipelined variant: 1 / (r,u) and alpha of iteration k in slot k & 1,
  // written by workgroup 0 of iteration k and read by iteration k + 1 only
  // (which then needs no division for beta)
  double gam[2];
  double alp[2];
  // two-level preconditioner: Gershgorin bound of D_c^-1 A_c (bits of a
  // non-negative double; written after the coarse assembly)
  unsigned long long cg_bits;
};

// Neighbour lists kept over several steps (skin > 0): the cell search
// writes a superset list at radius re_lap + skin, and every step filters
// it to the exact list at its own positions.  The superset is rebuilt (with
// a fresh cell sort) when a particle has moved skin/2 or more since the
// build, or left the grid; in between the particle order stays fixed.  One
// record on the device, written by the check and decision kernels of a step.
struct ListState {
  int32_t force;             // rebuild at the next decision
  int32_t rebuild;           // decision of the running step
  int32_t since;             // steps since the last build
  int32_t builds;            // builds since the host last cleared it
};

// Grid caps of the CG kernels: every workgroup of one kernel sums all the
// per-workgroup partials of the previous kernel, so their number is bounded.
constexpr int CG_SPMV_BLOCKS = 2048;
constexpr int CG_UPD_BLOCKS = 1024;
// Pipelined CG: workgroup size (one group of PCG_BLOCK / TEAM rows per
// workgroup) and the largest grid of the fused one-kernel iteration, whose
// workgroups all load every partial of the previous iteration (three
// doubles per workgroup); it is also kept within what runs in one wave of
// workgroups on the device.
#ifndef PCG_BLOCK
#define PCG_BLOCK 512
#endif
#ifndef PCG_MAX_BLOCKS
#define PCG_MAX_BLOCKS 1024
#endif
// fused schedule: each quantity of the per-workgroup partials in an array
// of its own, this long
constexpr int PCG_PSTRIDE = PCG_MAX_BLOCKS;
#ifndef PCG_SPLIT_BLOCK
#define PCG_SPLIT_BLOCK 256
#endif
constexpr int RED_BLOCK = 1024;  // the one workgroup of a CG reduction kernel
// split schedule: the per-workgroup partials of an iteration are first
// summed by PCG_SPLIT_G workgroups of RED2_BLOCK threads (contiguous slices,
// fixed order); the next iteration's workgroups sum those few
constexpr int PCG_SPLIT_G = 64, RED2_BLOCK = 256;
// Matrix entries per lane loaded ahead of the reduction in the pipelined
// CG iteration (6 x 8 lanes cover a 2-D row: at most 44 inner neighbours on
// a lattice at re = 4 l0)
#ifndef CG_UNROLL
#define CG_UNROLL 6
#endif

// Everything a kernel may touch, passed by value.
struct View {
  int64_t n;
  int kpad;          // per-row slot capacity rounded up to TEAM
  int max_neigh;
  int nx, ny, nz, ncell;
  double lo[3];
  double cs, inv_cs;
  float cs32;
  double re_n, re_lap, re_n2, re_lap2;
  float re_n_f, re_lap_f;
  double n0_n, n0_lap, lam_lap;
  double nu, rho, dt, beta, c0, alpha;
  double cg_tol2;
  double g[3];
  int gamma_i, kernel, grad, clamp;
  int source;         // MPS_SRC_*: PPE source term
  int laplacian;      // MPS_LAP_*: Laplacian of pressure in the PPE
  // lists kept over steps (null ls: a fresh list every step)
  ListState* ls;
  double half_skin2;  // (skin / 2)^2
  double re_s2;       // (re_lap + skin)^2, the superset's radius
  int kpad_s, cap_s;  // superset row capacity (slots, entries)
  int32_t* sk_list;   // superset lists (sliced, kpad_s slots per row)
  int32_t* sk_count;
  double* r_build;    // sorted positions at the last build
  double* red_blk;    // per-workgroup maxima of a step's order-free reductions
                      // (list displacement, coarse Gershgorin bound)
  int pc_block;       // block-Jacobi preconditioner (fused schedule only)
  // two-level preconditioner of the pipelined CG (null ac: Jacobi)
  double* ac;         // cell-level operator P^T A P, 3^DIM stencil slots,
                      // slot-major: ac[slot * ncell + cell]
  double* cwork;      // partial cell rows of workgroups (2 x rows/32 x 3^DIM)
  double* rc;         // cell residual of the Chebyshev steps
  double* xc;         // cell correction
  double* dc[2];      // Chebyshev directions (double buffered)
  double* pl_u;       // u = M^-1 r, q, w (stored: M is not diagonal)
  double* pl_q;
  double* pl_w;
  // sorted state, current buffers
  const double* pos;  double* pos_w;
  const double* vel;  double* vel_w;
  const int8_t* type; int8_t* type_w;
  const int32_t* id;  int32_t* id_w;
  const double* p_in; double* p_w;
  // per-step arrays (sorted order)
  int32_t* pcell;     // packed cell coordinates
  float4* posf;       // mixed, two per particle: r^k relative to the anchor
                      // cell + packed cell; FP32 u^k
  float4* rsf;        // mixed: r*  relative to the anchor cell + packed cell
  double* us;         // u*
  double* rs;         // r*
  double* nstar;
  double* src;        // PPE right-hand side from Dn/Dt (source != MPS_SRC_STD)
  int8_t* flags;
  // binning
  int32_t* cellid;    // old order
  int32_t* slot;      // old order
  int32_t* cell_count;
  int32_t* cell_local;  // exclusive scan of the counts inside each tile
  int32_t* tile_sum;    // total count of each tile
  int32_t* cell_start;
  int ntile;
  int32_t* perm;      // unordered scatter of the particles by cell
  // lists
  int32_t* nb_count;
  int32_t* nb_list;
  // short lists: the entries of each list within re_n at r*, in list
  // order, written by the density kernel for the p-hat and gradient kernels
  // (same layout and slot capacity as nb_list).  re_n2_keep: re_n^2 widened
  // by a relative 1e-4, so that the FP32 distance tests of the mixed path,
  // which round differently from the FP64 test of the density kernel, never
  // meet an entry it dropped.
  int32_t* nbn_count;
  int32_t* nbn_list;
  double re_n2_keep;

  // PPE
  int32_t* a_nnz;
  int32_t* a_col;
  void* a_val;        // float (mixed) or double
  double* diag;
  double* b;
  double* p;          // pressure (CG iterate), sorted order
  // CG
  double* r;
  double* z;
  double* pd[2];
  double* q;
  double* partA;      // [blocks][4]: (r,z), (r,r), (b,b) of assembly / update
  double* partB;      // [blocks]: (p, A p) of the SpMV workgroups
  int nspmv, nupd;    // grid sizes of the textbook SpMV and update kernels
  int nasmb;          // grid size of the assembly
  int npcg;           // grid size of the pipelined CG kernels (one row group each)
  int pcg_fused;      // 1: one kernel per iteration; 0: reduction + iteration
  int pcg_pred;       // split schedule: slot loads predicated on the row length
  CGScalars* sc;
  // pipelined CG (one kernel per iteration): m = D^-1 w (double buffered),
  // z, s; the direction p reuses pd[0]
  double* pl_z;
  double* pl_s;
  double* pl_m[2];
  double* pl_part[2]; // per-workgroup (r,u), (w,u), (r,r), double buffered
  double* pl_part2[2];// split schedule: sums of slices of pl_part (npcg2 each)
  int npcg2;
  int32_t* status;
  // two-phase / turbulence (null when single phase)
  const double* rho_s;   // smoothed density <rho>_i, sorted
  double* rho_s_w;       // permutation target
  const double* nu_l;    // laminar viscosity per particle, sorted
  double* nu_l_w;
  double* nut;           // Smagorinsky eddy viscosity
  double* mu;            // dynamic viscosity <rho> (nu + nu_t)
  double smag_c2;        // (Cs l0)^2
};

// Adjoint work arrays (sorted order).
struct AdjView {
  const double* pos_bar;   // r-bar of the step output
  const double* vel_bar;   // u-bar of the step output
  double* gbar;            // G-bar   [n][ps]
  double* phat_bar;        // phat-bar [n]
  double* pbar;            // p-bar (then n*-bar)  [n]
  double* nbar;            // n*-bar [n]
  double* rs_bar;          // r*-bar [n][ps]
  double* ut;              // u-tilde = u*-bar + dt r*-bar  [n][ps]
  double* sbar;            // S-bar [n][ps]
  double* pos_bar_in;      // r-bar of the step input  [n][ps]
  double* vel_bar_in;      // u-bar of the step input  [n][ps]
  int32_t* arg;            // p-hat argmin (sorted index)
  double* lam;             // PPE adjoint solution (lambda)
  double* part;            // [blocks][4]: nu-bar, g-bar
  // two-phase / turbulence (null when single phase)
  double* mubar;           // mu-bar [n]
  double* gsm;             // velocity-gradient bar of the Smagorinsky term [n][9]
};

// Packed cell coordinates: 10 bits per axis (x lowest); GHOST_CELL marks a
// particle outside the grid.
constexpr int32_t GHOST_CELL = -1;
__host__ __device__ inline int32_t pack_cell(int cx, int cy, int cz) {
  return cx | (cy << 10) | (cz << 20);
}
__device__ inline int ucx(int32_t pc) { return pc & 1023; }
__device__ inline int ucy(int32_t pc) { return (pc >> 10) & 1023; }
__device__ inline int ucz(int32_t pc) { return (pc >> 20) & 1023; }

// Position storage stride in doubles: 2-D uses double2, 3-D a padded double4.
template <int DIM>
struct PS { static constexpr int v = DIM == 2 ? 2 : 4; };

template <int DIM>
__device__ inline void load_vec(const double* a, int64_t i, double (&x)[DIM]) {
  if constexpr (DIM == 2) {
    double2 v = reinterpret_cast<const double2*>(a)[i];
    x[0] = v.x; x[1] = v.y;
  } else {
    const double2* p = reinterpret_cast<const double2*>(a) + 2 * i;
    double2 v0 = p[0], v1 = p[1];
    x[0] = v0.x; x[1] = v0.y; x[2] = v1.x;
  }
}
template <int DIM>
__device__ inline void store_vec(double* a, int64_t i, const double (&x)[DIM]) {
  if constexpr (DIM == 2) {
    reinterpret_cast<double2*>(a)[i] = make_double2(x[0], x[1]);
  } else {
    double2* p = reinterpret_cast<double2*>(a) + 2 * i;
    p[0] = make_double2(x[0], x[1]);
    p[1] = make_double2(x[2], 0.0);
  }
}

// Logical block index with consecutive particle ranges kept on one XCD:
// hardware dispatches workgroup b to XCD b % 8, so remap such that each XCD
// owns one contiguous chunk of the cell-sorted particles and the neighbour
// data it gathers stays in that XCD's L2.
__device__ inline int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Squared FP64 distance term by term, without contraction: the neighbour
// decision of the lists (search, superset filter, the prediction that
// filters kept lists), so that every path decides a pair the same way.
template <int DIM>
__device__ inline double dist2_exact(const double (&a)[DIM], const double (&b)[DIM]) {
#pragma clang fp contract(off)
  double dx = b[0] - a[0];
  double dy = b[1] - a[1];
  double s = dx * dx + dy * dy;
  if constexpr (DIM == 3) {
    double dz = b[2] - a[2];
    s = s + dz * dz;
  }
  return s;
}

// Team helpers: lanes of one team are contiguous (lane = row * TEAM + t).
__device__ inline int team_lane() { return threadIdx.x & (TEAM - 1); }

// Cross-lane moves through DPP (a source modifier of a VALU move: no LDS
// round trip, unlike a shuffle).  Lane-pattern controls of the GCN/CDNA DPP
// encoding used here: quad_perm [1,0,3,2] (lane ^ 1) = 0xB1, quad_perm
// [2,3,0,1] (lane ^ 2) = 0x4E, row_half_mirror (lane l <-> 7 - l within
// each 8 lanes) = 0x141, row_mirror (l <-> 15 - l within each 16) = 0x140.
// row_shl:k (lane l takes lane l + k within each 16) = 0x100 + k;
// row_bcast:15 (each row takes the last lane of the row before it) = 0x142,
// row_bcast:31 (rows 2 and 3 take lane 31) = 0x143.  The source lanes of
// these patterns must be active; a lane with no source reads 0 (bound_ctrl),
// so the destination needs no initial value (no extra move).
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;
constexpr int DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;
constexpr int DPP_SHL1 = 0x101, DPP_SHL2 = 0x102, DPP_SHL3 = 0x103, DPP_SHL4 = 0x104,
              DPP_SHL5 = 0x105, DPP_SHL6 = 0x106;

template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}
// The same restricted to the 16-lane rows in the mask ROWS; the other rows'
// results are undefined.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_u32_rows(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS>
__device__ inline double dpp_move_rows(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp_u32_rows<CTRL, ROWS>((uint32_t)b),
                 hi = dpp_u32_rows<CTRL, ROWS>((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}
template <int CTRL, class T>
__device__ inline T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte lanes");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = dpp_u32<CTRL>((uint32_t)b), hi = dpp_u32<CTRL>((uint32_t)(b >> 32));
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}
template <class T>
__device__ inline T read_lane(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}

// Sum over the 8 lanes of the team, valid in every lane of it: the
// butterfly ((l0 + l1) + (l2 + l3)) + ((l4 + l5) + (l6 + l7)), the same bits
// in all lanes (IEEE addition is commutative).
template <class T>
__device__ inline T team_sum(T v) {
  v += dpp_move<DPP_XOR1>(v);
  v += dpp_move<DPP_XOR2>(v);
  v += dpp_move<DPP_HALF_MIRROR>(v);
  return v;
}
template <class T>
__device__ inline T team_min(T v) {
  T w = dpp_move<DPP_XOR1>(v);
  v = w < v ? w : v;
  w = dpp_move<DPP_XOR2>(v);
  v = w < v ? w : v;
  w = dpp_move<DPP_HALF_MIRROR>(v);
  v = w < v ? w : v;
  return v;
}
// Sum over the wavefront in a fixed order (team sums, pairs of teams, then
// the four 16-lane rows ((r0 + r1) + (r2 + r3))), uniform result.  All 64
// lanes must be active.
template <class T>
__device__ inline T wave_sum(T v) {
  v = team_sum(v);
  v += dpp_move<DPP_MIRROR>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}
// The same sum valid in the last lane only (the bits of wave_sum): rows
// 1 and 3 add the last lane of the row before them (row_bcast:15), then row
// 3 adds the last lane of row 1 (row_bcast:31).  Rows 0 and 2 hold
// meaningless values afterwards.
__device__ inline double wave_sum_last(double v) {
  v = team_sum(v);
  v += dpp_move<DPP_MIRROR>(v);
  v += dpp_move_rows<DPP_BCAST15, 0xA>(v);
  v += dpp_move_rows<DPP_BCAST31, 0xC>(v);
  return v;
}
// Bit mask of the team's lanes for which pred holds (bit t = lane t).
__device__ inline uint32_t team_ballot(bool pred) {
  uint64_t m = __ballot(pred);
  int base = (threadIdx.x & (WAVE - 1)) & ~(TEAM - 1);
  return (uint32_t)((m >> base) & ((1u << TEAM) - 1));
}

// Sum over a row's matrix entries l, l + TEAM, ... < nnz (l = the team lane,
// or a later start on the same lane) of
// val(e) * x(col(e)), U entries per step so that U independent gathers are
// in flight per lane (the latency of the dependent index -> value load
// chain, not bandwidth, limits the SpMV); the order of the additions is
// fixed, so the result is reproducible.
template <int U, class VT, class F>
__device__ inline double row_dot(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                 int64_t row, int nnz, int kpad, int l, F&& x) {
  double s = 0.0;
  for (; l + (U - 1) * TEAM < nnz; l += U * TEAM) {
    const int64_t e0 = sl_index(row, l, kpad);
    int32_t j[U];
    double a[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = col[e0 + u * WAVE];
      a[u] = (double)val[e0 + u * WAVE];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x(j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) s += a[u] * xv[u];
  }
  for (; l < nnz; l += TEAM) {
    const int64_t e = sl_index(row, l, kpad);
    s += (double)val[e] * x(col[e]);
  }
  return s;
}

// 1/sqrt(x) for the kernel sums (x > 0): the hardware reciprocal square
// root, in FP64 refined by RSQ_NEWTON Newton-Raphson steps
// y <- y + y (1 - x y^2) / 2, which square the relative error, so that the
// result is within a few ulp (no correctly rounded sqrt and division).
#ifndef RSQ_NEWTON
#define RSQ_NEWTON 2
#endif
__device__ inline float rsqrt_k(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_k(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < RSQ_NEWTON; ++k) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// 1/x for the per-pair means of the two-phase sums (x > 0): the hardware
// reciprocal refined by two Newton-Raphson steps y <- y + y (1 - x y).
__device__ inline double rcp_k(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// The kernel weight (Eq. 4, or the cubic kernel) and its derivative from
// r^2 and ir = 1/r, zero at and beyond re (re2 = re^2).
template <class R>
__device__ inline R weight_r2(int kernel, R r2, R ir, R re, R re2) {
  if (!(r2 < re2)) return R(0);
  if (kernel == MPS_K_KOSHIZUKA) return re * ir - R(1);
  const R q = R(1) - r2 * ir / re;
  return q * q * q;
}
template <class R>
__device__ inline R dweight_r2(int kernel, R r2, R ir, R re, R re2) {
  if (!(r2 < re2)) return R(0);
  if (kernel == MPS_K_KOSHIZUKA) return -re * ir * ir;
  const R q = R(1) - r2 * ir / re;
  return R(-3) * q * q / re;
}

// Kernel weight (Eq. 4, or the cubic kernel), zero at and beyond re.
template <class R>
__device__ inline R weight(int kernel, R r, R re) {
  if (!(r < re)) return R(0);
  if (kernel == MPS_K_KOSHIZUKA) return re / r - R(1);
  R q = R(1) - r / re;
  return q * q * q;
}

// Kernel timing for the profiling mode: when a profiling scope around a
// single launch sets g_ext_timing, the launch goes through
// hipExtLaunchKernelGGL, whose events record the start and the end of that
// dispatch's execution (launch gaps excluded, as a kernel trace reports).
struct ExtTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;
};
extern thread_local ExtTiming* g_ext_timing;

template <class K, class... A>
inline void launch_k(K kernel, unsigned grid, unsigned block, hipStream_t s, A... args) {
  ExtTiming* et = g_ext_timing;
  if (et && !et->used) {
    et->used = true;
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, et->start, et->stop, 0u, args...);
  } else {
    kernel<<<grid, block, 0, s>>>(args...);
  }
}

// Parameter validation shared by the entry points (MPS_OK or MPS_E_ARG).
mps_status check_params(const mps_params* P, int64_t n);
// Text of the last error of a call made without a context (this thread).
const char* noctx_error();

// ---------------------------------------------------------------- launchers
int launch_bin(const View& v, int dim, hipStream_t s);
int launch_permute(const View& v, int dim, int precision, hipStream_t s);
int launch_neighbors(const View& v, int dim, int precision, hipStream_t s);
int launch_list_check(const View& v, int dim, hipStream_t s);
int launch_list_filter(const View& v, int dim, hipStream_t s);
int launch_list_force(const View& v, hipStream_t s);
int launch_export_lists(const View& v, int32_t* cell_out, int32_t* count_out,
                        int32_t* list_out, int dim, hipStream_t s);
// filter_kept: lists kept over steps, single phase -- the kernel also
// filters the superset into this step's exact lists (k_predict_keep), in
// place of launch_list_filter
int launch_predict(const View& v, int dim, int precision, bool filter_kept, hipStream_t s);
int launch_density(const View& v, int dim, int precision, int pmode, hipStream_t s);
int launch_viscosity(const View& v, int dim, int precision, hipStream_t s);
int launch_smooth_density(const View& v, const double* rho_raw, double* rho_out, int dim,
                          hipStream_t s);
int launch_assemble(const View& v, int dim, int precision, const double* rhs_sorted,
                    bool zero_x0, hipStream_t s);
int launch_cg_spmv(const View& v, int precision, hipStream_t s);
int launch_cg_update(const View& v, hipStream_t s);
int pcg_blocks(int64_t n, bool fused);
int pcg_fused_capacity(int precond);
int launch_pcg_setup(const View& v, int precision, int dim, hipStream_t s);
int launch_pcg_iter(const View& v, int precision, int parity, hipStream_t s);
int launch_pcg_reduce(const View& v, int parity, hipStream_t s);
// two-level preconditioner: the cell operator after the assembly, and
// target += P C P^T src on the pressure unknowns (restriction, Chebyshev
// steps, prolongation)
int launch_coarse_assemble(const View& v, int dim, int precision, hipStream_t s);
int launch_coarse_correct(const View& v, int dim, const double* src, double* target,
                          hipStream_t s);
int launch_gradient(const View& v, int dim, int precision, hipStream_t s);
int launch_scatter_orig(const View& v, const double* src, double* dst, int comps,
                        int stride, hipStream_t s);
int launch_gather_orig(const View& v, const double* src, double* dst, int comps,
                       int stride, hipStream_t s);
int launch_export_ppe(const View& v, int precision, double* diag, double* b,
                      int32_t* nnz, int32_t* cols, double* vals, hipStream_t s);
int cg_spmv_blocks(int64_t n);
// Workgroups of the assembly (its partials start the solve).
int assemble_blocks(int64_t n, bool pipelined);
int adj_partial_blocks(int64_t n);
int launch_adjoint_head(const View& v, const AdjView& a, int dim, int precision, int wc,
                        hipStream_t s);
int launch_adjoint_ppe(const View& v, const AdjView& a, int dim, hipStream_t s);
int launch_adjoint_tail(const View& v, const AdjView& a, int dim, hipStream_t s);
int cg_update_blocks(int64_t n);

}  // namespace mps
