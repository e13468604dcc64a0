// Cell-linked-list neighbour search (Section "Neighbouring search
// algorithms" of arXiv 2105.01677): particles are binned into a fixed
// background grid of cells with side cell_size >= re_lap, counting-sorted by
// cell, and each particle's list is gathered from its own and the adjacent
// cells.  The list is built once per step and kept for the whole step.
//
// Order of the sorted particles: by linear cell id, and inside a cell by
// original particle id, so that the layout -- and every floating-point sum
// over a list -- is independent of the order in which atomics resolved.
// Sorting = cell of each particle + atomic slot (k_bin), exclusive scan of
// the cell counts inside tiles of cells (k_scan_tiles), tile offsets and
// unordered scatter (k_scatter), rank inside the cell and permutation of the
// state (k_rank_permute).
#include "mps_internal.h"

namespace mps {

// With lists kept over steps, the cell sort and the superset search run
// only in the steps whose decision kernel asked for a build.
__device__ inline bool skip_build(const View& v) { return v.ls && !v.ls->rebuild; }

// The neighbour criterion d2 < re_lap^2 is evaluated on dist2_exact
// (mps_internal.h: rounded term by term, (dx*dx + dy*dy) + dz*dz), so the
// lists are reproducible bit for bit on any IEEE machine.

// a1: cell of every particle (current sorted order), rank inside its cell.
// A particle outside the grid becomes a ghost and goes to cell ncell.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_bin(View v, int8_t* type_cur) {
  if (skip_build(v)) return;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool active = i < v.n;
  int c = v.ncell;
  if (active) {
    int8_t t = type_cur[i];
    if (t != MPS_GHOST) {
      double x[DIM];
      load_vec<DIM>(v.pos, i, x);
      const int nn[3] = {v.nx, v.ny, v.nz};
      int ci[3] = {0, 0, 0};
      bool in = true, finite = true;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        finite = finite && isfinite(x[a]);
        double f = floor((x[a] - v.lo[a]) * v.inv_cs);
        if (!(f >= 0.0 && f < (double)nn[a])) in = false;
        else ci[a] = (int)f;
      }
      if (!finite) atomicOr(v.status, ST_NONFINITE);
      if (in) c = ci[0] + v.nx * (ci[1] + v.ny * ci[2]);
      else type_cur[i] = MPS_GHOST;
    }
    v.cellid[i] = c;
  }
  // one atomic per run of consecutive lanes in the same cell (the input is
  // the previous step's cell order, so runs are long): the run's first
  // lane adds the run length, the others take consecutive slots after it
  const int lane = threadIdx.x & (WAVE - 1);
  const int cprev = __shfl_up(c, 1, WAVE);
  const bool head = active && (lane == 0 || cprev != c);
  const uint64_t heads = __ballot(head);
  const int nact = __popcll(__ballot(active));
  const uint64_t upto = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t hb = heads & upto;
  const int h = hb ? 63 - __clzll(hb) : 0;
  const uint64_t after = heads & ~upto;
  const int next = after ? __ffsll((unsigned long long)after) - 1 : nact;
  int base = 0;
  if (head) base = atomicAdd(&v.cell_count[c], next - lane);
  base = __shfl(base, h, WAVE);
  if (active) v.slot[i] = base + (lane - h);
}

// Exclusive scan of the cell counts inside each tile of SCAN_TILE cells,
// one workgroup per tile (a thread scans SCAN_PER consecutive counts, then
// the workgroup its thread totals), and the tile's total; resets the counts
// for the next step.  The arrays are padded to whole tiles (padding counts
// stay 0) and cover ncell + 2 cells, so the start of cell ncell + 1 comes
// out as the total.
__global__ __launch_bounds__(SCAN_NT) void k_scan_tiles(View v) {
  if (skip_build(v)) return;
  constexpr int NW = SCAN_NT / WAVE, Q = SCAN_PER / 4;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  __shared__ int32_t wsum[NW];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
  const int4* src = reinterpret_cast<const int4*>(v.cell_count + base);
  int4 q[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) q[k] = src[k];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k) s += (q[k].x + q[k].y) + (q[k].z + q[k].w);
  int32_t inc = s;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += y;
  }
  if (lane == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  int32_t run = inc - s, total = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int32_t x = wsum[k];
    run += k < w ? x : 0;
    total += x;
  }
  int4* dst = reinterpret_cast<int4*>(v.cell_local + base);
  int4* cnt = reinterpret_cast<int4*>(v.cell_count + base);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    int4 o;
    o.x = run;
    run += q[k].x;
    o.y = run;
    run += q[k].y;
    o.z = run;
    run += q[k].z;
    o.w = run;
    run += q[k].w;
    dst[k] = o;
    cnt[k] = make_int4(0, 0, 0, 0);
  }
  if (threadIdx.x == 0) v.tile_sum[blockIdx.x] = total;
}

// Thread i scatters particle i (if i < n) to its cell's start + its atomic
// slot, and writes the start of cell i (if i < ncell + 2).  A start is the
// in-tile start plus the sum of the earlier tiles' totals, which every
// wavefront scans itself, 64 tiles at a time (one pass up to 262,144 cells).
__global__ __launch_bounds__(BLOCK) void k_scatter(View v) {
  if (skip_build(v)) return;
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int lane = threadIdx.x & (WAVE - 1);
  const bool part = i < v.n, cell = i < (int64_t)v.ncell + 2;
  const int c = part ? v.cellid[i] : 0;
  const int tp = c / SCAN_TILE, tc = cell ? (int)(i / SCAN_TILE) : 0;
  const int32_t lp = part ? v.cell_local[c] : 0, lc = cell ? v.cell_local[i] : 0;
  int32_t bp = 0, bc = 0, carry = 0;
  for (int g0 = 0; g0 < v.ntile; g0 += WAVE) {
    const int g = g0 + lane;
    const int32_t x = g < v.ntile ? v.tile_sum[g] : 0;
    int32_t inc = x;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int32_t y = __shfl_up(inc, o, WAVE);
      if (lane >= o) inc += y;
    }
    const int32_t ex = carry + inc - x;
    const int32_t ep = __shfl(ex, (tp - g0) & (WAVE - 1), WAVE);
    const int32_t ec = __shfl(ex, (tc - g0) & (WAVE - 1), WAVE);
    if (tp >= g0 && tp < g0 + WAVE) bp = ep;
    if (tc >= g0 && tc < g0 + WAVE) bc = ec;
    carry += __shfl(inc, WAVE - 1, WAVE);
  }
  if (part) v.perm[lp + bp + v.slot[i]] = (int32_t)i;
  if (cell) v.cell_start[i] = lc + bc;
}

// Final position of every particle and the permutation of the state in one
// pass (skipped once an error has been raised): inside its cell a particle's rank is the number of cell members with
// a smaller original id (cells hold a few tens of particles, read from the
// unordered scatter in perm), so the order does not depend on how the
// counting atomics resolved.  Ghosts keep their atomic slot: they take part
// in no sum.  Packed cell coordinates and, on the mixed path, FP32
// positions relative to the cell's lower corner are written alongside.
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_rank_permute(View v) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  // after an error raised earlier in this call no step writes state any
  // more, so the failing step's input buffer survives the steps enqueued
  // behind it
  if (i >= v.n || *v.status) return;
  const int32_t key = v.id[i];
  // a step that keeps the lists keeps the order: a plain copy into the
  // next buffer, with the cell each particle was binned in at the build
  const bool build = !skip_build(v);
  int64_t k;
  int32_t pc = GHOST_CELL;
  if (build) {
    const int c = v.cellid[i];
    const int b = v.cell_start[c];
    if (c == v.ncell) {
      k = b + v.slot[i];
    } else {
      const int e = v.cell_start[c + 1];
      int rank = 0;
      // four members per step, all loads issued before the compares (a
      // member past the cell end is read as the cell's first and not counted)
      for (int m = b; m < e; m += 4) {
        int32_t pm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pm[u] = v.perm[m + u < e ? m + u : b];
#pragma unroll
        for (int u = 0; u < 4; ++u) rank += (m + u < e && v.id[pm[u]] < key) ? 1 : 0;
      }
      k = b + rank;
      pc = pack_cell(c % v.nx, (c / v.nx) % v.ny, c / (v.nx * v.ny));
    }
  } else {
    k = i;
    pc = v.pcell[i];
  }
  double x[DIM], u[DIM] = {};
  load_vec<DIM>(v.pos, i, x);
  store_vec<DIM>(v.pos_w, k, x);
  // velocity and pressure are absent for a search of positions alone
  if (v.vel) {
    load_vec<DIM>(v.vel, i, u);
    store_vec<DIM>(v.vel_w, k, u);
  }
  v.type_w[k] = v.type[i];
  v.id_w[k] = key;
  if (v.p_in) v.p_w[k] = v.p_in[i];
  if (v.rho_s) {
    v.rho_s_w[k] = v.rho_s[i];
    v.nu_l_w[k] = v.nu_l[i];
  }
  int ci[3] = {0, 0, 0};
  if (pc != GHOST_CELL) {
    ci[0] = ucx(pc);
    ci[1] = ucy(pc);
    ci[2] = ucz(pc);
  }
  v.pcell[k] = pc;
  if (build && v.r_build) store_vec<DIM>(v.r_build, k, x);
  if constexpr (MIXED) {
    float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < DIM; ++a) r[a] = (float)(x[a] - (v.lo[a] + ci[a] * v.cs));
    float4 f;
    if constexpr (DIM == 2) f = make_float4(r[0], r[1], __int_as_float(pc), 0.f);
    else f = make_float4(r[0], r[1], r[2], __int_as_float(pc));
    v.posf[2 * k] = f;
    v.posf[2 * k + 1] = make_float4((float)u[0], (float)u[1], DIM == 3 ? (float)u[2] : 0.f, 0.f);
  }
}

// Wavefront-uniform loads through the constant address space: the arrays
// read this way are not written while the search runs, so the compiler may
// (and does) use scalar loads for them.
template <class T>
__device__ inline T ld_uniform(const T* a, int64_t i) {
  typedef const __attribute__((address_space(4))) T cT;
  return ((const cT*)a)[i];
}
template <int DIM>
__device__ inline void load_vec_uniform(const double* a, int64_t i, double (&x)[DIM]) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) x[k] = ld_uniform(a, PS<DIM>::v * i + k);
}

// a2: neighbour lists, one wavefront per group of SLICE consecutive sorted
// particles (the rows of one slice of the list layout).  The particles of a
// cell share their candidates: the 3 (2-D) or 9 (3-D) grid rows x-1 .. x+1
// of the 3^DIM block around the cell, each one contiguous index range of
// the sorted order.  The group is taken one cell at a time (a group spans
// one or two cells, rarely more); the wavefront lays that cell's ranges end
// to end, loads WAVE candidates at a time (one per lane) and tests each of
// the group's particles in the cell against them.  A particle's position is
// uniform (scalar loads), its hits are compacted with a wavefront ballot and
// appended in candidate order, so a list comes out in the same order as a
// per-particle scan of the ranges, and its list length is a uniform
// register.  Each candidate position is loaded once per group and cell
// instead of once per particle; the groups follow the particle order, so
// the XCD-aware block mapping splits the work evenly.  The particles are
// tested NBU at a time (their distance chains are independent) before their
// hits are appended.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_neighbors(View v) {
  // after an error raised earlier in the call the permutation wrote nothing,
  // so the packed cells need not match this step's cell starts: no search
  if (skip_build(v) || *v.status) return;
  constexpr int NR = DIM == 3 ? 9 : 3;  // cell rows of the 3^DIM block
  constexpr int G = SLICE;
  constexpr int NBU = 2;  // particles tested per pass (independent chains)
  static_assert(G == 8 && TEAM == 8 && WAVE == 64, "slot arithmetic below");
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t g0 = ((int64_t)xcd_block() * (BLOCK / WAVE) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE))) * G;
  if (g0 >= v.n) return;
  const int ng = (int)min((int64_t)G, v.n - g0);
  // row u of the group starts at slot u * TEAM of its slice
  int32_t* const gb = v.nb_list + (g0 / SLICE) * ((int64_t)v.kpad * SLICE);
  const double re2 = v.re_lap2;
  const unsigned maxn = (unsigned)v.max_neigh;
  int cnt[G];
#pragma unroll
  for (int u = 0; u < G; ++u) cnt[u] = 0;
  uint64_t coinc = 0;
  int s = 0;  // first row of the group not yet done
  while (s < ng) {
    const int32_t pc = ld_uniform(v.pcell, g0 + s);
    if (pc == GHOST_CELL) break;  // ghosts are sorted last: no neighbours
    const int cx = ucx(pc), cy = ucy(pc), cz = ucz(pc);
    const int c = cx + v.nx * (cy + v.ny * cz);
    // the run of the group in cell c (at least one row: progress even if
    // the cells were inconsistent)
    const int se = max(s + 1, (int)min((int64_t)ng, (int64_t)ld_uniform(v.cell_start, c + 1) - g0));
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, v.nx - 1);
    // the ranges end to end: candidate k of range q is particle k + dlt[q]
    int pre[NR], dlt[NR], total = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int y = cy - 1 + q % 3, z = DIM == 3 ? cz - 1 + q / 3 : 0;
      const bool in = y >= 0 && y < v.ny && z >= 0 && z < v.nz;
      const int base = v.nx * ((in ? y : cy) + v.ny * (in ? z : cz));
      const int jb = ld_uniform(v.cell_start, base + x0);
      const int je = in ? ld_uniform(v.cell_start, base + x1 + 1) : jb;
      pre[q] = total;
      dlt[q] = jb - total;
      total += je - jb;
    }
    for (int k0 = 0; k0 < total; k0 += WAVE) {
      const int k = k0 + lane;
      int d = dlt[0];
#pragma unroll
      for (int q = 1; q < NR; ++q) d = k >= pre[q] ? dlt[q] : d;
      const bool valid = k < total;
      const int j = valid ? k + d : (int)g0;
      double xj[DIM];
      load_vec<DIM>(v.pos, j, xj);
      // a lane past the ranges sits at infinity and never hits
#pragma unroll
      for (int a = 0; a < DIM; ++a) xj[a] = valid ? xj[a] : __builtin_inf();
#pragma unroll
      for (int u0 = 0; u0 < G; u0 += NBU) {
        bool in[NBU];
        bool any = false;
#pragma unroll
        for (int w = 0; w < NBU; ++w) {
          in[w] = u0 + w >= s && u0 + w < se;
          any = any || in[w];
        }
        if (!any) continue;
        double d2[NBU];
        bool hit[NBU];
        uint64_t m[NBU];
#pragma unroll
        for (int w = 0; w < NBU; ++w) {
          // a particle outside the cell's run tests a clamped one, no hit
          const int i = (int)g0 + min(max(u0 + w, s), se - 1);
          double xi[DIM];
          load_vec_uniform<DIM>(v.pos, i, xi);
          d2[w] = dist2_exact<DIM>(xi, xj);
          hit[w] = in[w] && j != (int)g0 + u0 + w && d2[w] < re2;
          m[w] = __builtin_amdgcn_ballot_w64(hit[w]);
        }
#pragma unroll
        for (int w = 0; w < NBU; ++w) {
          const int u = u0 + w;
          if (m[w]) {
            coinc |= __builtin_amdgcn_ballot_w64(hit[w] && d2[w] == 0.0);
            if (hit[w]) {
              const unsigned l = (unsigned)cnt[u] + __builtin_amdgcn_mbcnt_hi(
                                     (uint32_t)(m[w] >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m[w], 0u));
              // slot l of row u: (l / TEAM) * WAVE + u * TEAM + l % TEAM
              if (l < maxn) gb[(((l << 3) & ~63u) | (l & 7u)) + u * TEAM] = j;
            }
            cnt[u] += __popcll(m[w]);
          }
        }
      }
    }
    s = se;
  }
  int my = 0;
#pragma unroll
  for (int u = 0; u < G; ++u) my = lane == u ? cnt[u] : my;
  if (lane < ng) {
    if (my > (int)maxn) {
      atomicOr(v.status, ST_OVERFLOW);
      my = (int)maxn;
    }
    v.nb_count[g0 + lane] = my;
  }
  if (coinc && lane == 0) atomicOr(v.status, ST_COINCIDENT);
}

// Lists kept over steps, start of a step: the largest squared
// displacement of a particle since the build (positions are in the build's
// order until the next build), infinite if a particle has left the grid or
// is not finite; one maximum per workgroup (no atomics: device-scope
// atomics on one address serialise across the chip).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_list_check(View v) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  double d2 = 0.0;
  if (i < v.n && v.type[i] != MPS_GHOST) {
    double x[DIM], xb[DIM];
    load_vec<DIM>(v.pos, i, x);
    load_vec<DIM>(v.r_build, i, xb);
    const int nn[3] = {v.nx, v.ny, v.nz};
    bool force = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double f = floor((x[a] - v.lo[a]) * v.inv_cs);
      if (!(f >= 0.0 && f < (double)nn[a])) force = true;  // also NaN
      const double d = x[a] - xb[a];
      d2 += d * d;
    }
    if (force || !(d2 < 1e300)) d2 = __builtin_inf();
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) d2 = fmax(d2, __shfl_xor(d2, o, WAVE));
  __shared__ double sh[BLOCK / WAVE];
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int k = 1; k < BLOCK / WAVE; ++k) m = fmax(m, sh[k]);
    v.red_blk[blockIdx.x] = m;
  }
}

// The decision of the step (one workgroup over the workgroup maxima):
// build when forced or when a particle has moved skin/2 or more since the
// build (then no pair that is closer than re_lap now was farther than
// re_lap + skin then).
constexpr int DECIDE_NT = 1024;
__global__ __launch_bounds__(DECIDE_NT) void k_list_decide(View v, int nblk) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += DECIDE_NT) m = fmax(m, v.red_blk[b]);
  for (int o = WAVE / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
  __shared__ double sh[DECIDE_NT / WAVE];
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < DECIDE_NT / WAVE; ++k) m = fmax(m, sh[k]);
  ListState* ls = v.ls;
  const int rb = ls->force || !(m < v.half_skin2);
  ls->rebuild = rb;
  ls->since = rb ? 0 : ls->since + 1;
  ls->builds += rb;
  ls->force = 0;
}

// The exact list of every particle from its superset row: the members with
// d2 < re_lap^2 at the step's positions, d2 by the same term-by-term FP64
// expression as the cell search, in the superset's order (one team per
// particle, ballot compaction).  FILT_U entries per lane and step: their
// position gathers are in flight together while the next step's superset
// entries load (slot indices past the row clamped to its first slot).
#ifndef FILT_U
#define FILT_U 4
#endif
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_list_filter(View v) {
  constexpr int U = FILT_U;
  const int64_t row = (int64_t)xcd_block() * ROWS_PER_BLOCK + threadIdx.x / TEAM;
  const int t = team_lane();
  if (row >= v.n) return;
  const int cs = v.sk_count[row];
  double xi[DIM];
  load_vec<DIM>(v.pos, row, xi);
  const int64_t s0 = sl_index(row, t, v.kpad_s), e0 = sl_index(row, 0, v.kpad);
  const int ng = v.kpad_s / TEAM;
  int32_t jn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) jn[u] = v.sk_list[s0 + (int64_t)(u < ng ? u : 0) * WAVE];
  int count = 0;
  bool coinc = false;
  for (int k0 = 0; t + k0 * TEAM < cs; k0 += U) {
    int32_t j[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      in[u] = t + (k0 + u) * TEAM < cs;
      j[u] = in[u] ? jn[u] : (int32_t)row;
    }
    double xj[U][DIM];
#pragma unroll
    for (int u = 0; u < U; ++u) load_vec<DIM>(v.pos, j[u], xj[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + U + u;
      jn[u] = v.sk_list[s0 + (int64_t)(k < ng ? k : 0) * WAVE];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double d2 = dist2_exact<DIM>(xi, xj[u]);
      const bool hit = in[u] && d2 < v.re_lap2;
      coinc = coinc || (hit && d2 == 0.0);
      const uint32_t m = team_ballot(hit);
      if (hit) {
        const unsigned q = (unsigned)(count + __popc(m & ((1u << t) - 1u)));
        if (q < (unsigned)v.max_neigh)
          v.nb_list[e0 + (int64_t)(q / TEAM) * WAVE + (q % TEAM)] = j[u];
      }
      count += __popc(m);
    }
  }
  if (coinc) atomicOr(v.status, ST_COINCIDENT);
  if (count > v.max_neigh) {
    if (t == 0) atomicOr(v.status, ST_OVERFLOW);
    count = v.max_neigh;
  }
  if (t == 0) v.nb_count[row] = count;
}

__global__ void k_list_force(ListState* ls) {
  if (threadIdx.x == 0) ls->force = 1;
}

// Export: lists in original order with original ids, ascending; the cell
// of every particle at its current position (as the binning computes it:
// with lists kept over steps the particles keep the cells of the last
// build between builds).
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_export_lists(View v, int32_t* cell_out,
                                                        int32_t* count_out,
                                                        int32_t* list_out) {
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  // nothing is exported after an error (the lists may not have been built)
  if (k >= v.n || *v.status) return;
  const int64_t o = v.id[k];
  const int c = v.nb_count[k];
  if (count_out) count_out[o] = c;
  if (cell_out) {
    int cell = -1;
    if (v.type[k] != MPS_GHOST) {
      double x[DIM];
      load_vec<DIM>(v.pos, k, x);
      const int nn[3] = {v.nx, v.ny, v.nz};
      int ci[3] = {0, 0, 0};
      bool in = true;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double f = floor((x[a] - v.lo[a]) * v.inv_cs);
        if (!(f >= 0.0 && f < (double)nn[a])) in = false;
        else ci[a] = (int)f;
      }
      if (in) cell = ci[0] + v.nx * (ci[1] + v.ny * ci[2]);
    }
    cell_out[o] = cell;
  }
  if (!list_out) return;
  int32_t* row = list_out + o * v.max_neigh;
  for (int l = 0; l < c; ++l) {
    const int32_t key = v.id[v.nb_list[sl_index(k, l, v.kpad)]];
    int m = l - 1;
    while (m >= 0 && row[m] > key) {
      row[m + 1] = row[m];
      --m;
    }
    row[m + 1] = key;
  }
  for (int l = c; l < v.max_neigh; ++l) row[l] = -1;
}

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

int launch_bin(const View& v, int dim, hipStream_t s) {
  // type is binned in the current buffer (ghosts are marked in place)
  int8_t* type_cur = const_cast<int8_t*>(v.type);
  if (dim == 2) k_bin<2><<<nblk(v.n, BLOCK), BLOCK, 0, s>>>(v, type_cur);
  else k_bin<3><<<nblk(v.n, BLOCK), BLOCK, 0, s>>>(v, type_cur);
  k_scan_tiles<<<v.ntile, SCAN_NT, 0, s>>>(v);
  k_scatter<<<std::max(nblk(v.n, BLOCK), nblk((int64_t)v.ncell + 2, BLOCK)), BLOCK, 0, s>>>(v);
  return 0;
}

int launch_permute(const View& v, int dim, int precision, hipStream_t s) {
  const unsigned nb = nblk(v.n, BLOCK);
  if (dim == 2) {
    if (precision == MPS_MIXED) k_rank_permute<2, true><<<nb, BLOCK, 0, s>>>(v);
    else k_rank_permute<2, false><<<nb, BLOCK, 0, s>>>(v);
  } else {
    if (precision == MPS_MIXED) k_rank_permute<3, true><<<nb, BLOCK, 0, s>>>(v);
    else k_rank_permute<3, false><<<nb, BLOCK, 0, s>>>(v);
  }
  return 0;
}

int launch_neighbors(const View& v, int dim, int precision, hipStream_t s) {
  (void)precision;
  const unsigned nb = nblk(v.n, BLOCK / WAVE * SLICE);
  if (dim == 2) k_neighbors<2><<<nb, BLOCK, 0, s>>>(v);
  else k_neighbors<3><<<nb, BLOCK, 0, s>>>(v);
  return 0;
}

int launch_list_check(const View& v, int dim, hipStream_t s) {
  const unsigned nb = nblk(v.n, BLOCK);
  if (dim == 2) k_list_check<2><<<nb, BLOCK, 0, s>>>(v);
  else k_list_check<3><<<nb, BLOCK, 0, s>>>(v);
  k_list_decide<<<1, DECIDE_NT, 0, s>>>(v, (int)nb);
  return 0;
}

int launch_list_filter(const View& v, int dim, hipStream_t s) {
  const unsigned nb = nblk(v.n, ROWS_PER_BLOCK);
  if (dim == 2) k_list_filter<2><<<nb, BLOCK, 0, s>>>(v);
  else k_list_filter<3><<<nb, BLOCK, 0, s>>>(v);
  return 0;
}

int launch_list_force(const View& v, hipStream_t s) {
  k_list_force<<<1, 64, 0, s>>>(v.ls);
  return 0;
}

int launch_export_lists(const View& v, int32_t* cell_out, int32_t* count_out,
                        int32_t* list_out, int dim, hipStream_t s) {
  if (dim == 2) k_export_lists<2><<<nblk(v.n, BLOCK), BLOCK, 0, s>>>(v, cell_out, count_out, list_out);
  else k_export_lists<3><<<nblk(v.n, BLOCK), BLOCK, 0, s>>>(v, cell_out, count_out, list_out);
  return 0;
}

}  // namespace mps
