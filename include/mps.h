/*
 * mps.h -- C ABI of the MI355X (gfx950) implementation of the data-parallel
 * hot path of the Moving Particle Semi-implicit (MPS) method, arXiv
 * 2105.01677, Section "The Moving Particle Semi-implicit Method".
 *
 * One time step (mps_step) is:
 *   1. cell-linked-list neighbour search (Section "Neighbouring search
 *      algorithms": cells with sides equal to the interaction radius, the
 *      list constant for the whole step; neighbour cap 300, Section "CUDA");
 *   2. explicit prediction with the viscous Laplacian (Eq. 7) and gravity;
 *   3. particle number density (Eq. 5) and free-surface flags (Eq. 15);
 *   4. pressure: the PPE (Eq. 13) assembled as a sparse symmetric matrix in
 *      the row-wise manner of the listing "PPE assemble GPU code" and solved
 *      by preconditioned conjugate gradients, or the equation of state
 *      (Eq. 16) of the weakly-compressible model;
 *   5. pressure gradient (standard MPS, or Eq. 18) and first-order Euler
 *      update.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (HIP), contiguous, in the caller's
 *    original particle order; vectors are row-major [n][dim] FP64.  The
 *    caller owns them; the library keeps no alias after the call returns.
 *  - Work is enqueued on the stream given to mps_init.  Calls that return
 *    host scalars (iteration counts, residuals, statistics) or a status
 *    detected on the device synchronise that stream before returning.
 *  - The library owns all its scratch memory, allocated once in mps_init
 *    (and mps_tape_alloc); mps_step and mps_pressure_solve make no device
 *    allocation of their own.  mps_step captures its stages into HIP graphs
 *    the first time a stage shape is needed (a few per context, cached until
 *    mps_free); instantiating one is left to the HIP runtime.
 *  - Every function returns an mps_status and never aborts or prints.
 *    Argument errors leave the context untouched.  A numerical error
 *    (NEIGH_OVERFLOW, COINCIDENT, NONFINITE) marks the context poisoned:
 *    further steps return MPS_E_POISONED until mps_set_state.
 *    mps_last_error gives a text description of the last error.
 *  - One context per stream; contexts are independent of each other.
 */
#ifndef MPS_H
#define MPS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_ctx mps_ctx; /* opaque, owned by the library */

typedef enum {
  MPS_OK = 0,
  MPS_E_ARG = -1,            /* invalid argument or parameter */
  MPS_E_NOMEM = -2,          /* device allocation failed */
  MPS_E_NEIGH_OVERFLOW = -3, /* a particle has more than max_neigh neighbours */
  MPS_E_CG_NOCONV = -4,      /* CG reached cg_maxit; last iterate kept */
  MPS_E_NONFINITE = -5,      /* NaN or Inf in positions or velocities */
  MPS_E_COINCIDENT = -6,     /* two particles at distance 0 (Eq. 4 diverges) */
  MPS_E_DEVICE = -7,         /* HIP runtime error */
  MPS_E_POISONED = -8,       /* an earlier numerical error; call mps_set_state */
  MPS_E_SCRATCH = -9         /* the input needs more than the fixed scratch of an
                                allocation-free entry point */
} mps_status;

/* Particle types (int8 per particle).  Wall particles are pressure unknowns
 * like fluid; dummy particles only complete the number density and the
 * viscous sums near walls (listing "PPE assemble GPU code": bcon == -1).
 * A particle that leaves the background grid becomes a GHOST and takes no
 * further part; the library sets this type itself. */
enum { MPS_FLUID = 0, MPS_WALL = 1, MPS_DUMMY = 2, MPS_GHOST = 3 };
/* Per-particle flags of the last step (int8). */
enum { MPS_FLAG_GHOST = -2, MPS_FLAG_DUMMY = -1, MPS_FLAG_INNER = 0, MPS_FLAG_SURFACE = 1 };
enum { MPS_PPE_CG = 0, MPS_WC_EOS = 1 };         /* pressure model */
enum { MPS_K_KOSHIZUKA = 0, MPS_K_CUBIC = 1 };   /* Eq. 4 / cubic kernel */
enum { MPS_FP64 = 0, MPS_MIXED = 1 };            /* precision of the path */
enum { MPS_GRAD_STD = 0, MPS_GRAD_CMPS = 1 };    /* standard / Eq. 18 */
/* PPE source term: (n* - n0)/(n0 dt^2) (Eq. 13); the higher-order source
 * from Dn/Dt at r*, u* (Eq. 21, MPS-HS); the same plus the error-compensating
 * parts of Eq. 24 (Eq. 25, ECS) */
enum { MPS_SRC_STD = 0, MPS_SRC_HS = 1, MPS_SRC_HS_ECS = 2 };
/* Laplacian of pressure in the PPE: Eq. 7, 2d/(lambda n0) sum_j p_ij w_ij;
 * or the higher-order form of Eq. 23 (MPS-HL), (1/n0) sum_j 2 r_e p_ij /
 * r_ij^3 over r_ij < re_lap (the printed equation lost the power of r_ij;
 * this one has the units of a Laplacian and, with the printed factor 2,
 * tends to the exact Laplacian of a quadratic field in two and three
 * dimensions as re_lap/l0 grows) */
enum { MPS_LAP_STD = 0, MPS_LAP_HL = 1 };
/* Preconditioner of the pipelined CG: the diagonal of A (Jacobi); or an
 * additive two-level preconditioner D^-1 + P C P^T, P the aggregation of
 * the pressure unknowns by background grid cell, C three Chebyshev steps on
 * the cell-level operator P^T A P (for the large systems the paper solves
 * by ICCG: same solution, fewer iterations); or one damped Neumann step
 * of block Jacobi, D^-1 - 1.5 D^-1 (A_B - D) D^-1 with A_B the diagonal
 * blocks of A over runs of 64 consecutive cell-sorted rows (symmetric
 * positive definite for the PPE matrices; applied inside the one-kernel
 * iteration, so only for systems whose 64-row groups are all resident on
 * the device at once: up to 49,152 particles on MI355X; larger systems get
 * MPS_E_ARG at mps_init).  Either non-Jacobi choice needs cg_pipelined = 1
 * and pmode = MPS_PPE_CG (else MPS_E_ARG). */
enum { MPS_PC_JACOBI = 0, MPS_PC_TWO_LEVEL = 1, MPS_PC_BLOCK = 2 };

typedef struct {
  int32_t dim;              /* 2 or 3 */
  int32_t pmode;            /* MPS_PPE_CG or MPS_WC_EOS */
  int32_t kernel;           /* MPS_K_KOSHIZUKA or MPS_K_CUBIC */
  int32_t precision;        /* MPS_FP64, or MPS_MIXED: FP32 neighbour sums and
                               matrix values on cell-relative FP32 positions,
                               FP64 diagonal, right-hand side, CG vectors,
                               dot products and pressure */
  int32_t grad;             /* MPS_GRAD_STD or MPS_GRAD_CMPS */
  int32_t clamp_negative_p; /* 1: p <- max(p, 0) after the pressure step */
  int32_t max_neigh;        /* neighbour cap, 1..1024 (the paper uses 300) */
  int32_t cg_maxit;         /* CG iteration limit */
  int32_t grid_n[3];        /* background grid cells per axis (1 for unused) */
  int32_t cg_pipelined;     /* 0: CG with two kernels (two reductions) per
                               iteration; 1: pipelined CG, one kernel and one
                               reduction per iteration (same solution) */
  double l0;                /* initial particle spacing (m) */
  double re_n;              /* radius for number density, flags, gradient (m) */
  double re_lap;            /* radius for the Laplacian (viscous, PPE) (m) */
  double rho;               /* density (kg/m^3) */
  double nu;                /* kinematic viscosity (m^2/s) */
  double g[3];              /* body acceleration (m/s^2) */
  double dt;                /* time step (s) */
  double beta;              /* free-surface threshold (Eq. 15), 0.97 */
  double c0;                /* speed of sound of the equation of state (m/s) */
  double gamma;             /* exponent of Eq. 16, a positive integer (7) */
  double alpha;             /* artificial compressibility on the PPE diagonal,
                               alpha/dt^2 (1e-7) */
  double cg_tol;            /* stop when ||b - A p|| <= cg_tol ||b|| */
  double grid_lo[3];        /* lower corner of the background grid (m) */
  double cell_size;         /* cell side, >= re_lap (m) */
  double smagorinsky_cs;    /* Smagorinsky constant Cs of the sub-particle-scale
                               eddy viscosity (0 = off; 0.12 typical) */
  int32_t source;           /* MPS_SRC_*: PPE source term (PPE model only;
                               the adjoint needs MPS_SRC_STD) */
  int32_t laplacian;        /* MPS_LAP_*: Laplacian of pressure in the PPE
                               (PPE model only; the adjoint needs
                               MPS_LAP_STD) */
  double skin;              /* 0: neighbour lists built every step.  > 0
                               (m, below re_lap; cell_size >= re_lap + skin):
                               lists kept over steps - a superset at radius
                               re_lap + skin is built with a fresh cell sort
                               and filtered every step to the exact list;
                               it is rebuilt when a particle has moved
                               skin/2 since the build or left the grid.  The
                               lists are the same sets; only the order of
                               the particles and of the list entries, hence
                               the rounding of the sums, differs.  A
                               superset row beyond 1.2 max_neigh ((re_lap +
                               skin)/re_lap)^dim entries is reported as
                               MPS_E_NEIGH_OVERFLOW.  The adjoint needs 0. */
  int32_t precond;          /* MPS_PC_*: preconditioner of the CG (the
                               two-level one needs cg_pipelined = 1) */
} mps_params;

typedef struct {
  int32_t steps;           /* steps taken by the call */
  int32_t cg_iters_last;   /* CG iterations of the last step (PPE mode) */
  int64_t cg_iters_total;  /* CG iterations summed over the call */
  double cg_relres_last;   /* ||b - A p|| / ||b|| of the last step */
  int64_t n_surface;       /* free-surface particles after the last step */
  int64_t n_ghost;         /* ghost particles */
  int64_t list_entries;    /* neighbour-list entries of the last step */
  int64_t ppe_nnz;         /* off-diagonal matrix entries of the last step */
  int32_t cg_redone;       /* steps whose speculative solve (see mps_step)
                              did not converge and that were redone */
  int32_t list_builds;     /* steps that built their neighbour lists with a
                              cell sort (all of them when skin = 0) */
  int64_t short_entries;   /* entries within re_n at the predicted positions
                              r* (Eq. 5), the lists that p-hat and the
                              pressure gradient walk, of the last step */
} mps_step_stats;

/* Kernel classes for mps_profile: cell binning + sort + permutation (a1),
 * neighbour lists (a2), viscous prediction (a3), number density / flags /
 * equation of state (a4), PPE assembly (a5), the two CG kernels (a6) and
 * the pressure gradient + update (a8). */
enum {
  MPS_KC_SORT = 0, MPS_KC_NEIGH, MPS_KC_PREDICT, MPS_KC_DENSITY, MPS_KC_ASSEMBLE,
  MPS_KC_CG_SPMV, MPS_KC_CG_UPDATE, MPS_KC_GRADIENT, MPS_KC_COUNT
};

/* Create a context for n particles.  pos, vel: [n][dim] FP64; type: [n]
 * int8 (MPS_FLUID, MPS_WALL or MPS_DUMMY).  rho_i, nu_i: [n] per-particle
 * density and laminar kinematic viscosity, or NULL for params->rho / nu.
 * Any of them, or smagorinsky_cs > 0, selects the two-phase / turbulence
 * model (Section "Fluid flow models"): each particle carries a smoothed
 * density <rho>_i = sum_j rho_j w / sum_j w over non-dummy neighbours
 * (re_n), computed here once; the viscous term uses the harmonic mean of
 * the dynamic viscosities mu = <rho>(nu_i + nu_t) with the Smagorinsky
 * eddy viscosity nu_t = (Cs l0)^2 sqrt(2 S:S) (Eq. for tau/rho with the
 * k term absorbed into the pressure); the PPE coupling uses
 * 2/(<rho>_i + <rho>_j) and the update 1/<rho>_i.
 * hip_stream is a hipStream_t (NULL = default stream; step stages are then
 * launched one by one instead of as HIP graphs).
 * Errors: MPS_E_ARG (bad parameters: dim, radii, grid, cap, n < 1, gamma
 * not integer), MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_init(const mps_params* params, int64_t n, const double* pos,
                    const double* vel, const int8_t* type, const double* rho_i,
                    const double* nu_i, void* hip_stream, mps_ctx** out);

/* Release every resource of the context (NULL is allowed). */
mps_status mps_free(mps_ctx* ctx);

/* Text of the last error of the context (static storage; never NULL); for
 * ctx = NULL, that of this thread's last call made without a context. */
const char* mps_last_error(const mps_ctx* ctx);

/* Build the neighbour lists at the current positions (step 1) and export
 * them in original order.  cell_id: [n] linear cell index
 * (x fastest, -1 for ghosts) or NULL; count: [n]; list: [n][max_neigh]
 * ascending original ids, padded with -1.  The set is exactly
 * { j != i : d2 < re_lap^2 } with d2 = (dx*dx + dy*dy) + dz*dz rounded term
 * by term in FP64 (dx = x_j - x_i), over particles that are not ghosts.
 * Errors: MPS_E_NEIGH_OVERFLOW, MPS_E_COINCIDENT, MPS_E_POISONED; after an
 * error the outputs are unspecified. */
mps_status mps_neighbors(mps_ctx* ctx, int32_t* cell_id, int32_t* count,
                         int32_t* list);

/* Allocation-free variant of mps_neighbors, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same cell sort and neighbour lists,
 * for n particles at positions the caller passes, without a context.  No
 * device or host allocation is made: the work arrays are carved out of a
 * fixed device array of MPS_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU
 * holds from the library's load until the process ends (its address is
 * looked up once per device on the first call there).
 * params: as for mps_init (only dim, l0, radii, grid and max_neigh are
 * used); pos: [n][dim] FP64, type: [n] int8 (MPS_FLUID..MPS_GHOST), device
 * pointers, read only.  cell_id, count, list: outputs as for mps_neighbors
 * (device pointers, each may be NULL).  hip_stream: hipStream_t (NULL = the
 * default stream); the call synchronises it to read the status.
 * Work needed: about n (16 ps + 30 + 4 kpad) bytes (ps = 2 in 2-D, 4 in
 * 3-D; kpad = max_neigh rounded up to 8) plus 12 bytes per cell; e.g. the
 * 44,832-particle 2-D dam break at max_neigh = 300 takes 57 MB.
 * Every call on one GPU uses that GPU's one array: concurrent calls on the
 * same GPU (other streams or threads) race and must be serialised by the
 * caller; a call leaves its data in the array, and clears what must start
 * at zero itself.
 * Errors: MPS_E_ARG (parameters, NULL pos/type, a type outside
 * MPS_FLUID..MPS_GHOST), MPS_E_SCRATCH (n, max_neigh and the grid need more
 * than the fixed array; nothing is launched), MPS_E_NEIGH_OVERFLOW,
 * MPS_E_COINCIDENT, MPS_E_NONFINITE, MPS_E_DEVICE; after an error the
 * outputs are unspecified.  mps_last_error(NULL) gives the text of this
 * thread's last such error. */
#define MPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mps_status mps_neighbors_noalloc(const mps_params* params, int64_t n, const double* pos,
                                 const int8_t* type, int32_t* cell_id, int32_t* count,
                                 int32_t* list, void* hip_stream);

/* Advance nsteps time steps (steps 1-5 above).  stats may be NULL.
 * PPE model on a non-null stream: each step after the first is enqueued
 * whole with a CG iteration count guessed from the previous steps, and the
 * next step is enqueued before the previous one's solve is checked; a step
 * whose solve did not converge within its count is redone from its input
 * with polled CG batches, the step after it discarded (same results;
 * counted in stats->cg_redone).
 * A numerical error (NEIGH_OVERFLOW, COINCIDENT, NONFINITE) raised in the
 * k-th step of the call ends the call there: stats->steps = k - 1 steps
 * were completed, and the context's state (mps_get_state) is the failing
 * step's input; no step behind it writes state.
 * Errors: MPS_E_NEIGH_OVERFLOW, MPS_E_COINCIDENT, MPS_E_NONFINITE,
 * MPS_E_CG_NOCONV (the step still completes with the last iterate),
 * MPS_E_POISONED. */
mps_status mps_step(mps_ctx* ctx, int32_t nsteps, mps_step_stats* stats);

/* Run steps 1-3 and the PPE assembly (Eq. 13, listing "PPE assemble GPU
 * code") at the current state without advancing it, then solve A p = rhs
 * by CG from p = 0.  rhs: [n] in original order, or NULL for the PPE source
 * b_i = (n*_i - n0)/(n0 dt^2); entries of rows that are not pressure
 * unknowns (free surface, dummy, ghost) are ignored and their p is 0.
 * p: [n] output (device), the unclamped solution.  iters, relres: host
 * pointers or NULL.  The state is unchanged.  Errors as mps_step. */
mps_status mps_pressure_solve(mps_ctx* ctx, const double* rhs, double* p,
                              int32_t* iters, double* relres);

/* Export the system assembled by the last mps_step (PPE mode) or
 * mps_pressure_solve, in original order: diag [n], b [n], nnz [n]
 * off-diagonal entries per row, cols/vals [n][max_neigh] (original column
 * ids and FP64 values, row order unspecified).  Any pointer may be NULL.
 * Errors: MPS_E_ARG if no system has been assembled. */
mps_status mps_get_ppe(mps_ctx* ctx, double* diag, double* b, int32_t* nnz,
                       int32_t* cols, double* vals);

/* Export the state in original order; any pointer may be NULL.
 * pos, vel: [n][dim]; p: [n] pressure of the last step; n_star: [n] number
 * density of the last step (at the predicted positions); flags: [n]
 * (MPS_FLAG_*); type: [n]. */
mps_status mps_get_state(mps_ctx* ctx, double* pos, double* vel, double* p,
                         double* n_star, int8_t* flags, int8_t* type);

/* Replace positions and velocities (original order, [n][dim]); types are
 * kept unless type is non-NULL.  Clears a poisoned context. */
mps_status mps_set_state(mps_ctx* ctx, const double* pos, const double* vel,
                         const int8_t* type);

/* Device memory held by the context (state, work arrays, tape), bytes.
 * Host pointer.  Errors: MPS_E_ARG. */
mps_status mps_device_bytes(const mps_ctx* ctx, int64_t* bytes);

/* Two-phase model: smoothed density <rho> and Smagorinsky eddy viscosity
 * nu_t of the last step, [n] each in original order (device; either may be
 * NULL).  Errors: MPS_E_ARG for a single-phase context. */
mps_status mps_get_phase(mps_ctx* ctx, double* rho_s, double* nu_t);

/* The lattice constants the context uses: n0 for re_n and re_lap, lambda
 * for re_lap (Eq. 5 and the weighted mean of r^2 of Eq. 7 at an interior
 * particle of the initial lattice).  Host pointers, any may be NULL. */
mps_status mps_constants(const mps_ctx* ctx, double* n0_n, double* n0_lap,
                         double* lambda_lap);

/* ------------------------------------------------------------ adjoint
 * Reverse-mode derivative of the step (hand-written adjoint kernels), for
 * gradients of a loss on a final state with respect to the viscosity nu,
 * the body acceleration g and the initial velocities.  Lists, free-surface
 * flags, the p-hat argmin and the clamp masks of each step are frozen.  In
 * the PPE model the adjoint of the pressure solve is the transposed solve
 * A lambda = x-bar, run with the same CG kernels (A is symmetric).  The
 * standard pressure gradient is supported (grad = MPS_GRAD_STD), in the
 * single-phase and in the two-phase + Smagorinsky model (then nu_bar is
 * the derivative with respect to a common shift of the per-particle
 * laminar viscosities, and the reverse of the eddy viscosity, of the
 * harmonic-mean pair viscosities and of the per-particle densities is
 * included; the smoothed densities are constants).
 * Typical use (checkpointing every K steps): save a slot every K steps in
 * the forward run; for each segment in reverse, load its checkpoint,
 * re-run the K steps saving each step's input state, then walk back with
 * mps_tape_load + mps_step_adjoint. */

/* Allocate nslots state slots (positions, velocities, pressure, types of
 * the context's particle storage) and the adjoint work arrays.  Frees any
 * previous tape.  Errors: MPS_E_ARG, MPS_E_NOMEM. */
mps_status mps_tape_alloc(mps_ctx* ctx, int32_t nslots);

/* Copy the current state into / from a slot (stream-ordered, no sync); a
 * load also restores the slot's particle order of the two-phase densities
 * and viscosities.  Errors: MPS_E_ARG (bad slot, or loading a slot never
 * saved). */
mps_status mps_tape_save(mps_ctx* ctx, int32_t slot);
mps_status mps_tape_load(mps_ctx* ctx, int32_t slot);

/* Adjoint of one step taken from the CURRENT state (r^k, u^k): given the
 * cotangents pos_bar, vel_bar of the step's output (r^{k+1}, u^{k+1}),
 * returns those of its input in pos_bar_prev, vel_bar_prev (device,
 * original order, [n][dim] FP64; may not alias the inputs) and this step's
 * contributions to dL/dnu (*nu_bar, host) and dL/dg (g_bar[dim], host);
 * either may be NULL.  Recomputes the step's forward stages first; the
 * state is not advanced.  Every pressure option has an adjoint: either
 * Laplacian (Eq. 7 or the HL form of Eq. 23), each source (Eq. 13, HS of
 * Eq. 21, HS + ECS of Eq. 24-25) and either gradient (standard or Eq. 18).
 * Errors: MPS_E_ARG (no tape; lists kept with a skin, which have no
 * adjoint), the errors of mps_step. */
mps_status mps_step_adjoint(mps_ctx* ctx, const double* pos_bar, const double* vel_bar,
                            double* pos_bar_prev, double* vel_bar_prev, double* nu_bar,
                            double* g_bar);

/* Per-kernel timing: when bit k of class_mask is set, every launch of
 * kernel class k (MPS_KC_*) is bracketed by a pair of HIP events on the
 * context's stream and its duration accumulated (the CG kernels, launched
 * one per scope, record the events from their own dispatch, so their time
 * excludes launch gaps).  A profiling aid for
 * roofline measurements; a mask of 0 switches it off.  Resets the totals.
 * Errors: MPS_E_DEVICE if events cannot be created. */
mps_status mps_profile(mps_ctx* ctx, uint32_t class_mask);

/* Accumulated milliseconds and launch counts per kernel class since the
 * last mps_profile call (host arrays of MPS_KC_COUNT entries, or NULL).
 * Synchronises the stream. */
mps_status mps_profile_read(mps_ctx* ctx, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* MPS_H */
