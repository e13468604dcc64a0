/*
 * MPS oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of one time step of the Moving
 * Particle Semi-implicit method (Koshizuka & Oka; as restated in Section
 * "The Moving Particle Semi-implicit Method" of arXiv 2105.01677).  It exists
 * to check the HIP implementation; only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the HIP library and must never be linked into it.
 *
 * Pins (tests/test_oracle_pins.py): each function is checked against
 * closed forms, brute force, library routines or invariants.  Parity
 * unpinned: multi-step dam-break trajectories (orc_run) beyond a few dozen
 * steps, which are chaotic; the tests compare them over 20 steps only (the
 * smooth water drop over 300).
 *
 * Every array is in original particle order, row-major [n][dim], FP64.
 * Particle types: 0 fluid, 1 wall, 2 dummy, 3 ghost (left the grid).
 * Flags: -2 ghost, -1 dummy, 0 inner, 1 free surface.
 */
#ifndef MPS_ORACLE_H
#define MPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim, pmode, kernel, grad, clamp, max_neigh, cg_maxit;
  int32_t grid_n[3];
  double l0, re_n, re_lap, rho, nu, g[3], dt, beta, c0, gamma, alpha, cg_tol;
  double grid_lo[3], cell_size, smag_cs;
  int32_t source; /* PPE source: 0 Eq. 13, 1 Eq. 21 (HS), 2 Eq. 25 (HS + ECS) */
  int32_t laplacian; /* PPE Laplacian: 0 Eq. 7, 1 Eq. 23 (HL) */
  /* PPE solve: 0 CG from p = 0 to a relative residual of 1e-13 (the
   * reference for parity checks); 1 CG from the previous step's pressure to
   * cg_tol, the stopping rule of the GPU path (for timing the oracle on the
   * same work per step; needs orc_run, which keeps the pressure) */
  int32_t cg_warm;
} orc_params;

/* Every pointer may be NULL (that output is skipped).  list/aval are
 * [n][max_neigh]: row i holds count[i] ascending neighbour ids, then -1/0. */
typedef struct {
  int32_t *cell, *count, *list;
  double *us, *rs, *nstar;
  int8_t *flags;
  double *diag, *b, *aval;
  double *p, *phat, *gradp;
  double *nut;
  double *pos, *vel;
  int8_t *type;
  int32_t cg_iters;
  double cg_relres;
} orc_step_out;

/* Lattice constants n0 and lambda (Eq. 5 and the weighted mean of r^2 used
 * by Eq. 7) of an interior particle of a square (dim 2) or cubic (dim 3)
 * lattice of spacing l0, for radius re and kernel (0 Eq. 4, 1 cubic). */
int orc_lattice_constants(int dim, double l0, double re, int kernel,
                          double* n0, double* lambda, int32_t* count);

/* Kernel weight w(r) for radius re (Eq. 4 / cubic kernel). */
double orc_weight(int kernel, double r, double re);

/* Neighbour lists by the definition: all j != i, neither a ghost, with
 * d^2 < re_lap^2.  Returns 0, -3 (more than max_neigh) or -6 (coincident). */
int orc_neighbors_brute(const orc_params* P, int64_t n, const double* pos,
                        const int8_t* type, int32_t* count, int32_t* list);
/* The same lists through the cell-linked list of Section "Neighbouring
 * search algorithms" (cells of side cell_size, own + adjacent cells). */
int orc_neighbors_cells(const orc_params* P, int64_t n, const double* pos,
                        const int8_t* type, int32_t* cell, int32_t* count,
                        int32_t* list);

/* One time step.  flags_override (may be NULL) replaces the free-surface
 * decision (used when a flag sits on the n* = beta n0 tie). */
int orc_step(const orc_params* P, int64_t n, const double* pos,
             const double* vel, const int8_t* type, const int8_t* flags_override,
             const double* rho_s, const double* nu_i, orc_step_out* out);

/* nsteps time steps; state arrays are updated in place.  rho_s (smoothed
 * density) and nu_i (laminar viscosity) per particle select the two-phase
 * model (NULL: single phase with P->rho, P->nu).  p_out, flags_out: the last
 * step's pressure and flags (or NULL); with P->cg_warm, p_out also brings
 * in the pressure of the step before the first (the first solve's start).
 * cg_iters_out: CG iterations summed over the steps (or NULL). */
int orc_run(const orc_params* P, int64_t n, double* pos, double* vel,
            int8_t* type, int32_t nsteps, const double* rho_s, const double* nu_i,
            double* p_out, int8_t* flags_out, int64_t* cg_iters_out);

/* Smoothed density of the two-phase model, fixed before the run. */
int orc_smoothed_density(const orc_params* P, int64_t n, const double* pos,
                         const int8_t* type, const double* rho_i, double* rho_s);

/* p-hat and the pressure gradient (standard or Eq. 18) of a given pressure
 * field p at positions rs, lists taken at rs. */
int orc_pressure_gradient(const orc_params* P, int64_t n, const double* rs,
                          const int8_t* type, const double* p, double* phat,
                          double* gradp);

/* p-hat, the pressure gradient of a given pressure field p at rs and the
 * first-order Euler update from the predicted state (rs, us): the last part
 * of the step on its own.  rho_s (may be NULL): smoothed densities of the
 * two-phase model.  pos_out, vel_out: [n][dim]. */
int orc_pressure_update(const orc_params* P, int64_t n, const double* rs,
                        const double* us, const int8_t* type, const double* p,
                        const double* rho_s, double* pos_out, double* vel_out);

/* Loss after nsteps (w_ke * mean fluid kinetic energy + w_var * variance of
 * the free-surface height) and its forward-mode derivatives along d/dnu,
 * d/dg_x and <d/du0, dir>: out[4] = {L, dL/dnu, dL/dgx, <dL/du0, dir>}.
 * rho_s, nu_i (may be NULL): the two-phase model's smoothed densities and
 * laminar viscosities; d/dnu is then the derivative with respect to a shift
 * of every particle's laminar viscosity by the same amount. */
int orc_rollout_grad(const orc_params* P, int64_t n, const double* pos,
                     const double* vel, const int8_t* type, int32_t nsteps,
                     const double* dir, double w_ke, double w_var, const double* rho_s,
                     const double* nu_i, double* out);
/* The same loss of a given final state and last-step flags. */
double orc_loss(const orc_params* P, int64_t n, const double* pos,
                const double* vel, const int8_t* type, const int8_t* flags,
                double w_ke, double w_var);
/* Host threads of the OpenMP loops (n >= 1); returns the count in effect. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
