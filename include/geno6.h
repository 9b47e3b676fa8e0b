/*
 * geno6.h - C ABI of the sixth-order non-compact finite-volume scheme in one
 * dimension with GENO reconstruction (Zhao & Xu, "A generalized ENO
 * reconstruction in compact GKS for compressible flow simulations",
 * Sec. 4.1), the HLLC Riemann flux and the classical four-stage fourth-order
 * Runge-Kutta method (the non-compact pairing named in Sec. 2), for gfx950.
 *
 * Method. At every face x_{j+1/2} each conservative variable is
 * reconstructed on both sides from the averages of cells j-2..j+3:
 *   R = chi p^5 + (1 - chi) sum_k w_k p_k          (Sec. 4.1, Eq. (3))
 * with p^5 the quintic of the six-cell stencil S_0, p_1, p_2 the quadratics
 * of S_1 = {j-2, j-1, j}, S_2 = {j-1, j, j+1}, p_3, p_4 the cubics of
 * S_3 = {j-1..j+2}, S_4 = {j..j+3} (the right-side state mirrors every
 * stencil about the face); IS_k of Jiang-Shu type on the target cell
 * (Eq. (6)); chi = tanh(C alpha)/tanh(C) (Eq. (4)); alpha from
 * IS^tau = |(IS_1 + IS_3)/2 - IS_2|, IS^H = max IS_k, IS^L = min IS_k with
 * r = 2 (Eq. (5), (7), (9)); w_k ~ d_k / (IS_k + eps)^2 (Eq. (8)).
 * A side state with rho <= 0, p <= 0 or a non-finite entry is replaced by
 * its target cell's average (guard). The HLLC flux uses the wave speeds
 * S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L, u_R + a_R).
 *
 * Conventions (shared with geno_gks.h: error codes GENO_*, boundary codes
 * GENO_BC_*, geno_last_error, geno_stats).
 * Pointers: U, L, UL, UR, F, chi, ws, dt_out are DEVICE pointers owned by
 *   the caller; structs are HOST pointers. Every call only enqueues work on
 *   `stream` (hipStream_t as void*, NULL = default stream), allocates
 *   nothing, and synchronises only when a geno_stats pointer is given.
 * State layout: SoA float64 U[field][pitch], fields (rho, rho U, rho E),
 *   cell i (0 <= i < n) of field f at f * pitch + i; pitch from
 *   geno6_grid_init (n rounded up to a multiple of 64; the padding is never
 *   read). Boundary ghost cells are formed inside the kernels from the
 *   interior values (no ghost storage).
 * Face arrays: [field][n + 1] with face s between cells s-1 and s.
 */
#ifndef GENO6_H
#define GENO6_H

#include <stddef.h>

#include "geno_gks.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GENO6_ABI_VERSION 3

/* fixed-state ends of this path (the GENO_BC_FIXED code of geno_gks.h):
 * the three ghost cells of an end hold the states of geno6_params.ghost
 * (inflow, or a fixed profile) */
#define GENO6_BC_FIXED GENO_BC_FIXED

/* variables the reconstruction works on (the GENO_VARS_* codes) */
#define GENO6_VARS_CONSERVATIVE GENO_VARS_CONSERVATIVE
#define GENO6_VARS_CHARACTERISTIC GENO_VARS_CHARACTERISTIC

/* Method parameters.
 * gamma: ratio of specific heats (> 1).
 * C, eps: path-function steepness and indicator floor of Eq. (4), (5), (8)
 *   (the paper: 20 and 1e-15).
 * d: linear weights of S_1..S_4 in Eq. (8); the paper boosts the central
 *   sub-stencil by C_0 = 8: d = (1, 8, 1, 1), S_2 being the one centred on
 *   the target cell. All must be > 0.
 * cfl: dt = cfl * dx / max over cells of (|u| + a), taken from the state at
 *   the start of each step (the paper runs with CFL >= 0.5; default 0.5).
 * bc: low and high end (GENO_BC_PERIODIC on both or neither;
 *   GENO_BC_TRANSMISSIVE copies the end cell; GENO_BC_REFLECTING mirrors
 *   the cells with the momentum negated; GENO6_BC_FIXED takes the states of
 *   `ghost`).
 * ghost: conserved states (rho, rho U, rho E) of the three ghost cells of
 *   each end for GENO6_BC_FIXED: ghost[0][k] is cell -1-k, ghost[1][k] is
 *   cell n+k (k = 0 next to the grid). Unused for the other kinds.
 * dt_fixed: if > 0, every step uses this dt instead of the CFL condition.
 * variables: GENO6_VARS_CONSERVATIVE (default) reconstructs rho, rho U,
 *   rho E component by component; GENO6_VARS_CHARACTERISTIC projects the
 *   stencil's states on the left eigenvectors of the Euler flux Jacobian at
 *   the Roe average of the two cells at the face, reconstructs the three
 *   characteristic fields and maps both face states back with the right
 *   eigenvectors (a face whose Roe average has no real sound speed keeps
 *   the conservative variables). The paper does not say which variables it
 *   reconstructs. */
typedef struct geno6_params {
  int version;
  double gamma;
  double C;
  double eps;
  double d[4];
  double cfl;
  int bc[2];
  double dt_fixed;
  int variables;
  double ghost[2][3][3];
} geno6_params;

typedef struct geno6_grid {
  int n;           /* cells (>= 3) */
  int pitch;       /* elements per field row (n rounded up to 64) */
  double x0, x1, dx;
  geno6_params params;
} geno6_grid;

/* Defaults: gamma 1.4, C 20, eps 1e-15, d (1, 8, 1, 1), cfl 0.5, periodic,
 * dt_fixed 0, conservative variables. */
int geno6_params_default(geno6_params* p);

/* Fills *g for n uniform cells on [x0, x1] and copies *p. GENO_EINVAL for
 * n < 3, n too large for 32-bit indexing, x1 <= x0 or bad parameters;
 * GENO_EVERSION for a params version other than GENO6_ABI_VERSION. */
int geno6_grid_init(geno6_grid* g, int n, double x0, double x1, const geno6_params* p);

/* Bytes of the device workspace of geno6_step (control block, 1024 slots of
 * wave-speed maxima and three stage arrays of 3 * pitch doubles). */
size_t geno6_workspace_bytes(const geno6_grid* g);

/* Reconstruction and flux at every face s = 0..n (Sec. 4.1 and the HLLC
 * flux): UL, UR the guarded left and right states, F the HLLC flux, each
 * [3][n + 1]; chi (may be NULL) the path function of every side and
 * variable (characteristic field with GENO6_VARS_CHARACTERISTIC) before the
 * guard, [side(2)][3][n + 1]. Any of UL, UR, F may be NULL. */
int geno6_faces(const geno6_grid* g, const double* U, double* UL, double* UR, double* F,
                double* chi, void* stream);

/* Semi-discrete right-hand side L = -(F_{j+1/2} - F_{j-1/2}) / dx of every
 * cell, L in the state layout. */
int geno6_rhs(const geno6_grid* g, const double* U, double* L, void* stream);

/* nsteps classical Runge-Kutta steps of U in place:
 *   k_1 = L(U), k_2 = L(U + dt/2 k_1), k_3 = L(U + dt/2 k_2),
 *   k_4 = L(U + dt k_3), U <- U + dt (k_1 + 2 k_2 + 2 k_3 + k_4) / 6,
 * dt from the CFL condition on U at the start of the step (computed on the
 * device; the host never waits between steps) unless dt_fixed > 0.
 * ws: geno6_workspace_bytes(g) bytes of device memory.
 * dt_out (device, may be NULL): nsteps doubles, the step sizes.
 * stats (host, may be NULL): if given, the call waits for the stream and
 *   fills guard (side states replaced) and nonfinite (cells with a
 *   non-finite value, rho <= 0 or p <= 0 after a step, summed over the
 *   steps) and last_dt; it then returns GENO_ENONPHYS if nonfinite > 0. */
int geno6_step(const geno6_grid* g, double* U, void* ws, int nsteps, double* dt_out,
               geno_stats* stats, void* stream);

/* ---- many small grids ----------------------------------------------------
 * The paper's 1-D problems have 200 to 1800 cells, far too few to fill the
 * GPU: one launch per stage is then latency-bound. geno6_step_batch advances
 * ngrids grids of the same geometry and parameters (different states) by
 * nsteps steps in ONE launch: one work-group per grid (1024 lanes; 512 with
 * characteristic variables) runs all steps and stages (each grid keeps its
 * own CFL time step), with the stage arithmetic of geno6_step in the same
 * order, so each grid's result equals geno6_step on that grid alone, bit for
 * bit. Intended for small grids (the work-group sweeps its grid in passes of
 * 1023, resp. 511, cells).
 * U (device): ngrids states one after the other, each in the layout above
 *   (3 * pitch doubles), advanced in place.
 * ws: geno6_batch_workspace_bytes(g, ngrids) bytes (control block and three
 *   stage arrays per grid).
 * dt_out (device, may be NULL): [ngrids][nsteps] step sizes.
 * stats: as geno6_step (counts summed over the grids; last_dt of grid 0). */
#define GENO6_BATCH_MAX 65535
size_t geno6_batch_workspace_bytes(const geno6_grid* g, int ngrids);
int geno6_step_batch(const geno6_grid* g, int ngrids, double* U, void* ws, int nsteps,
                     double* dt_out, geno_stats* stats, void* stream);

/* Kernel kinds of geno6_step and geno6_step_batch for the timing hooks. */
enum {
  GENO6_K_INIT = 0,   /* wave-speed maxima of the initial state */
  GENO6_K_DT,         /* time step of a step from the maxima (one work-group) */
  GENO6_K_STAGE,      /* one Runge-Kutta stage: GENO on both sides of every
                         face, HLLC, flux difference and the stage combination
                         (the last stage also forms the next maxima) */
  GENO6_K_SMALL,      /* geno6_step_batch: all steps of all grids */
  GENO6_NKERNELS
};

/* Per-kernel timing of geno6_step, as geno_timing_enable / geno_timing_read
 * of geno_gks.h (events bound to each kernel's dispatch; not thread-safe). */
int geno6_timing_enable(int max_launches);
int geno6_timing_read(int nkinds, double* ms_total, long long* launches);

/* Floating-point operations (add, sub, mul, div, sqrt and each exp count 1)
 * as the device functions execute them, host array of 3: costs[0] one face
 * of a stage whose six sides keep chi = 1 (both sides of the three
 * variables with their indicators, guard tests, HLLC); costs[1] the extra
 * work of one side with chi < 1 (exponential, low-order weights, blend);
 * costs[2] one cell (flux difference and stage combination, averaged over
 * the four stages). */
int geno6_op_costs(double* costs);

#ifdef __cplusplus
}
#endif

#endif /* GENO6_H */
