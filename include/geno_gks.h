/*
 * geno_gks.h - C ABI of the MI355X (gfx950) library for the compact
 * gas-kinetic scheme with GENO reconstruction (Zhao & Xu, "A generalized ENO
 * reconstruction in compact GKS for compressible flow simulations").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers. Arrays named W, dW, face_state, chi, F, Ft, Wint, ws are DEVICE
 *   pointers owned by the caller (the library never frees them). Structs
 *   (geno_params, geno_grid, geno_stats) are HOST pointers.
 * Streams. `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream). Every call only enqueues work on that stream and returns; the
 *   library allocates nothing and synchronises nothing, except gks_step when a
 *   geno_stats pointer is given (it then waits for the stream to read the
 *   counters back).
 * Errors. Every call returns 0 (GENO_OK) or a negative code; no exception
 *   crosses the ABI. geno_last_error() returns a thread-local message for the
 *   last failure on the calling thread.
 * Layout of the state. Structure of arrays, planar
 *   [field][row][column] with NG = 2 ghost cells on every side of the grid:
 *   element (field f, interior row j in [-2, ny+2), interior column i in
 *   [-2, nx+2)) sits at index (f * rows + (j + 2)) * pitch + (i + 2), where
 *   pitch and rows come from geno_grid_init (1-D: rows = 1, j = 0 only).
 *   Fields: 1-D W = (rho, rhoU, rhoE) and dW = (d/dx of each);
 *           2-D W = (rho, rhoU, rhoV, rhoE) and dW = (d/dx of the four
 *           fields, then d/dy of the four fields).
 *   dW holds physical cell-averaged gradients (not scaled by the cell size).
 *   Element types: W is float64 in every precision mode. dW, face_state,
 *   F, Ft and Wint are float64 with GENO_F64 and float32 with GENO_MIXED;
 *   chi is float64 in both.
 *   Ghost cells belong to the library: calls overwrite them (except those
 *   of GENO_BC_FIXED ends, which the caller fills); interior cells are
 *   written only by gks_step.
 */
#ifndef GENO_GKS_H
#define GENO_GKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GENO_ABI_VERSION 5

/* error codes */
#define GENO_OK 0
#define GENO_EINVAL (-1)     /* null pointer, bad size, unsupported parameter */
#define GENO_EVERSION (-2)   /* geno_params.version != GENO_ABI_VERSION */
#define GENO_EHIP (-3)       /* a HIP runtime call failed */
#define GENO_ENONPHYS (-4)   /* non-physical state found when stats were read */

/* boundary conditions (per side) */
#define GENO_BC_PERIODIC 0
#define GENO_BC_TRANSMISSIVE 1
#define GENO_BC_REFLECTING 2   /* wall: mirror image, normal momentum negated */
#define GENO_BC_FIXED 3        /* 1-D only: the caller's ghost cells of W and dW
                                  (two per end, averages and physical
                                  gradients) are kept as given: an inflow
                                  state or a fixed profile; the library never
                                  writes them and carries them into its
                                  stage arrays */

/* variables of the normal reconstruction */
#define GENO_VARS_CONSERVATIVE 0
#define GENO_VARS_CHARACTERISTIC 1

/* arithmetic of the reconstruction and the flux */
#define GENO_F64 0     /* everything in float64 */
#define GENO_MIXED 1   /* reconstruction, tangential step and gas-kinetic flux in
                          float32, and dW and the face buffers stored in float32;
                          the small-eps divisions of the smoothness indicators
                          (Eq. (5), (8)), the time-fit coefficients of the flux,
                          the conservative update of W, the stored stage
                          combination and dt stay in float64 */

/* Method parameters.
 * C, eps, r, rL, d: GENO constants of Sec. 3 (Eq. (4), (5), (8)): the paper
 *   uses C = 20, eps = 1e-15, r = 2 on structured meshes, r^L = 2 and the
 *   central sub-stencil weight C_0 = 8, i.e. d = (1, 8, 1) for the 8th-order
 *   compact stencils S_1, S_2, S_3 of Sec. 4.2. This library implements
 *   r = rL = 2 only (other values give GENO_EINVAL).
 * gamma: ratio of specific heats.
 * tau_c1, tau_c2: collision time of the BGK flux,
 *   tau = tau_c1 dt + tau_c2 dt |p_l - p_r| / (p_l + p_r).
 * cfl: dt = cfl * min over interior cells of min(dx/(|U|+c), dy/(|V|+c)).
 * bc: x-low, x-high, y-low, y-high (GENO_BC_*); periodic must be set on both
 *   sides of an axis.
 * dt_fixed: if > 0, every step of gks_step uses this dt instead of the CFL
 *   condition (the default is 0).
 * eps_ulps: GENO_MIXED only. float32 face values and the gradients formed
 *   from their differences carry rounding of several units in the last place,
 *   and with eps = 1e-15 the indicators of that noise read as discontinuities.
 *   The mixed form therefore uses eps + (eps_ulps * 2^-24 * qmax)^2 in Eq. (5)
 *   and (8), qmax the largest |value| of the stencil (0 gives the plain eps).
 *   In a run, the float32 fluxes also leave rounding of about one unit in the
 *   last place per step in W (dt/dx times the rounding of F), which
 *   accumulates over the steps; the default is 64.
 *   The same bound sets where the mixed flux takes tau = C1 dt: a Gauss point
 *   whose |p_l - p_r| / (p_l + p_r) is at most eps_ulps * 2^-24 (rounding
 *   noise of the two reconstructed states) is evaluated in that limit. The
 *   terms this drops are of order that ratio times the relative difference
 *   of the states or of h |grad W| / |W|, below the float32 unit roundoff.
 * variables: GENO_VARS_CONSERVATIVE (default) reconstructs the conserved
 *   variables component by component; GENO_VARS_CHARACTERISTIC projects the
 *   averages and h-scaled normal gradients of the four stencil cells of the
 *   normal step on the left eigenvectors of the Euler flux Jacobian along
 *   the face normal at the Roe average of the two cells at the face,
 *   reconstructs the characteristic fields (values and derivatives: three in
 *   1-D; four in 2-D, the speeds un - c, un, un (shear), un + c) and maps both
 *   face states back with the right eigenvectors (a face whose Roe average
 *   has no real sound speed keeps the conservative variables). The 2-D
 *   tangential step then works on the conservative face values. The paper
 *   does not say which variables it reconstructs. Not combined with the
 *   learned gate (GENO_EINVAL), whose network predicts conservative chi.
 * gate_delta: learned gate (2-D gks_step only). If > 0, once per step, on
 *   the state at its start, the loaded network (geno_mlp_load) predicts chi
 *   of every cell and direction from its stencil; where the prediction is
 *   >= 1 - gate_delta the cell's two face-sides of that direction take
 *   chi = 1 (the linear reconstruction) without forming the smoothness
 *   indicators, in both stages of the step; elsewhere plain GENO decides.
 *   0 (default) = off. */
typedef struct geno_params {
  int version;
  int precision;   /* GENO_F64 or GENO_MIXED */
  double gamma;
  double C;
  double eps;
  double r;
  double rL;
  double d[3];
  double tau_c1;
  double tau_c2;
  double cfl;
  int bc[4];
  double dt_fixed;
  double eps_ulps;
  double gate_delta;
  int variables;   /* GENO_VARS_* */
  int fuse;        /* 2-D gks_step (and the batched form): whether the normal
                      step runs inside the face kernels, one per direction,
                      so that the face-row values stay on chip (fused), or as
                      a launch of its own that writes them to the workspace.
                      Bitwise the same results. 1 (default): automatic, fused
                      when the launch has enough work-groups to fill the
                      device (4096 tiles; about a 512^2 grid) and not for
                      characteristic variables in the mixed form (both
                      measured faster the other way); 2: always fused; 0:
                      never. Work counting always takes the separate launch. */
} geno_params;

/* Grid description filled by geno_grid_init. */
typedef struct geno_grid {
  int ndim;        /* 1 or 2 */
  int nx, ny;      /* interior cells (ny = 1 in 1-D) */
  int pitch;       /* elements per padded row (>= nx + 4, multiple of 16) */
  int rows;        /* padded rows per field (ny + 4 in 2-D, 1 in 1-D) */
  double x0, x1, y0, y1;
  double dx, dy;
  geno_params params;
} geno_grid;

/* Counters returned by gks_step when asked for. */
typedef struct geno_stats {
  long long guard;      /* point states replaced by their cell average (rho<=0, p<=0 or non-finite) */
  long long nonfinite;  /* non-physical interior cells (non-finite, rho <= 0 or p <= 0) summed
                           over the steps of the call */
  double last_dt;       /* time step of the last step */
} geno_stats;

/* Library ABI version (GENO_ABI_VERSION). */
int geno_abi_version(void);

/* Thread-local message of the last failed call ("" if none). */
const char* geno_last_error(void);

/* Default parameters: the paper's GENO constants (Sec. 3), gamma = 1.4,
 * tau_c1 = 0, tau_c2 = 1, cfl = 0.5, transmissive boundaries, FP64. */
int geno_params_default(geno_params* p);

/* Fills *g for an ndim-dimensional uniform grid of nx (x ny) cells on
 * [x0, x1] (x [y0, y1]); copies *p. GENO_EINVAL for sizes < 1 (1-D: ny is
 * ignored), inverted intervals or unsupported parameters. */
int geno_grid_init(geno_grid* g, int ndim, int nx, int ny, double x0, double x1,
                   double y0, double y1, const geno_params* p);

/* Number of elements of one state array (W: nv fields; dW: ndim * nv); the
 * element type follows the precision mode (see the layout above). */
size_t geno_state_elems(const geno_grid* g, int nfields);

/* Bytes of the device workspace needed by gks_step / gks_flux. */
size_t gks_workspace_bytes(const geno_grid* g);

/* GENO reconstruction (Sec. 3, Eq. (3)-(9); 8th-order compact stencils of
 * Sec. 4.2, Eq. (13)-(14)) on every face of direction dir (0: x, 1: y; 1-D:
 * 0) after filling the ghost cells of W and dW in place.
 * face_state (device, caller-allocated): per face, per Gauss point, per side,
 *   the reconstructed state at the point after the positivity guard:
 *   [side(2)][gauss(G)][quant(Q)][var(nv)][nfy][nfx] elements with
 *   1-D: G = 1, Q = 2 (value, h * d/dn), nfy = 1, nfx = nx + 1;
 *   2-D: G = 2 (the points +-h/(2 sqrt 3) about the face centre, the
 *        negative tangential offset first), Q = 3 (value, h * d/dn,
 *        h * d/dt), x-faces nfy = ny, nfx = nx + 1; y-faces nfy = ny + 1,
 *        nfx = nx. Face (a, b) of x lies between cells (b-1, a) and (b, a);
 *        of y between (b, a-1) and (b, a). Side 0 = the lower-index cell.
 *   h is the cell size along the normal (d/dn) or the tangent (d/dt).
 *   Variables stay in the (x, y) frame.
 *   Followed by the second derivatives of the points that the time stepping
 *   of the gradients uses (the mean over the two sides; zero at a point with
 *   a guarded side): [gauss(G)][quant2(Q2)][var][nfy][nfx] with
 *   1-D: Q2 = 1 (h^2 d2/dn2, the GENO blend of Eq. (3) applied to the
 *        second derivatives of p^7 and of the sub-stencil quadratics);
 *   2-D: Q2 = 3 (h_n^2 d2/dn2 of the face-row; h_n h_t d2/dndt = chi_t
 *        (psi_{t+1} - psi_{t-1})/2 from the h-scaled normal derivatives psi
 *        of the rows t-1, t+1; h_t^2 d2/dt2 = chi_t (phi_{t+1} - 2 phi_t +
 *        phi_{t-1}) from the face-row values phi, chi_t the weight of the
 *        tangential step). In all (2 G Q + G Q2) nv planes.
 * chi (device, may be NULL): path function of the normal reconstruction per
 *   [side][var][row][face] over the rows the tangential step reads:
 *   1-D 1 x (nx+1); x-faces (ny+2) x (nx+1) (rows -1..ny); y-faces
 *   (ny+1) x (nx+2) (columns -1..nx) - the same face-row layout with rows and
 *   faces swapped, i.e. [side][var][face a][column b]. With characteristic
 *   variables var indexes the characteristic fields of each face (speeds
 *   u - c, u, u + c in 1-D; un - c, un, un (shear), un + c in 2-D).
 * ws: workspace of gks_workspace_bytes(g) bytes. */
int geno_reconstruct(const geno_grid* g, void* W, void* dW, int dir, void* face_state,
                     void* chi, void* ws, void* stream);

/* Gas-kinetic interface flux (BGK solution of the standard high-order GKS;
 * the paper defers its details to the literature, Sec. 2) at every point of
 * face_state (layout of geno_reconstruct), with time step dt and the
 * collision time of geno_params. Outputs per face, averaged over the Gauss
 * points with weights 1/2 (Sec. 2 face quadrature), [var][nfy][nfx]:
 *   F    = flux at the start of the step, from fitting F + t dF/dt to the
 *          time integrals of the flux over dt/2 and dt;
 *   Ft   = dF/dt of that fit;
 *   Wint = three blocks [3][var][nfy][nfx]: the conserved state of the
 *          interface solution at t = dt/2 and at t = dt, and the second time
 *          derivative W_tt of the interface equilibrium (the Euler equations'
 *          -d_x(A W_t) - d_y(B W_t) from the points' first and second
 *          derivatives).
 * Any of F, Ft, Wint may be NULL. dir as in geno_reconstruct. */
int gks_flux(const geno_grid* g, const void* face_state, double dt, int dir, void* F,
             void* Ft, void* Wint, void* stream);

/* nsteps steps of the two-stage fourth-order GKS update of W and dW in place
 * (Eq. (1): face fluxes; Eq. (2): cell-averaged gradients from the interface
 * values by the Gauss theorem). Each step: dt from the CFL condition on the
 * current state; stage 1 W* = W + dt/2 L + dt^2/8 dL/dt, with gradients from
 * the interface values W(dt/2) + dt^2/8 W_tt at the stage time; stage 2
 * W = W + dt L + dt^2/6 dL/dt + dt^2/3 dL/dt(W*), with gradients from the
 * interface values at the end of the step, W(dt) + dt^2/6 (W_tt + 2 W_tt*)
 * (the same two-stage structure applied to the interface values: W(t) of
 * the interface solution and W_tt of its equilibrium, W_tt* from stage 2).
 * ws: workspace of gks_workspace_bytes(g) bytes.
 * dt_out (device, may be NULL): nsteps doubles, the step sizes.
 * stats (host, may be NULL): if given, the call waits for the stream and
 *   fills the counters; returns GENO_ENONPHYS if a non-physical cell
 *   (non-finite, rho <= 0 or p <= 0) was found after any step. */
int gks_step(const geno_grid* g, void* W, void* dW, void* ws, int nsteps, double* dt_out,
             geno_stats* stats, void* stream);

/* Size of the device memory gks_step_noalloc works in: 64 MiB on every
 * device the library runs on (enough for the workspace of a 2-D float64 grid
 * of up to about 300 x 300 cells, mixed precision about 410 x 410; see
 * gks_workspace_bytes). */
#define GENO_NOALLOC_SCRATCH_BYTES (64u << 20)

/* gks_step without a workspace argument and without allocating: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). The same steps, kernels
 * and results as gks_step (bitwise), with the workspace taken from a
 * file-scope device array of GENO_NOALLOC_SCRATCH_BYTES that each device
 * holds from the library's load until the process ends. The caller passes
 * the state and the outputs as for gks_step.
 * Calls on one device share that device's array and keep the last call's
 * contents in it (every entry a step reads is written by that step first):
 * calls that overlap on one device (other streams, other host threads)
 * race; serialise them. No work counting (geno_count_enable) is done.
 * Errors: GENO_EINVAL if the grid's workspace (gks_workspace_bytes) exceeds
 * GENO_NOALLOC_SCRATCH_BYTES, for a bad grid, null W or dW, or nsteps < 0;
 * otherwise as gks_step. Never calls hipMalloc, hipFree or an allocating
 * library routine. */
int gks_step_noalloc(const geno_grid* g, void* W, void* dW, int nsteps, double* dt_out,
                     geno_stats* stats, void* stream);

/* The paper's comparison of nonlinear reconstructions (Sec. 5), on every
 * face-side of direction dir, from the stencils of the normal step: the
 * share of the high-order linear reconstruction each method keeps.
 *   method 0: GENO, its path function chi (Eq. (4));
 *   method 1: WENO-Z weights w~_k = d_k (1 + tau_Z / (IS_k + eps)) on the
 *             three sub-stencils, tau_Z = |IS_1 - IS_3| (the outer two);
 *   method 2: TENO weights: scale separation (1/(IS_k + eps))^7 normalised,
 *             sub-stencils with a share <= teno_ct cut (the paper uses 1e-6,
 *             1e-3 for its Titarev-Toro run);
 * with chi = min_k w_k / d_k for WENO-Z and TENO (d_k the linear weights of
 * geno_params normalised to sum 1; TENO's chi is 1 or 0).
 * chi3 (device): [3][2][nvar][n0][n1] doubles, [method][side][var] planes in
 * the face-row layout of geno_reconstruct's chi. Fills the ghost layers of
 * W, dW like geno_reconstruct; ws: workspace of gks_workspace_bytes(g).
 * The comparison works on the conservative variables whatever
 * geno_params.variables says. */
int geno_linearity(const geno_grid* g, void* W, void* dW, int dir, double* chi3, double teno_ct,
                   void* ws, void* stream);

/* Conserved totals (diagnostic): totals[f] = |cell| * sum over the interior
 * cells of W[f] for every field f (3 in 1-D, 4 in 2-D), |cell| = dx (1-D) or
 * dx dy (2-D). The update is in conservation form (Eq. (1)): on periodic
 * grids these totals stay constant up to rounding. Compensated summation
 * (Neumaier) in a fixed order, so the result is deterministic and within a
 * few units in the last place of the exactly rounded sum.
 * W: device, the state layout of gks_step; totals: device, nfields doubles.
 * Asynchronous on stream; no workspace. */
int geno_conserved_totals(const geno_grid* g, const void* W, double* totals, void* stream);

/* ---- batched form --------------------------------------------------------
 * Many independent 2-D grids advanced together. Grids may differ in size and
 * boundary conditions; every other field of geno_params (method constants,
 * precision, cfl, dt_fixed, eps_ulps) must be equal across the batch. Each
 * grid keeps its own time step (its own CFL condition). Results are
 * identical to gks_step on each grid alone, in every mode:
 *   GENO_BATCH_EAGER: each kernel kind runs as one launch over the work of
 *     every grid (work-group ranges concatenated; each work-group looks up
 *     its grid): per stage a prep launch (each grid's dt and queues), the
 *     fused x- and y-face launches (params.fuse; the normal step inside the
 *     face kernels), the tau > 0 queue and the update, ten launches per
 *     step (twelve with fuse = 0 or characteristic variables: separate
 *     normal-step launches per direction);
 *   GENO_BATCH_GRAPH: the same launches captured once as a HIP graph and
 *     replayed;
 *   GENO_BATCH_PERSISTENT: reserved for one persistent launch per step (a
 *     device work queue over the blocks of all phases of all grids, each
 *     block started once its grid's previous phase is complete). Not
 *     available in this build: the call returns GENO_EINVAL.
 * A step's graph is kept across calls (up to 8 graphs, the least recently
 * used replaced) and reused while the device, workspace, batch plan and
 * method constants are the same. */
#define GENO_BATCH_EAGER 0
#define GENO_BATCH_GRAPH 1
#define GENO_BATCH_PERSISTENT 2

/* Work-group shapes of the batched launches (chosen by geno_autotune_batched
 * or given by the caller). block_*: threads per work-group of the normal GENO,
 * face, tau > 0 and update launches: 128, 256 or 512 (0 = 256); the fused
 * face launches have fixed tiles (block_normal and block_faces serve the
 * two-launch path). The update's
 * size also serves the start-of-call launch. slow_faces_per_block: the tau > 0
 * launch gives each grid ceil(faces / slow_faces_per_block) work-groups
 * (between 1 and 1024; 0 = 2048). */
typedef struct geno_tuning {
  int version;
  int block_normal;
  int block_faces;
  int block_slow;
  int block_update;
  int slow_faces_per_block;
} geno_tuning;

/* Defaults: 256-thread work-groups, 2048 faces per tau > 0 work-group. */
int geno_tuning_default(geno_tuning* t);

/* Largest batch accepted by the batched calls. */
#define GENO_BATCH_MAX 4096

/* Bytes of the device workspace of a batch of ngrids grids (grids: host
 * array); 0 if the batch is invalid. */
size_t gks_batched_workspace_bytes(int ngrids, const geno_grid* grids);

/* nsteps steps of every grid of the batch in place (the two-stage update of
 * gks_step on each grid).
 * grids: host array of ngrids grid descriptions (2-D only).
 * W, dW: host arrays of ngrids device pointers, each laid out as for
 *   gks_step on its grid (element types of the batch's precision).
 * ws: workspace of gks_batched_workspace_bytes bytes.
 * tune: work-group shapes (NULL = defaults).
 * use_graph: the mode, GENO_BATCH_EAGER, GENO_BATCH_GRAPH or
 *   GENO_BATCH_PERSISTENT (GENO_EINVAL otherwise); in the graph modes the
 *   stream must not be the NULL stream (GENO_EINVAL otherwise).
 * step_ms (host, may be NULL): nsteps floats, the duration of each step from
 *   events recorded between the steps on the stream.
 * stats (host, may be NULL): counters summed over the grids.
 * The call waits for the stream (it copies the batch table to ws first and
 * reads the timings or counters back when asked). */
int gks_step_batched(int ngrids, const geno_grid* grids, void* const* W, void* const* dW, void* ws,
                     int nsteps, const geno_tuning* tune, int use_graph, float* step_ms,
                     geno_stats* stats, void* stream);

/* Number of batched-step graphs instantiated by this process so far (a call
 * that reuses a kept graph does not add one). Measurement support. */
long long geno_batched_graphs_built(void);

/* Autotuner of the batched work-group shapes: for each launch kind in turn
 * (normal GENO, faces, tau > 0 faces, update) it runs trial_steps steps of
 * the batch with every candidate shape (block sizes 128, 256, 512; for the
 * tau > 0 launch also 512, 2048 and 8192 faces per work-group) and keeps the
 * one with the least summed kernel time (events bound to the dispatches).
 * The trials advance the given state: pass a copy. Writes the choice to
 * *out. */
int geno_autotune_batched(int ngrids, const geno_grid* grids, void* const* W, void* const* dW,
                          void* ws, int trial_steps, geno_tuning* out, void* stream);

/* ---- learned gate ---------------------------------------------------------
 * A small network predicts the path function chi (Eq. (4)) of a cell and
 * direction from its normalised 5-cell stencil; it is trained on stencils the
 * solver harvests, and plain GENO is the fallback wherever the prediction is
 * below 1 - gate_delta.
 * Network: 40 inputs -> 64 -> 64 (GELU, tanh form) -> 1 (sigmoid);
 * parameters are 6849 floats in the order W1[64][40], b1[64], W2[64][64],
 * b2[64], w3[64], b3.
 * Input of cell j along a direction (face frame: normal momentum second): per
 * conserved variable q, den = max - min of q over cells j-2..j+2 +
 * 1e-12 |q_j| + 1e-300; features (q_m - q_j)/den, m = -2..2, then
 * h (dq/dn)_m / den, m = -2..2, each clipped to [-64, 64]; variable-major.
 * Target: the smallest plain-GENO chi over the cell's two face-sides of the
 * direction (left state of its face j+1/2, right state of its face j-1/2) and
 * the four variables. */
#define GENO_MLP_NIN 40
#define GENO_MLP_NPARAM 6849

/* Network input X[ncell][40] (float) and target y[ncell] (float, may be NULL)
 * of every interior cell (row-major, x fastest) for direction dir of a 2-D
 * grid, after filling the ghost cells of W and dW in place; targets from
 * float64 plain GENO. ws: workspace of gks_workspace_bytes(g). */
int geno_harvest(const geno_grid* g, void* W, void* dW, int dir, float* X, float* y, void* ws,
                 void* stream);

/* Device scratch of geno_mlp_grad for a minibatch of n samples. */
size_t geno_mlp_train_workspace_bytes(int n);

/* Training in float32 (device pointers): gradient of the mean binary
 * cross-entropy of the network (params) on X[n][40], y[n] into grad[6849],
 * and the loss itself into loss[0] (may be NULL). Deterministic. */
int geno_mlp_grad(const float* params, const float* X, const float* y, int n, float* grad,
                  float* loss, void* ws, void* stream);

/* One Adam step on params with moments m, v (t counts from 1). */
int geno_mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr,
                  float beta1, float beta2, float eps, void* stream);

/* Float32 forward pass (reference of the training kernels): prob[n]. */
int geno_mlp_forward(const float* params, const float* X, int n, float* prob, void* stream);

/* Loads a trained network (device float params[6849]) as the library's
 * bfloat16 copy used by the gate and geno_mlp_infer, on the current device.
 * Waits for the stream. */
int geno_mlp_load(const float* params, void* stream);

/* Inference with the loaded network on bfloat16 matrix cores (float32
 * accumulation): prob[n] for X[n][40] (device). */
int geno_mlp_infer(const float* X, int n, float* prob, void* stream);

/* The gate's prediction for every interior cell of a 2-D grid and direction
 * (inputs built on the device from W, dW as geno_harvest does; ghost cells
 * filled in place): prob[ncell]. */
int geno_gate_prob(const geno_grid* g, void* W, void* dW, int dir, float* prob, void* ws,
                   void* stream);

/* ---- measurement support ------------------------------------------------
 * Kernel kinds of gks_step reported by geno_timing_read / geno_work_read. */
enum {
  GENO_K_INIT = 0,     /* ghost cells of the initial state + its CFL partial minima */
  GENO_K_NORMAL_X,     /* normal GENO on x-face rows */
  GENO_K_NORMAL_Y,     /* normal GENO on y-face columns */
  GENO_K_FACES_X,      /* tangential step + gas-kinetic flux, x-faces with tau = 0 */
  GENO_K_FACES_Y,
  GENO_K_SLOW,         /* the same for the faces of both directions queued with
                          tau > 0 at a Gauss point (full BGK solution) */
  GENO_K_UPDATE_1,     /* stage-1 update, gradients, ghost cells of the stage state */
  GENO_K_UPDATE_2,     /* stage-2 update, gradients, ghost cells, CFL partial minima */
  GENO_K_FACES_1D,     /* 1-D: GENO + flux per face */
  GENO_K_GATE,         /* learned gate of both directions (network inference) */
  GENO_K_NORMAL_XY,    /* 2-D gks_step: normal GENO of both directions in one
                          launch (its work is counted under NORMAL_X and
                          NORMAL_Y) */
  GENO_K_FUSED_X,      /* 2-D gks_step with params.fuse: normal GENO, tangential
                          step and flux of the x-faces in one launch */
  GENO_K_FUSED_Y,      /* the same for the y-faces */
  GENO_NKERNELS
};

/* Work classes counted per kernel kind while counting is enabled. */
enum {
  GENO_W_UNITS = 0,    /* threads' work units: face-row variables, faces, cells */
  GENO_W_EQUAL,        /* gas-kinetic points with tau = 0 and equal states (no
                          half-space moments) */
  GENO_W_LOW,          /* reconstructions that form the low-order part (chi < 1) */
  GENO_W_FAST,         /* gas-kinetic points with tau = 0 and different states */
  GENO_W_SLOW,         /* gas-kinetic points evaluated with tau > 0 */
  GENO_W_GUARD,        /* point states replaced by the cell average */
  GENO_W_GATED,        /* face-sides whose indicators the gate skipped */
  GENO_NCLASS
};

/* Enables per-kernel timing in gks_step: each of the next max_launches
 * launches is made with a start and a stop event bound to the kernel's own
 * dispatch (hipExtLaunchKernel), so the recorded interval is the kernel's
 * execution, not the queue around it. Events are created here, once; 0
 * disables and releases them. Not thread-safe: intended for benchmarks. */
int geno_timing_enable(int max_launches);

/* Enables (on != 0) or disables counting of the work classes in gks_step.
 * Each work-group adds its sums to its own slot of a device buffer (no
 * atomics), so counting hardly changes kernel durations; the buffer is
 * allocated on the current device by the first counted gks_step call and
 * cleared at the start of every counted call. Not thread-safe. */
int geno_count_enable(int on);

/* Waits for the recorded events, writes per kernel kind the summed duration
 * in milliseconds and the launch count (arrays of nkinds entries, host), and
 * starts a new recording. */
int geno_timing_read(int nkinds, double* ms_total, long long* launches);

/* Work counts of the last counted gks_step call: counts[kind * nclass +
 * class], host array (zeros if none). Waits for the stream. */
int geno_work_read(int nkinds, int nclass, long long* counts, void* stream);

/* Floating-point operations per work item of each class and kernel kind, as
 * executed by the device functions (add, sub, mul, div, sqrt, compare-free;
 * each elementary function call counts 1): costs[kind * nclass + class] for
 * the grid's dimension. Units: the per-unit cost excludes the optional
 * branches, which the other classes add. */
int geno_op_costs(const geno_grid* g, int nkinds, int nclass, double* costs);

/* Name of a kernel kind ("" if out of range). */
const char* geno_kernel_name(int kind);

#ifdef __cplusplus
}
#endif

#endif /* GENO_GKS_H */
