/*
 * geno_tri.h - C ABI of the fourth-order compact GENO reconstruction on 2-D
 * triangular meshes (Zhao & Xu, "A generalized ENO reconstruction in compact
 * GKS for compressible flow simulations", Sec. 4.3, with the GENO blend,
 * Eq. (3)-(4), the ultimate smoothness indicator, Eq. (5), the indicators of
 * Eq. IS-highorder-1 and IS-tau, and the ENO weights of Eq. (8) from Sec. 3),
 * for gfx950.
 *
 * Method, per cell Omega_j (target) and per variable, data being the cell
 * averages and averaged gradients of the compact scheme:
 *   q^H = p^3: the cubic whose average on Omega_j is exact and which fits in
 *     least squares the averages of the nine other cells of S_0 (the three
 *     edge neighbours Omega_{j_k} and their six other neighbours) and the
 *     h-scaled averaged gradients of Omega_j and of the three edge
 *     neighbours (the compact stencil of Sec. 4.3; the paper defers the
 *     least-squares details to its references);
 *   p_k, k = 1..3: the linear polynomial on S_k = {Omega_j, Omega_{j_k}}
 *     whose average on Omega_j is exact and which fits in least squares the
 *     average and h-scaled gradient of Omega_{j_k};
 *   IS^H = sum over multi-indices 1 <= |l| <= 3 of h^{2|l|-2} int (D^l q^H)^2,
 *   IS~^H the same over |l| <= 2, IS^tau = |IS^H - IS~^H| (Eq. IS-tau);
 *   IS_k = int |grad p_k|^2; IS^L = (sum IS_k - min - max)/(k_0 - 2), k_0 = 3;
 *   alpha^{H,L} = 1 + (IS^tau/(IS^{H,L} + eps))^r with r = 3,
 *   alpha = 2 alpha^H/(alpha^H + alpha^L), chi = tanh(C alpha)/tanh(C);
 *   w_k ~ d_k/(IS_k + eps)^2 with d_k = 1;
 *   R = chi p^3 + (1 - chi) sum_k w_k p_k.
 * h = sqrt(|Omega_j|). Component-wise on the given variables.
 *
 * Mesh (host arrays, periodic or not - translations carry the periods):
 *   xv    [ncell][3][2] vertex coordinates of each triangle, counter-clockwise;
 *   nbr   [ncell][3]    the cell across edge e (vertex e to vertex e+1);
 *   shift [ncell][3][2] translation that places nbr[c][e], as given by its
 *                       own xv, next to cell c (zero inside the domain).
 * Every cell must have three neighbours (closed or periodic mesh).
 *
 * Conventions as geno_gks.h (error codes GENO_*, geno_last_error).
 */
#ifndef GENO_TRI_H
#define GENO_TRI_H

#include <stddef.h>

#include "geno_gks.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Doubles per cell of the operator table (stencil indices, h, least-squares
 * operators of the candidates, scaled vertices, and the geometry of the step:
 * area, 4 area / perimeter, per edge the outward unit normal, length,
 * neighbour, the neighbour's index of the same edge and ownership; then two
 * slots of a mesh-wide list of the owned (cell, edge) pairs, which the step
 * walks one edge per thread). */
size_t geno_tri_table_doubles(void);

/* Mesh layer, host only (no device access; call once per mesh): fills the
 * operator table ops (HOST array of ncell * geno_tri_table_doubles()
 * doubles, owned by the caller; entries stored in pairs, entry e of cell c
 * at index ((e / 2) * ncell + c) * 2 + e % 2) from the mesh arrays
 * above. The caller copies it to device memory for geno_tri_reconstruct.
 * GENO_EINVAL for ncell < 1, null pointers, a neighbour index out of range,
 * a neighbour that does not point back across the same edge (with the
 * opposite translation), a degenerate (non counter-clockwise) triangle or a
 * rank-deficient least-squares system. */
int geno_tri_build(int ncell, const double* xv, const int* nbr, const double* shift, double* ops);

/* GENO reconstruction of every cell at the two Gauss points of each of its
 * edges (points t = 1/2 -+ 1/(2 sqrt 3) along edge e from vertex e to e+1).
 * ops: DEVICE copy of the table from geno_tri_build (16-byte aligned).
 * W (device): cell averages [nv][ncell]; dW (device): averaged gradients
 *   [2][nv][ncell] (d/dx rows, then d/dy rows). nv in 1..GENO_TRI_MAXV.
 * out (device): [point(6) = 2 e + g][quant(3)][nv][ncell], quant 0 the value,
 *   1 and 2 h d/dx and h d/dy of R (h of the cell).
 * chi (device, may be NULL): [nv][ncell] path function of each cell.
 * sec (device, may be NULL): [point(6)][3][nv][ncell], h^2 times the second
 *   derivatives d_xx, d_xy, d_yy of R: chi times those of p^3 (the linear
 *   candidates have none).
 * Asynchronous on stream; allocates nothing. */
#define GENO_TRI_MAXV 4
int geno_tri_reconstruct(int ncell, int nv, const void* ops, const double* W, const double* dW,
                         double* out, double* chi, double* sec, void* stream);

/* Bytes of the device workspace of geno_tri_step on a mesh of ncell cells
 * (0 for ncell < 1). */
size_t geno_tri_workspace_bytes(int ncell);

/* nsteps steps of the compact GKS on the mesh (Sec. 4.3 with Sec. 2,
 * Eq. (1)-(2)), in place, float64, conserved variables (rho, rho u, rho v,
 * rho E) of the 2-D Euler equations:
 *   per stage: the reconstruction above at the edge Gauss points (values,
 *   gradients, second derivatives); per edge, once, from its owner cell
 *   (the smaller (cell, edge) pair of its two sides): at both Gauss points
 *   the owner's state on the left and the neighbour's on the right, a side
 *   with rho <= 0, p <= 0 or a non-finite value replaced by its cell average
 *   with zero derivatives, the gas-kinetic solution of gks_flux in the frame
 *   of the owner's outward unit normal (F, dF/dt, W(dt/2), W(dt), phi W_tt),
 *   rotated back and averaged over the two points; per cell, Eq. (1) and the
 *   Gauss-theorem gradients of Eq. (2) over its three edges;
 *   the two-stage fourth-order combination of gks_step (cell averages and
 *   the interface values of the gradient update alike);
 *   dt = cfl min over cells of d / (|u| + c), d = 4 |Omega| / perimeter (the
 *   inscribed circle's diameter), or p->dt_fixed if positive.
 * ops: DEVICE copy of the table of geno_tri_build.
 * W (device): [4][ncell]; dW (device): [2][4][ncell] (d/dx rows, then d/dy).
 * ws (device): geno_tri_workspace_bytes(ncell) bytes.
 * p (host): the method constants gamma, tau_c1, tau_c2, cfl, dt_fixed of a
 *   geno_params (version GENO_ABI_VERSION, precision GENO_F64); the
 *   reconstruction's constants are those of geno_tri_reconstruct.
 * dt_out (device, may be NULL): nsteps doubles.
 * stats (host, may be NULL): waits for the stream, fills the counters and
 *   returns GENO_ENONPHYS if a non-physical cell was found after any step.
 * GENO_EINVAL for ncell < 1, null pointers, nsteps < 0 or bad constants. */
int geno_tri_step(int ncell, const void* ops, double* W, double* dW, void* ws, int nsteps,
                  const geno_params* p, double* dt_out, geno_stats* stats, void* stream);

/* Floating-point operations per cell and variable of geno_tri_reconstruct
 * (as the kernel executes them; add, sub, mul, div, sqrt, tanh count 1). */
double geno_tri_op_cost(void);

#ifdef __cplusplus
}
#endif

#endif /* GENO_TRI_H */
