/*
 * CPU FP64 oracle of the compact gas-kinetic scheme with GENO reconstruction
 * (Zhao & Xu, "A generalized ENO reconstruction in compact GKS for
 * compressible flow simulations").
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library. It shares
 * no code, header, table or constant with the HIP library: every weight it
 * uses is obtained here by solving the defining moment systems, the GKS
 * moments come from a generic polynomial-times-Maxwellian integrator, and the
 * micro-slopes are solved by Gaussian elimination rather than closed forms.
 *
 * Paper passages followed (equation numbers of the paper):
 *   Sec. 2   Eq. (1)  finite-volume update; face integrals by Gauss quadrature
 *   Sec. 2   Eq. (2)  cell-averaged gradients from the Gauss theorem
 *   Sec. 3   Eq. (3)  GENO blend R = chi q^H + (1-chi) q^L
 *   Sec. 3.1 Eq. (4)  path function chi = tanh(C alpha)/tanh(C)
 *   Sec. 3.2 Eq. (5)  ultimate smoothness indicator alpha
 *   Sec. 3.2 Eq. (6)-(7) IS of Jiang-Shu type; IS^H = Max{IS_k}
 *   Sec. 3.3 Eq. (8)  ENO low-order combination q^L; Eq. (9) IS^L = Min{IS_k}
 *   Sec. 4.2 Eq. (13)-(14) 8th-order compact stencils S_0..S_3 and IS^tau
 * The paper defers the GKS flux, the two-stage fourth-order (S2O4) time
 * stepping, ghost cells, the collision time and the 2-D structured scheme to
 * the literature. Those parts follow the standard BGK interface solution of
 * high-order GKS and are marked "reading" where they are defined below.
 *
 * Layout of every state array handed in: SoA, interior cells only,
 * [field][ny][nx] (1-D: ny = 1). Gradients are physical (not h-scaled).
 * Fields 1-D: W = (rho, rhoU, rhoE), dW = (d_x W).
 * Fields 2-D: W = (rho, rhoU, rhoV, rhoE), dW = (d_x W[4], d_y W[4]).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

/* ---------------------------------------------------------------------- */
/* Parameters (plain double array from the caller)                         */
/* ---------------------------------------------------------------------- */
enum {
  PI_GAMMA = 0, PI_CPATH, PI_EPS, PI_R, PI_RL, PI_D1, PI_D2, PI_D3,
  PI_TAUC1, PI_TAUC2, PI_CFL, PI_BCXL, PI_BCXH, PI_BCYL, PI_BCYH,
  PI_GHOST,     /* 24 values, 1-D fixed ends: [end][layer][W (3), dW (3)] */
  PI_CHAR = PI_GHOST + 24,   /* 1 = characteristic-variable reconstruction (normal step) */
  PI_GUPD,   /* time stepping of the gradients: 0 the two-stage fourth-order
                structure on the interface values (default), 1 the BGK
                interface state at dt/2 of each stage (earlier reading) */
  PI_COUNT
};

typedef struct {
  double gamma, Cpath, eps, r, rL, d[3], tc1, tc2, cfl;
  int bc[4];           /* 0 periodic, 1 transmissive, 2 reflecting, 3 fixed (1-D only):
                          x-lo, x-hi, y-lo, y-hi */
  double ghost[2][2][6];  /* fixed ends: [end][layer 0 = next to the grid][W, dW] */
  int characteristic;     /* reconstruct characteristic variables in the normal step */
  int gupd;               /* gradient update reading (PI_GUPD) */
  int ndim, nx, ny;
  double dx, dy;
  double K;            /* internal degrees of freedom of the BGK model */
  int nv;              /* conserved variables: 3 in 1-D, 4 in 2-D */
} ocfg;

static void cfg_from(ocfg *c, int ndim, int nx, int ny, double dx, double dy,
                     const double *p) {
  c->gamma = p[PI_GAMMA]; c->Cpath = p[PI_CPATH]; c->eps = p[PI_EPS];
  c->r = p[PI_R]; c->rL = p[PI_RL];
  c->d[0] = p[PI_D1]; c->d[1] = p[PI_D2]; c->d[2] = p[PI_D3];
  c->tc1 = p[PI_TAUC1]; c->tc2 = p[PI_TAUC2]; c->cfl = p[PI_CFL];
  for (int i = 0; i < 4; ++i) c->bc[i] = (int)p[PI_BCXL + i];
  for (int e = 0; e < 2; ++e)
    for (int l = 0; l < 2; ++l)
      for (int q = 0; q < 6; ++q) c->ghost[e][l][q] = p[PI_GHOST + (e * 2 + l) * 6 + q];
  c->characteristic = (int)p[PI_CHAR];
  c->gupd = (int)p[PI_GUPD];
  c->ndim = ndim; c->nx = nx; c->ny = (ndim == 1) ? 1 : ny;
  c->dx = dx; c->dy = dy;
  /* Internal degrees of freedom so that gamma = (K + D + 2)/(K + D) with
   * D translational dimensions carried explicitly (reading: standard GKS). */
  c->K = (ndim == 1) ? (3.0 - c->gamma) / (c->gamma - 1.0)
                     : (4.0 - 2.0 * c->gamma) / (c->gamma - 1.0);
  c->nv = (ndim == 1) ? 3 : 4;
}

/* ---------------------------------------------------------------------- */
/* Small dense solver (Gaussian elimination with partial pivoting)         */
/* ---------------------------------------------------------------------- */
/* Solves A x = b in place (A is n x n row-major, destroyed). long double
 * variant used once at start-up for the reconstruction operators. */
static int solve_ld(int n, long double *A, long double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabsl(A[i * n + k]) > fabsl(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0L) return -1;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        long double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t;
      }
      long double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      long double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    long double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
    b[k] = s / A[k * n + k];
  }
  return 0;
}

/* Same in double, for the per-point 3x3 / 4x4 micro-slope systems. */
static int solve_d(int n, double *A, double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return -1;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t;
      }
      double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
    b[k] = s / A[k * n + k];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Reconstruction operators, obtained by solving the defining systems       */
/* ---------------------------------------------------------------------- */
/* Average over [a, b] of y^k, and of d/dy (y^k). */
static long double avg_mono(int k, long double a, long double b) {
  return (powl(b, k + 1) - powl(a, k + 1)) / ((long double)(k + 1) * (b - a));
}
static long double avg_dmono(int k, long double a, long double b) {
  if (k == 0) return 0.0L;
  return (powl(b, k) - powl(a, k)) / (b - a);
}

/* Linear high-order reconstruction p^7 (Sec. 4.2, stencil S_0 = {j-1..j+2}):
 * the degree-7 polynomial whose averages and averaged h-scaled derivatives
 * match those of the four cells. Coordinate y = (x - x_{j+1/2})/h, cell j-1+m
 * occupies [m-2, m-1]. Data order: (Q_{-1}, G_{-1}, Q_0, G_0, Q_1, G_1, Q_2, G_2),
 * G = h * (cell-averaged derivative). H_val / H_der / H_d2: weights of the
 * face value, of h times the face derivative and of h^2 times the second
 * derivative. */
static double H_val[8], H_der[8], H_d2[8];

/* Low-order sub-stencil quadratics p_k (Sec. 4.2, S_1 = {j-1, j} with the
 * gradient of cell j-1, S_2 = {j-1, j, j+1}, S_3 = {j, j+1, j+2}) for the
 * cell c on side s of the face (s = +1: face on the right of c, left state;
 * s = -1: face on the left of c, right state; the stencils are mirrored).
 * Coordinate xi = (x - x_c)/h. SUB[s][k][coef][datum] maps the data of cells
 * c-2..c+2 (order Q_{c-2}, G_{c-2}, ..., Q_{c+2}, G_{c+2}) to the monomial
 * coefficients of p_k. */
static double SUB[2][3][3][10];

/* Quadratic through three averages over [-3/2,-1/2], [-1/2,1/2], [1/2,3/2]
 * (tangential high-order candidate): TQ[coef][datum]. */
static double TQ[3][3];

static int ops_ready = 0;
static void build_psi(void);

static int build_ops(void) {
  /* p^7 */
  {
    long double A[64], rhs[8];
    double Hv[8], Hd[8], H2[8];
    for (int col = 0; col < 8; ++col) {
      /* column col of the inverse: solve with unit right-hand side */
      for (int m = 0; m < 4; ++m) {
        long double a = (long double)(m - 2), b = (long double)(m - 1);
        for (int k = 0; k < 8; ++k) {
          A[(2 * m) * 8 + k] = avg_mono(k, a, b);
          A[(2 * m + 1) * 8 + k] = avg_dmono(k, a, b);
        }
      }
      for (int i = 0; i < 8; ++i) rhs[i] = (i == col) ? 1.0L : 0.0L;
      if (solve_ld(8, A, rhs)) return -1;
      Hv[col] = (double)rhs[0];           /* p(0) */
      Hd[col] = (double)rhs[1];           /* h p'(0) */
      H2[col] = (double)(2.0L * rhs[2]);  /* h^2 p''(0) */
    }
    memcpy(H_val, Hv, sizeof Hv);
    memcpy(H_der, Hd, sizeof Hd);
    memcpy(H_d2, H2, sizeof H2);
  }
  /* quadratics */
  for (int si = 0; si < 2; ++si) {
    int s = (si == 0) ? +1 : -1;
    for (int k = 0; k < 3; ++k) {
      /* constraints: list of (cell offset, kind) kind 0 = average, 1 = derivative average */
      int off[3], kind[3];
      if (k == 0) { off[0] = -s; kind[0] = 0; off[1] = -s; kind[1] = 1; off[2] = 0; kind[2] = 0; }
      else if (k == 1) { off[0] = -1; kind[0] = 0; off[1] = 0; kind[1] = 0; off[2] = 1; kind[2] = 0; }
      else { off[0] = 0; kind[0] = 0; off[1] = s; kind[1] = 0; off[2] = 2 * s; kind[2] = 0; }
      for (int col = 0; col < 3; ++col) {
        long double A[9], rhs[3];
        for (int row = 0; row < 3; ++row) {
          long double a = off[row] - 0.5L, b = off[row] + 0.5L;
          for (int q = 0; q < 3; ++q)
            A[row * 3 + q] = kind[row] ? avg_dmono(q, a, b) : avg_mono(q, a, b);
        }
        for (int i = 0; i < 3; ++i) rhs[i] = (i == col) ? 1.0L : 0.0L;
        if (solve_ld(3, A, rhs)) return -1;
        /* constraint col refers to datum index 2*(off+2) + kind */
        int datum = 2 * (off[col] + 2) + kind[col];
        for (int q = 0; q < 3; ++q) {
          /* accumulate (each datum appears in at most one constraint) */
          SUB[si][k][q][datum] = (double)rhs[q];
        }
      }
    }
  }
  /* tangential quadratic */
  for (int col = 0; col < 3; ++col) {
    long double A[9], rhs[3];
    for (int row = 0; row < 3; ++row)
      for (int q = 0; q < 3; ++q) A[row * 3 + q] = avg_mono(q, row - 1.5L, row - 0.5L);
    for (int i = 0; i < 3; ++i) rhs[i] = (i == col) ? 1.0L : 0.0L;
    if (solve_ld(3, A, rhs)) return -1;
    for (int q = 0; q < 3; ++q) TQ[q][col] = (double)rhs[q];
  }
  build_psi();
  ops_ready = 1;
  return 0;
}

/* 3-point Gauss-Legendre on [-1/2, 1/2]: exact for degree <= 5. */
static const double GL3_X[3] = {-0.38729833462074168852, 0.0, 0.38729833462074168852};
static const double GL3_W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

/* Smoothness indicator of a quadratic c0 + c1 xi + c2 xi^2 on its own cell,
 * Eq. (6) with m = 1 and derivatives up to order 2 (a quadratic has no
 * third derivative): sum_l h^(2l-1) int (d^l p/dx^l)^2 dx, in xi units. */
static double is_quadratic(const double c[3]) {
  double s = 0.0;
  for (int q = 0; q < 3; ++q) {
    double x = GL3_X[q];
    double d1 = c[1] + 2.0 * c[2] * x;
    double d2 = 2.0 * c[2];
    s += GL3_W[q] * (d1 * d1 + d2 * d2);
  }
  return s;
}

/* ---------------------------------------------------------------------- */
/* GENO at one face for one side and one conserved component               */
/* ---------------------------------------------------------------------- */
/* Ultimate smoothness indicator and path function, Eq. (4)-(5). */
static double path_function(const ocfg *P, double IStau, double ISH, double ISL) {
  double aH = 1.0 + pow(IStau / (ISH + P->eps), P->r);
  double aL = 1.0 + pow(IStau / (ISL + P->eps), P->r);
  double alpha = 2.0 * aH / (aH + aL);
  return tanh(P->Cpath * alpha) / tanh(P->Cpath);
}

/* dat: Q_{c-2}, G_{c-2}, ..., Q_{c+2}, G_{c+2} about the reconstructing cell
 * c; si = 0 for the left state (face at xi = +1/2), 1 for the right state
 * (face at xi = -1/2). qH, hqH, h2qH: shared linear value, h * derivative and
 * h^2 * second derivative. Output: value, h * derivative, h^2 * second
 * derivative and chi at the face. The second derivative follows the blend of
 * Eq. (3) with the same weights (the quadratics' second derivatives 2 c_2 in
 * the low-order part); the time stepping of the gradients uses it. */
static void geno_side(const ocfg *P, const double dat[10], int si, double qH, double hqH,
                      double h2qH, double *val, double *hder, double *h2der, double *chi_out) {
  double xf = (si == 0) ? 0.5 : -0.5;
  double c[3][3], IS[3], pv[3], pd[3], p2[3];
  for (int k = 0; k < 3; ++k) {
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int m = 0; m < 10; ++m) s += SUB[si][k][q][m] * dat[m];
      c[k][q] = s;
    }
    IS[k] = is_quadratic(c[k]);
    pv[k] = c[k][0] + c[k][1] * xf + c[k][2] * xf * xf;
    pd[k] = c[k][1] + 2.0 * c[k][2] * xf;
    p2[k] = 2.0 * c[k][2];
  }
  /* Eq. (7) and Eq. (9): structured-mesh IS^H and IS^L */
  double ISH = IS[0], ISL = IS[0];
  for (int k = 1; k < 3; ++k) { if (IS[k] > ISH) ISH = IS[k]; if (IS[k] < ISL) ISL = IS[k]; }
  /* Eq. (14): IS^tau of the 8th-order compact scheme */
  double IStau = fabs((IS[1] + IS[2]) / 2.0 - IS[0]);
  double chi = path_function(P, IStau, ISH, ISL);
  /* Eq. (8): ENO combination of the sub-stencil polynomials */
  double wt[3], wsum = 0.0;
  for (int k = 0; k < 3; ++k) { wt[k] = P->d[k] / pow(IS[k] + P->eps, P->rL); wsum += wt[k]; }
  double qL = 0.0, hqL = 0.0, h2qL = 0.0;
  for (int k = 0; k < 3; ++k) {
    qL += (wt[k] / wsum) * pv[k]; hqL += (wt[k] / wsum) * pd[k]; h2qL += (wt[k] / wsum) * p2[k];
  }
  /* Eq. (3) and Eq. (13), same weights for the derivatives */
  *val = chi * qH + (1.0 - chi) * qL;
  *hder = chi * hqH + (1.0 - chi) * hqL;
  *h2der = chi * h2qH + (1.0 - chi) * h2qL;
  *chi_out = chi;
}

/* Full GENO at face j+1/2 for one component. q[0..3] = averages of cells
 * j-1..j+2 (stencil S_0), g[0..3] = their h-scaled averaged derivatives.
 * out_l / out_r: value, h * derivative, chi, h^2 * second derivative. */
static void geno_face(const ocfg *P, const double q[4], const double g[4],
                      double out_l[4], double out_r[4]) {
  /* linear part: one polynomial per face, shared by both sides (Sec. 4.2) */
  double qH = 0.0, hqH = 0.0, h2qH = 0.0;
  for (int m = 0; m < 4; ++m) {
    qH += H_val[2 * m] * q[m] + H_val[2 * m + 1] * g[m];
    hqH += H_der[2 * m] * q[m] + H_der[2 * m + 1] * g[m];
    h2qH += H_d2[2 * m] * q[m] + H_d2[2 * m + 1] * g[m];
  }
  /* data about the reconstructing cell: left state uses cells j-2..j+2
   * (j-2 carries zero weight), right state cells j-1..j+3 (j+3 zero weight) */
  double dl[10] = {0}, dr[10] = {0};
  for (int m = 0; m < 4; ++m) {
    dl[2 * (m + 1)] = q[m]; dl[2 * (m + 1) + 1] = g[m];
    dr[2 * m] = q[m]; dr[2 * m + 1] = g[m];
  }
  geno_side(P, dl, 0, qH, hqH, h2qH, &out_l[0], &out_l[1], &out_l[3], &out_l[2]);
  geno_side(P, dr, 1, qH, hqH, h2qH, &out_r[0], &out_r[1], &out_r[3], &out_r[2]);
}

/* ---------------------------------------------------------------------- */
/* Ghost cells (reading: the paper only names the boundary conditions)     */
/* ---------------------------------------------------------------------- */
#define NG 2

typedef struct {
  int nxt, nyt;        /* padded sizes */
  double *W, *dW;      /* [nv][nyt][nxt], [ndim*nv][nyt][nxt] */
} gstate;

static inline size_t gidx(const gstate *g, int f, int j, int i) {
  return ((size_t)f * g->nyt + j) * g->nxt + i;
}

static int gstate_alloc(const ocfg *P, gstate *g) {
  g->nxt = P->nx + 2 * NG;
  g->nyt = (P->ndim == 1) ? 1 : P->ny + 2 * NG;
  size_t n = (size_t)g->nxt * g->nyt;
  g->W = (double *)calloc(n * P->nv, sizeof(double));
  g->dW = (double *)calloc(n * P->nv * P->ndim, sizeof(double));
  return (g->W && g->dW) ? 0 : -1;
}
static void gstate_free(gstate *g) { free(g->W); free(g->dW); }

static void gstate_load(const ocfg *P, gstate *g, const double *W, const double *dW) {
  int oy = (P->ndim == 1) ? 0 : NG;
  for (int f = 0; f < P->nv; ++f)
    for (int j = 0; j < P->ny; ++j)
      for (int i = 0; i < P->nx; ++i)
        g->W[gidx(g, f, j + oy, i + NG)] = W[((size_t)f * P->ny + j) * P->nx + i];
  for (int f = 0; f < P->nv * P->ndim; ++f)
    for (int j = 0; j < P->ny; ++j)
      for (int i = 0; i < P->nx; ++i)
        g->dW[gidx(g, f, j + oy, i + NG)] = dW[((size_t)f * P->ny + j) * P->nx + i];
}

/* Periodic: ghost cells copy the periodic image (values and all gradients).
 * Transmissive: ghost value = nearest interior cell, ghost gradient normal to
 * that boundary = 0, tangential gradient = nearest interior cell.
 * 2-D: x-ghosts of the interior rows first, then y-ghosts of every column,
 * which fills the corners. */
/* Boundary codes: 0 periodic, 1 transmissive (nearest interior cell, zero
 * normal derivative), 2 reflecting wall (mirror image: the normal momentum
 * changes sign; a derivative normal to the wall changes sign unless its
 * field does, a tangential one changes sign with its field), 3 fixed states
 * (1-D: given averages and gradients of the ghost cells, as an inflow state
 * or a fixed wave profile). */
static double wall_sign_w(int f, int m) { return f == m ? -1.0 : 1.0; }

static void fill_ghosts(const ocfg *P, gstate *g) {
  int nv = P->nv, nx = P->nx, ny = P->ny;
  int oy = (P->ndim == 1) ? 0 : NG;
  int j0 = oy, j1 = oy + ny;
  for (int j = j0; j < j1; ++j) {
    for (int gl = 1; gl <= NG; ++gl) {
      int il = NG - gl, ih = NG + nx - 1 + gl;          /* ghost columns */
      int sl, sh;
      if (P->bc[0] == 0) sl = NG + nx - gl; else if (P->bc[0] == 2) sl = NG + gl - 1; else sl = NG;
      if (P->bc[1] == 0) sh = NG + gl - 1; else if (P->bc[1] == 2) sh = NG + nx - gl; else sh = NG + nx - 1;
      for (int f = 0; f < nv; ++f) {
        g->W[gidx(g, f, j, il)] = (P->bc[0] == 2 ? wall_sign_w(f, 1) : 1.0) * g->W[gidx(g, f, j, sl)];
        g->W[gidx(g, f, j, ih)] = (P->bc[1] == 2 ? wall_sign_w(f, 1) : 1.0) * g->W[gidx(g, f, j, sh)];
      }
      for (int d = 0; d < P->ndim; ++d)
        for (int f = 0; f < nv; ++f) {
          int ff = d * nv + f;
          double vl = g->dW[gidx(g, ff, j, sl)], vh = g->dW[gidx(g, ff, j, sh)];
          if (d == 0 && P->bc[0] == 1) vl = 0.0;
          if (d == 0 && P->bc[1] == 1) vh = 0.0;
          if (P->bc[0] == 2) vl *= wall_sign_w(f, 1) * (d == 0 ? -1.0 : 1.0);
          if (P->bc[1] == 2) vh *= wall_sign_w(f, 1) * (d == 0 ? -1.0 : 1.0);
          g->dW[gidx(g, ff, j, il)] = vl;
          g->dW[gidx(g, ff, j, ih)] = vh;
        }
      if (P->ndim == 1)   /* fixed ends overwrite the images */
        for (int f = 0; f < nv; ++f) {
          if (P->bc[0] == 3) {
            g->W[gidx(g, f, j, il)] = P->ghost[0][gl - 1][f];
            g->dW[gidx(g, f, j, il)] = P->ghost[0][gl - 1][3 + f];
          }
          if (P->bc[1] == 3) {
            g->W[gidx(g, f, j, ih)] = P->ghost[1][gl - 1][f];
            g->dW[gidx(g, f, j, ih)] = P->ghost[1][gl - 1][3 + f];
          }
        }
    }
  }
  if (P->ndim == 1) return;
  for (int i = 0; i < g->nxt; ++i) {
    for (int gl = 1; gl <= NG; ++gl) {
      int jl = NG - gl, jh = NG + ny - 1 + gl;
      int sl, sh;
      if (P->bc[2] == 0) sl = NG + ny - gl; else if (P->bc[2] == 2) sl = NG + gl - 1; else sl = NG;
      if (P->bc[3] == 0) sh = NG + gl - 1; else if (P->bc[3] == 2) sh = NG + ny - gl; else sh = NG + ny - 1;
      for (int f = 0; f < nv; ++f) {
        g->W[gidx(g, f, jl, i)] = (P->bc[2] == 2 ? wall_sign_w(f, 2) : 1.0) * g->W[gidx(g, f, sl, i)];
        g->W[gidx(g, f, jh, i)] = (P->bc[3] == 2 ? wall_sign_w(f, 2) : 1.0) * g->W[gidx(g, f, sh, i)];
      }
      for (int d = 0; d < 2; ++d)
        for (int f = 0; f < nv; ++f) {
          int ff = d * nv + f;
          double vl = g->dW[gidx(g, ff, sl, i)], vh = g->dW[gidx(g, ff, sh, i)];
          if (d == 1 && P->bc[2] == 1) vl = 0.0;
          if (d == 1 && P->bc[3] == 1) vh = 0.0;
          if (P->bc[2] == 2) vl *= wall_sign_w(f, 2) * (d == 1 ? -1.0 : 1.0);
          if (P->bc[3] == 2) vh *= wall_sign_w(f, 2) * (d == 1 ? -1.0 : 1.0);
          g->dW[gidx(g, ff, jl, i)] = vl;
          g->dW[gidx(g, ff, jh, i)] = vh;
        }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* GKS flux at one point (reading: standard BGK interface solution)        */
/* ---------------------------------------------------------------------- */
/* Polynomials in (u, v, z) with z = xi^2 (sum of squared internal
 * velocities), stored as a list of terms c * u^i v^j z^k.
 * Degree bounds: u <= 7, v <= 7, z <= 3 (the second time derivative of the
 * interface state needs moments of psi times degree-5 polynomials). */
#define DU 8
#define DV 8
#define DZ 4
#define MAXT 128
typedef struct { int n; unsigned char e[MAXT][3]; double c[MAXT]; } poly;

static void poly_zero(poly *p) { p->n = 0; }

/* adds c u^i v^j z^k, merging with an existing term of the same monomial */
static void poly_add_term(poly *p, int i, int j, int k, double c) {
  if (i >= DU || j >= DV || k >= DZ) abort();        /* degree bound exceeded */
  for (int t = 0; t < p->n; ++t)
    if (p->e[t][0] == i && p->e[t][1] == j && p->e[t][2] == k) { p->c[t] += c; return; }
  if (p->n >= MAXT) abort();
  p->e[p->n][0] = (unsigned char)i; p->e[p->n][1] = (unsigned char)j; p->e[p->n][2] = (unsigned char)k;
  p->c[p->n] = c; ++p->n;
}

static void poly_add(poly *p, const poly *q, double s) {
  for (int t = 0; t < q->n; ++t) poly_add_term(p, q->e[t][0], q->e[t][1], q->e[t][2], s * q->c[t]);
}

static void poly_mul(const poly *a, const poly *b, poly *out) {
  poly r; poly_zero(&r);
  for (int x = 0; x < a->n; ++x)
    for (int y = 0; y < b->n; ++y)
      poly_add_term(&r, a->e[x][0] + b->e[y][0], a->e[x][1] + b->e[y][1], a->e[x][2] + b->e[y][2],
                    a->c[x] * b->c[y]);
  *out = r;
}

/* Moments of a Maxwellian normalised by its density, over all velocities or
 * over one half-space of u. */
typedef struct { double mu[DU], mv[DV], mz[DZ]; } mtab;

/* half: 0 full space, +1 for u > 0, -1 for u < 0 */
static void moments(double U, double V, double lam, double K, int half, int has_v, mtab *m) {
  if (half == 0) { m->mu[0] = 1.0; m->mu[1] = U; }
  else {
    double t0 = 0.5 * erfc(-half * sqrt(lam) * U);
    double t1 = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    m->mu[0] = t0;
    m->mu[1] = U * t0 + half * t1;
  }
  for (int n = 0; n + 2 < DU; ++n)
    m->mu[n + 2] = U * m->mu[n + 1] + (n + 1) / (2.0 * lam) * m->mu[n];
  for (int n = 0; n < DV; ++n) m->mv[n] = 0.0;
  m->mv[0] = 1.0;
  if (has_v) {
    m->mv[1] = V;
    for (int n = 0; n + 2 < DV; ++n)
      m->mv[n + 2] = V * m->mv[n + 1] + (n + 1) / (2.0 * lam) * m->mv[n];
  }
  /* <z^n> over the K internal degrees of freedom: prod_{i<n} (K + 2i) / (2 lam)^n */
  m->mz[0] = 1.0;
  for (int n = 1; n < DZ; ++n) m->mz[n] = m->mz[n - 1] * (K + 2.0 * (n - 1)) / (2.0 * lam);
}

static double poly_moment(const poly *p, const mtab *m) {
  double s = 0.0;
  for (int t = 0; t < p->n; ++t) s += p->c[t] * m->mu[p->e[t][0]] * m->mv[p->e[t][1]] * m->mz[p->e[t][2]];
  return s;
}

/* collision invariants psi = (1, u, [v,] (u^2 [+ v^2] + z)/2) */
static void psi_poly(int nv, int k, poly *p) {
  poly_zero(p);
  if (k == 0) poly_add_term(p, 0, 0, 0, 1.0);
  else if (k == 1) poly_add_term(p, 1, 0, 0, 1.0);
  else if (k == 2 && nv == 4) poly_add_term(p, 0, 1, 0, 1.0);
  else {
    poly_add_term(p, 2, 0, 0, 0.5); poly_add_term(p, 0, 0, 1, 0.5);
    if (nv == 4) poly_add_term(p, 0, 2, 0, 0.5);
  }
}

/* psi_k and psi_i psi_k as polynomials, built once (index 0: 1-D, 1: 2-D) */
static poly PSI[2][4], PSIPSI[2][4][4];
static void build_psi(void) {
  for (int d = 0; d < 2; ++d) {
    int nv = d ? 4 : 3;
    for (int k = 0; k < nv; ++k) psi_poly(nv, k, &PSI[d][k]);
    for (int i = 0; i < nv; ++i)
      for (int k = 0; k < nv; ++k) poly_mul(&PSI[d][i], &PSI[d][k], &PSIPSI[d][i][k]);
  }
}

/* a . psi as a polynomial */
static void slope_poly(int nv, const double *a, poly *p) {
  poly_zero(p);
  for (int k = 0; k < nv; ++k) poly_add(p, &PSI[nv == 4][k], a[k]);
}

/* <w psi_k> for k = 0..nv-1 */
static void moment_vec(int nv, const poly *w, const mtab *m, double *out) {
  for (int k = 0; k < nv; ++k) {
    poly r; poly_mul(w, &PSI[nv == 4][k], &r);
    out[k] = poly_moment(&r, m);
  }
}

typedef struct { double rho, U, V, lam; } prim;

static prim to_prim(const ocfg *P, const double *W) {
  prim p;
  p.rho = W[0];
  p.U = W[1] / W[0];
  p.V = (P->nv == 4) ? W[2] / W[0] : 0.0;
  double rE = W[P->nv - 1];
  double pr = (P->gamma - 1.0) * (rE - 0.5 * p.rho * (p.U * p.U + p.V * p.V));
  p.lam = p.rho / (2.0 * pr);
  return p;
}

/* micro slope a with <a psi> = w over the full-space Maxwellian of pr:
 * Gaussian elimination on the moment matrix M_ik = <psi_i psi_k>. */
static void micro_slope(const ocfg *P, const prim *pr, const double *w, double *a) {
  int nv = P->nv;
  mtab m; moments(pr->U, pr->V, pr->lam, P->K, 0, nv == 4, &m);
  double A[16], b[4];
  for (int i = 0; i < nv; ++i) {
    for (int k = 0; k < nv; ++k) A[i * nv + k] = poly_moment(&PSIPSI[nv == 4][i][k], &m);
    b[i] = w[i];
  }
  solve_d(nv, A, b);
  for (int i = 0; i < nv; ++i) a[i] = b[i];
}

/* Time derivative A from the compatibility condition
 * <(a u + b v + A) psi> = 0 over the full-space Maxwellian of pr. */
static void time_slope(const ocfg *P, const prim *pr, const double *a, const double *b, double *At) {
  int nv = P->nv;
  mtab m; moments(pr->U, pr->V, pr->lam, P->K, 0, nv == 4, &m);
  poly pa, pb, ua, vb, s, u1, v1;
  slope_poly(nv, a, &pa);
  poly_zero(&u1); poly_add_term(&u1, 1, 0, 0, 1.0);
  poly_mul(&pa, &u1, &ua);
  s = ua;
  if (nv == 4) {
    slope_poly(nv, b, &pb);
    poly_zero(&v1); poly_add_term(&v1, 0, 1, 0, 1.0);
    poly_mul(&pb, &v1, &vb);
    poly_add(&s, &vb, 1.0);
  }
  double rhs[4]; moment_vec(nv, &s, &m, rhs);
  for (int k = 0; k < nv; ++k) rhs[k] = -rhs[k];
  micro_slope(P, pr, rhs, At);
}

/* (a.psi)(b.psi) and u (a.psi) / v (a.psi) as polynomials */
static void prod_poly(const poly *a, const poly *b, poly *out) { poly_mul(a, b, out); }
static void u_times(const poly *a, poly *out) {
  poly u1; poly_zero(&u1); poly_add_term(&u1, 1, 0, 0, 1.0); poly_mul(a, &u1, out);
}
static void v_times(const poly *a, poly *out) {
  poly v1; poly_zero(&v1); poly_add_term(&v1, 0, 1, 0, 1.0); poly_mul(a, &v1, out);
}

/* Second time derivative of the equilibrium state at the interface (Euler
 * level; the time stepping of the gradients applies the two-stage
 * fourth-order structure to the interface values and needs it). The
 * equilibrium g = rho_c g~ of W_c varies in space and time with micro-slopes:
 * d_x g = g a, d_y g = g b, d_t g = g A, and
 *   d_x (g a) = g (a a + a_x),  d_y (g a) = g (b a + a_y),  a_y = b_x, ...
 * Taking moments, with M x = <x psi> over g~:
 *   M a_x = W_xx / rho - <a a psi>, M a_y = W_xy / rho - <a b psi>,
 *   M b_y = W_yy / rho - <b b psi>;
 *   M A = -<(u a + v b) psi> (compatibility);
 *   M A_x = -<(u (a a + a_x) + v (a b + b_x)) psi> - <a A psi>,
 *   M A_y = -<(u (a b + a_y) + v (b b + b_y)) psi> - <b A psi>
 * (the x and y derivatives of the compatibility condition), and
 *   W_tt = -d_x <u psi g A> - d_y <v psi g A>
 *        = -rho <(u (a A + A_x) + v (b A + A_y)) psi>.
 * ac, bc, Ac: the equilibrium micro-slopes; sxx, sxy, syy: physical second
 * derivatives (face frame, x normal). 1-D drops every v and y term. */
static void equilibrium_wtt(const ocfg *P, const prim *pc, const double *ac, const double *bc,
                            const double *Ac, const double *sxx, const double *sxy,
                            const double *syy, double *Wtt) {
  int nv = P->nv, has_v = (nv == 4);
  mtab mc; moments(pc->U, pc->V, pc->lam, P->K, 0, has_v, &mc);
  poly pa, pb, pA, aa, ab, bb, aA, bA, tmp, t2, sum;
  slope_poly(nv, ac, &pa);
  slope_poly(nv, Ac, &pA);
  prod_poly(&pa, &pa, &aa);
  prod_poly(&pa, &pA, &aA);
  double rhs[4] = {0, 0, 0, 0}, ax[4], ay[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0}, Ax[4];
  double Ay[4] = {0, 0, 0, 0};
  double m1[4], m2[4];
  /* a_x */
  moment_vec(nv, &aa, &mc, m1);
  for (int k = 0; k < nv; ++k) rhs[k] = sxx[k] / pc->rho - m1[k];
  micro_slope(P, pc, rhs, ax);
  if (has_v) {
    slope_poly(nv, bc, &pb);
    prod_poly(&pa, &pb, &ab);
    prod_poly(&pb, &pb, &bb);
    prod_poly(&pb, &pA, &bA);
    moment_vec(nv, &ab, &mc, m1);
    for (int k = 0; k < nv; ++k) rhs[k] = sxy[k] / pc->rho - m1[k];
    micro_slope(P, pc, rhs, ay);                 /* = b_x */
    moment_vec(nv, &bb, &mc, m1);
    for (int k = 0; k < nv; ++k) rhs[k] = syy[k] / pc->rho - m1[k];
    micro_slope(P, pc, rhs, by);
  }
  poly pax, pay, pby;
  slope_poly(nv, ax, &pax);
  /* A_x */
  sum = aa; poly_add(&sum, &pax, 1.0); u_times(&sum, &tmp);
  if (has_v) {
    slope_poly(nv, ay, &pay);
    slope_poly(nv, by, &pby);
    t2 = ab; poly_add(&t2, &pay, 1.0); v_times(&t2, &sum); poly_add(&tmp, &sum, 1.0);
  }
  poly_add(&tmp, &aA, 1.0);
  moment_vec(nv, &tmp, &mc, m1);
  for (int k = 0; k < nv; ++k) rhs[k] = -m1[k];
  micro_slope(P, pc, rhs, Ax);
  if (has_v) {
    /* A_y */
    sum = ab; poly_add(&sum, &pay, 1.0); u_times(&sum, &tmp);
    t2 = bb; poly_add(&t2, &pby, 1.0); v_times(&t2, &sum); poly_add(&tmp, &sum, 1.0);
    poly_add(&tmp, &bA, 1.0);
    moment_vec(nv, &tmp, &mc, m1);
    for (int k = 0; k < nv; ++k) rhs[k] = -m1[k];
    micro_slope(P, pc, rhs, Ay);
  }
  /* W_tt */
  poly pAx, pAy;
  slope_poly(nv, Ax, &pAx);
  sum = aA; poly_add(&sum, &pAx, 1.0); u_times(&sum, &tmp);
  if (has_v) {
    slope_poly(nv, Ay, &pAy);
    t2 = bA; poly_add(&t2, &pAy, 1.0); v_times(&t2, &sum); poly_add(&tmp, &sum, 1.0);
  }
  moment_vec(nv, &tmp, &mc, m2);
  for (int k = 0; k < nv; ++k) Wtt[k] = -pc->rho * m2[k];
}

/* Weight of the second-order term of the interface value at a point with
 * side states pl, pr (see gks_point). */
#define SECOND_ORDER_R0 1e-1
#define SECOND_ORDER_R1 1e-2
static double second_order_weight(const ocfg *P, const prim *pl, const prim *pr,
                                  const double *Wl, const double *Wr,
                                  const double *dnl, const double *dnr, double dt) {
  double prl = pl->rho / (2.0 * pl->lam), prr = pr->rho / (2.0 * pr->lam);
  double cl = sqrt(P->gamma * prl / pl->rho), cr = sqrt(P->gamma * prr / pr->rho);
  double r = fabs(prl - prr) / (prl + prr);
  double rr = fabs(pl->rho - pr->rho) / (pl->rho + pr->rho);
  double ru = fabs(pl->U - pr->U) / (cl + cr), rv = fabs(pl->V - pr->V) / (cl + cr);
  if (rr > r) r = rr;
  if (ru > r) r = ru;
  if (rv > r) r = rv;
  double cb = 0.5 * (cl + cr), rs = pl->rho + pr->rho;
  for (int k = 0; k < P->nv; ++k) {
    double sc = (k == 0) ? rs : (k == P->nv - 1) ? fabs(Wl[k]) + fabs(Wr[k]) : rs * cb;
    double rd = dt * cb * fabs(dnl[k] - dnr[k]) / sc;
    if (rd > r) r = rd;
  }
  if (r <= SECOND_ORDER_R1) return 1.0;
  double x = (r - SECOND_ORDER_R1) / (SECOND_ORDER_R0 - SECOND_ORDER_R1);
  return x < 1.0 ? 1.0 - x * x : 0.0;
}

/* Integrated flux over [0, delta] and the interface state at t = delta of
 * the BGK solution
 *   f = (1 - e) g0 + ((t+tau) e - tau)(abar u + bbar v) g0 + (t - tau(1 - e)) Abar g0
 *     + e sum_s H_s g_s [1 - (t + tau)(a_s u + b_s v) - tau A_s],  e = exp(-t/tau)
 * at one point of a face. Inputs are in the face frame (normal velocity
 * first). dn*, dt*: physical normal / tangential derivatives of the left and
 * right conserved states; snn, snt, stt: physical second derivatives of the
 * point (normal-normal, normal-tangential, tangential-tangential; 1-D: snn
 * only), averaged over the sides. Outputs the fitted F, dF/dt (from delta =
 * dt/2 and dt), the interface state W(dt/2) and W(dt) of the solution, and
 * the weighted equilibrium second time derivative phi W_tt. */
static void gks_point(const ocfg *P, const double *Wl, const double *Wr,
                      const double *dnl, const double *dnr, const double *dtl,
                      const double *dtr, const double *snn, const double *snt,
                      const double *stt, double dt, double *F, double *Ft, double *Wh,
                      double *Wf, double *Wtt) {
  int nv = P->nv, has_v = (nv == 4);
  double K = P->K;
  prim pl = to_prim(P, Wl), pr = to_prim(P, Wr);
  mtab ml_half, mr_half;
  moments(pl.U, pl.V, pl.lam, K, +1, has_v, &ml_half);
  moments(pr.U, pr.V, pr.lam, K, -1, has_v, &mr_half);
  /* interface equilibrium W^c from the half-space sums */
  poly one; poly_zero(&one); poly_add_term(&one, 0, 0, 0, 1.0);
  double hl[4], hr[4], Wc[4];
  moment_vec(nv, &one, &ml_half, hl);
  moment_vec(nv, &one, &mr_half, hr);
  for (int k = 0; k < nv; ++k) Wc[k] = pl.rho * hl[k] + pr.rho * hr[k];
  prim pc = to_prim(P, Wc);
  mtab mc; moments(pc.U, pc.V, pc.lam, K, 0, has_v, &mc);

  /* spatial micro-slopes */
  double w[4] = {0, 0, 0, 0}, al[4], ar[4], bl[4] = {0, 0, 0, 0}, br[4] = {0, 0, 0, 0};
  double ac[4], bc[4] = {0, 0, 0, 0};
  for (int k = 0; k < nv; ++k) w[k] = dnl[k] / pl.rho;
  micro_slope(P, &pl, w, al);
  for (int k = 0; k < nv; ++k) w[k] = dnr[k] / pr.rho;
  micro_slope(P, &pr, w, ar);
  for (int k = 0; k < nv; ++k) w[k] = 0.5 * (dnl[k] + dnr[k]) / pc.rho;
  micro_slope(P, &pc, w, ac);
  if (has_v) {
    for (int k = 0; k < nv; ++k) w[k] = dtl[k] / pl.rho;
    micro_slope(P, &pl, w, bl);
    for (int k = 0; k < nv; ++k) w[k] = dtr[k] / pr.rho;
    micro_slope(P, &pr, w, br);
    for (int k = 0; k < nv; ++k) w[k] = 0.5 * (dtl[k] + dtr[k]) / pc.rho;
    micro_slope(P, &pc, w, bc);
  }
  /* time slopes from compatibility */
  double Al[4], Ar[4], Ac[4];
  time_slope(P, &pl, al, bl, Al);
  time_slope(P, &pr, ar, br, Ar);
  time_slope(P, &pc, ac, bc, Ac);
  /* The second-order term of the interface value (reading): phi W_tt, the
   * equilibrium's W_tt weighted by phi(r), r the largest jump between the
   * two sides relative to its scale: of the states (pressure and density:
   * |a_l - a_r| / (a_l + a_r); velocity components: over the sum of the
   * sound speeds) and of the normal derivatives over the distance a sound
   * wave covers in dt (dt c |d_l - d_r| over the variable's scale: the
   * density sum, that sum times c for the momenta, the energy sum; c the
   * mean sound speed). phi = 1 for r <= r1 = 1e-2, 1 - x^2 with
   * x = (r - r1) / (r0 - r1) up to r0 = 1e-1, and 0 beyond: 1 for smooth
   * data, whose two sides agree in state and slope up to the truncation
   * error, and 0 at a discontinuity of the state or of its slope (a shock,
   * a contact, the foot of a shock), where the interface value keeps the
   * BGK solution's own time dependence. phi is continuous, and exactly 1
   * over the range of smooth data. */
  double phi = second_order_weight(P, &pl, &pr, Wl, Wr, dnl, dnr, dt);
  if (phi > 0.0) {
    equilibrium_wtt(P, &pc, ac, bc, Ac, snn, snt, stt, Wtt);
    for (int k = 0; k < nv; ++k) Wtt[k] *= phi;
  } else {
    for (int k = 0; k < nv; ++k) Wtt[k] = 0.0;
  }

  /* moment vectors */
  poly u1, v1, pa, pb, t1, t2, uone;
  poly_zero(&u1); poly_add_term(&u1, 1, 0, 0, 1.0);
  poly_zero(&v1); poly_add_term(&v1, 0, 1, 0, 1.0);
  uone = u1;
  /* (a u + b v) polynomial for a given pair */
  #define SPACE_POLY(A_, B_, OUT_) do { \
      slope_poly(nv, A_, &pa); poly_mul(&pa, &u1, &t1); OUT_ = t1; \
      if (has_v) { slope_poly(nv, B_, &pb); poly_mul(&pb, &v1, &t2); poly_add(&OUT_, &t2, 1.0); } \
    } while (0)

  poly sc, sl, sr, Acp, Alp, Arp, tmp;
  SPACE_POLY(ac, bc, sc);
  SPACE_POLY(al, bl, sl);
  SPACE_POLY(ar, br, sr);
  slope_poly(nv, Ac, &Acp);
  slope_poly(nv, Al, &Alp);
  slope_poly(nv, Ar, &Arp);

  /* flux moments <u X psi> and state moments <X psi> */
  double c_u[4], c_us[4], c_uA[4], c_1[4], c_s[4], c_A[4];
  double l_u[4], l_us[4], l_uA[4], l_1[4], l_s[4], l_A[4];
  double r_u[4], r_us[4], r_uA[4], r_1[4], r_s[4], r_A[4];
  moment_vec(nv, &uone, &mc, c_u);
  poly_mul(&sc, &u1, &tmp); moment_vec(nv, &tmp, &mc, c_us);
  poly_mul(&Acp, &u1, &tmp); moment_vec(nv, &tmp, &mc, c_uA);
  moment_vec(nv, &one, &mc, c_1);
  moment_vec(nv, &sc, &mc, c_s);
  moment_vec(nv, &Acp, &mc, c_A);
  moment_vec(nv, &uone, &ml_half, l_u);
  poly_mul(&sl, &u1, &tmp); moment_vec(nv, &tmp, &ml_half, l_us);
  poly_mul(&Alp, &u1, &tmp); moment_vec(nv, &tmp, &ml_half, l_uA);
  moment_vec(nv, &one, &ml_half, l_1);
  moment_vec(nv, &sl, &ml_half, l_s);
  moment_vec(nv, &Alp, &ml_half, l_A);
  moment_vec(nv, &uone, &mr_half, r_u);
  poly_mul(&sr, &u1, &tmp); moment_vec(nv, &tmp, &mr_half, r_us);
  poly_mul(&Arp, &u1, &tmp); moment_vec(nv, &tmp, &mr_half, r_uA);
  moment_vec(nv, &one, &mr_half, r_1);
  moment_vec(nv, &sr, &mr_half, r_s);
  moment_vec(nv, &Arp, &mr_half, r_A);
  #undef SPACE_POLY

  /* collision time (reading): tau = C1 dt + C2 dt |pl - pr| / (pl + pr) */
  double prl = pl.rho / (2.0 * pl.lam), prr = pr.rho / (2.0 * pr.lam);
  double tau = P->tc1 * dt + P->tc2 * dt * fabs(prl - prr) / (prl + prr);

  double Fd[2][4];
  for (int q = 0; q < 2; ++q) {
    double del = (q == 0) ? 0.5 * dt : dt;
    double c1, c2, c3, c4, c5, c6;
    if (tau > 0.0) {
      double e = exp(-del / tau);
      double em = -expm1(-del / tau);
      /* time integrals of the weights of the BGK solution over [0, del] */
      c1 = del - tau * em;
      c5 = 2.0 * tau * tau - tau * (del + 2.0 * tau) * e;
      c2 = c5 - tau * del;
      c3 = 0.5 * del * del - tau * del + tau * tau * em;
      c4 = tau * em;
      c6 = tau * tau * em;
    } else {
      c1 = del; c2 = 0.0; c3 = 0.5 * del * del; c4 = 0.0; c5 = 0.0; c6 = 0.0;
    }
    for (int k = 0; k < nv; ++k) {
      Fd[q][k] = pc.rho * (c1 * c_u[k] + c2 * c_us[k] + c3 * c_uA[k])
               + pl.rho * (c4 * l_u[k] - c5 * l_us[k] - c6 * l_uA[k])
               + pr.rho * (c4 * r_u[k] - c5 * r_us[k] - c6 * r_uA[k]);
    }
  }
  /* fit F(t) = F + t dF/dt to the two integrals */
  for (int k = 0; k < nv; ++k) {
    F[k] = (4.0 * Fd[0][k] - Fd[1][k]) / dt;
    Ft[k] = 4.0 * (Fd[1][k] - 2.0 * Fd[0][k]) / (dt * dt);
  }
  /* interface state at t = dt/2 and t = dt */
  for (int q = 0; q < 2; ++q) {
    double del = (q == 0) ? 0.5 * dt : dt, e, em, k1, k2, k3, k4, k5;
    if (tau > 0.0) {
      e = exp(-del / tau); em = -expm1(-del / tau);
      k1 = em; k2 = (del + tau) * e - tau; k3 = del - tau * em;
      k4 = del + tau; k5 = tau;
    } else {
      e = 0.0; em = 1.0; k1 = 1.0; k2 = 0.0; k3 = del; k4 = 0.0; k5 = 0.0;
    }
    double *Wo = (q == 0) ? Wh : Wf;
    for (int k = 0; k < nv; ++k) {
      Wo[k] = pc.rho * (k1 * c_1[k] + k2 * c_s[k] + k3 * c_A[k])
            + e * (pl.rho * (l_1[k] - k4 * l_s[k] - k5 * l_A[k])
                 + pr.rho * (r_1[k] - k4 * r_s[k] - k5 * r_A[k]));
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Face states                                                             */
/* ---------------------------------------------------------------------- */
/* A reconstructed point state is admissible if rho > 0, p > 0 and finite
 * (reading; the paper applies no positivity fix-up). */
static int admissible(const ocfg *P, const double *W) {
  for (int k = 0; k < P->nv; ++k) if (!isfinite(W[k])) return 0;
  if (!(W[0] > 0.0)) return 0;
  double ke = 0.0;
  for (int k = 1; k < P->nv - 1; ++k) ke += W[k] * W[k];
  double p = (P->gamma - 1.0) * (W[P->nv - 1] - 0.5 * ke / W[0]);
  return p > 0.0;
}

/* Normal GENO for the face between cells (i, j) and (i+1, j) along x (dir 0)
 * or between (i, j) and (i, j+1) along y (dir 1) in ghosted coordinates.
 * out[side][quant][var]: quant 0 value, 1 h * normal derivative, 2 h^2 * second
 * normal derivative; chi[side][var]. */
/* Characteristic variables (reading; the paper does not name the variables
 * it reconstructs): right eigenvectors of the Euler flux Jacobian in the
 * normal direction `dir` at the Roe average of the two cells at the face.
 * In the normal frame (normal velocity un, tangential ut) the columns belong
 * to the speeds un - c, un, un (shear, 2-D only), un + c; the left vectors are
 * the inverse matrix, by Gaussian elimination. Components are stored in the
 * state order (rho, rho U, [rho V,] rho E), so along y the two momentum rows
 * trade places. Returns nonzero when the average has no real sound speed
 * (the face then keeps the conservative variables). */
static int roe_eigen(const ocfg *P, int dir, const double *Wa, const double *Wb,
                     double R[4][4], double L[4][4]) {
  const int nv = P->nv, e = nv - 1;
  const int in = 1 + dir, it = 2 - dir;   /* normal and (2-D) tangential momentum */
  const double g = P->gamma;
  double sa = sqrt(Wa[0]), sb = sqrt(Wb[0]);
  double vel[2][3], H[2];
  const double *Ws[2] = {Wa, Wb};
  for (int s = 0; s < 2; ++s) {
    const double *W = Ws[s];
    double ke = 0.0;
    for (int k = 1; k < e; ++k) { vel[s][k] = W[k] / W[0]; ke += W[k] * vel[s][k]; }
    double p = (g - 1.0) * (W[e] - 0.5 * ke);
    H[s] = (W[e] + p) / W[0];
  }
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = 1; k < e; ++k) v[k] = (sa * vel[0][k] + sb * vel[1][k]) / (sa + sb);
  const double Hr = (sa * H[0] + sb * H[1]) / (sa + sb);
  double q2 = 0.0;
  for (int k = 1; k < e; ++k) q2 += v[k] * v[k];
  const double c2 = (g - 1.0) * (Hr - 0.5 * q2);
  if (!(c2 > 0.0)) return 1;
  const double c = sqrt(c2), un = v[in];
  double Rm[4][4];
  memset(Rm, 0, sizeof Rm);
  /* acoustic and entropy columns: 0 (un - c), 1 (un), nv - 1 (un + c) */
  const int cols[3] = {0, 1, nv - 1};
  const double shift[3] = {-c, 0.0, c};
  for (int q = 0; q < 3; ++q) {
    int col = cols[q];
    Rm[0][col] = 1.0;
    for (int k = 1; k < e; ++k) Rm[k][col] = v[k];
    Rm[in][col] += shift[q];
    Rm[e][col] = (q == 1) ? 0.5 * q2 : Hr + shift[q] * un;
  }
  if (nv == 4) {   /* shear column: tangential momentum */
    Rm[it][2] = 1.0;
    Rm[e][2] = v[it];
  }
  for (int col = 0; col < nv; ++col) {
    double A[16], b[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < nv; ++r)
      for (int k = 0; k < nv; ++k) A[r * nv + k] = Rm[r][k];
    b[col] = 1.0;
    if (solve_d(nv, A, b)) return 1;
    for (int r = 0; r < nv; ++r) L[r][col] = b[r];
  }
  for (int r = 0; r < nv; ++r)
    for (int k = 0; k < nv; ++k) R[r][k] = Rm[r][k];
  return 0;
}

static void normal_face(const ocfg *P, const gstate *g, int dir, int i, int j,
                        double out[2][3][4], double chi[2][4]) {
  int nv = P->nv;
  double h = (dir == 0) ? P->dx : P->dy;
  double R[4][4], L[4][4];
  if (P->characteristic) {
    /* the two cells at the face are m = 0 and m = 1 of the normal stencil */
    double Wa[4], Wb[4];
    for (int v = 0; v < nv; ++v) {
      Wa[v] = g->W[gidx(g, v, j, i)];
      Wb[v] = g->W[gidx(g, v, dir == 0 ? j : j + 1, dir == 0 ? i + 1 : i)];
    }
    if (!roe_eigen(P, dir, Wa, Wb, R, L)) {
      double val[2][4], der[2][4], d2[2][4];
      for (int c = 0; c < nv; ++c) {
        double q[4] = {0, 0, 0, 0}, gg[4] = {0, 0, 0, 0};
        for (int m = -1; m <= 2; ++m) {
          int ii = (dir == 0) ? i + m : i, jj = (dir == 0) ? j : j + m;
          for (int v = 0; v < nv; ++v) {
            q[m + 1] += L[c][v] * g->W[gidx(g, v, jj, ii)];
            gg[m + 1] += L[c][v] * h * g->dW[gidx(g, dir * nv + v, jj, ii)];
          }
        }
        double l[4], r[4];
        geno_face(P, q, gg, l, r);
        val[0][c] = l[0]; der[0][c] = l[1]; chi[0][c] = l[2]; d2[0][c] = l[3];
        val[1][c] = r[0]; der[1][c] = r[1]; chi[1][c] = r[2]; d2[1][c] = r[3];
      }
      for (int s = 0; s < 2; ++s)
        for (int v = 0; v < nv; ++v) {
          double a0 = 0.0, a1 = 0.0, a2 = 0.0;
          for (int c = 0; c < nv; ++c) {
            a0 += R[v][c] * val[s][c]; a1 += R[v][c] * der[s][c]; a2 += R[v][c] * d2[s][c];
          }
          out[s][0][v] = a0;
          out[s][1][v] = a1;
          out[s][2][v] = a2;
        }
      return;
    }
  }
  for (int v = 0; v < nv; ++v) {
    double q[4], gg[4];
    for (int m = -1; m <= 2; ++m) {
      int ii = (dir == 0) ? i + m : i, jj = (dir == 0) ? j : j + m;
      q[m + 1] = g->W[gidx(g, v, jj, ii)];
      gg[m + 1] = h * g->dW[gidx(g, dir * nv + v, jj, ii)];
    }
    double l[4], r[4];
    geno_face(P, q, gg, l, r);
    out[0][0][v] = l[0]; out[0][1][v] = l[1]; out[0][2][v] = l[3]; chi[0][v] = l[2];
    out[1][0][v] = r[0]; out[1][1][v] = r[1]; out[1][2][v] = r[3]; chi[1][v] = r[2];
  }
}

/* Tangential step to a Gauss point (reading, 2-D only). phi[3] are the
 * face-averaged values of rows j-1, j, j+1 (one side, one variable); eta is
 * the Gauss point in units of the face length about the row centre. The
 * high-order candidate is the quadratic with these three averages; the
 * low-order one is the ENO combination (d = 1) of the two one-sided linear
 * polynomials; they are blended with the path function of Eq. (4)-(5) using
 * IS = h * int (p')^2 of each linear polynomial, IS^H = max, IS^L = min,
 * IS^tau = |IS_+ - IS_-|. Returns the value; *hder = h * tangential
 * derivative, *chi_t = the blend weight. */
static double tangential(const ocfg *P, const double phi[3], double eta, double *hder,
                         double *chi_t) {
  double c[3];
  for (int q = 0; q < 3; ++q) c[q] = TQ[q][0] * phi[0] + TQ[q][1] * phi[1] + TQ[q][2] * phi[2];
  double vH = c[0] + c[1] * eta + c[2] * eta * eta;
  double dH = c[1] + 2.0 * c[2] * eta;
  double sm = phi[1] - phi[0], sp = phi[2] - phi[1];
  double ISm = sm * sm, ISp = sp * sp;
  double ISH = ISm > ISp ? ISm : ISp, ISL = ISm < ISp ? ISm : ISp;
  double chi = path_function(P, fabs(ISp - ISm), ISH, ISL);
  double wm = 1.0 / pow(ISm + P->eps, P->rL), wp = 1.0 / pow(ISp + P->eps, P->rL);
  double sL = (wm / (wm + wp)) * sm + (wp / (wm + wp)) * sp;
  double vL = phi[1] + eta * sL;
  *hder = chi * dH + (1.0 - chi) * sL;
  if (chi_t) *chi_t = chi;
  return chi * vH + (1.0 - chi) * vL;
}

/* Second derivatives at the points of a face for the time stepping of the
 * gradients (reading, 2-D; the paper gives no structured 2-D scheme): per
 * side, h_t^2 d_tt = chi_t (phi_{j+1} - 2 phi_j + phi_{j-1}) (the second
 * derivative of the tangential quadratic, weighted like its value; the
 * low-order candidate is linear), and h_n h_t d_nt = chi_t (psi_{j+1} -
 * psi_{j-1}) / 2 from the h-scaled normal derivatives psi of the three rows;
 * h_n^2 d_nn is the normal step's value of the centre row. The point takes
 * the mean of the two sides (the averaged slopes of the equilibrium part of
 * the flux are taken the same way). */
static void side_second(const double phi[3], const double psi[3], double chi_t, double *stt,
                        double *snt) {
  *stt = chi_t * (phi[2] - 2.0 * phi[1] + phi[0]);
  *snt = chi_t * 0.5 * (psi[2] - psi[0]);
}

/* Gauss points of a face (reading of the 2-point rule on a face):
 * +-1/(2 sqrt 3) of the face length about its centre, weights 1/2. */
static const double GAUSS_ETA[2] = {-0.28867513459481288225, 0.28867513459481288225};

/* ---------------------------------------------------------------------- */
/* One stage: fluxes, Lagrangian, interface states                         */
/* ---------------------------------------------------------------------- */
/* Point data of Gauss point gp on the 2-D face with normal-step results
 * o[row t-1, t, t+1][side][quant][var] (x/y frame): per side the state, the
 * h-scaled normal and tangential derivatives after the tangential step and
 * the positivity guard, and the h-scaled second derivatives of the point
 * (h_n^2 d_nn, h_n h_t d_nt, h_t^2 d_tt; zero when a side is guarded).
 * (ci, cj)[side]: the own cells of the two sides. Returns the guard count. */
static int face_point(const ocfg *P, const gstate *g, double o[3][2][3][4], int gp,
                      const int ci[2], const int cj[2], double S[2][4], double Dn[2][4],
                      double Dt[2][4], double Sec[3][4]) {
  int nv = P->nv, guard = 0, ok[2];
  double ss[2][3][4];
  for (int side = 0; side < 2; ++side) {
    for (int v = 0; v < nv; ++v) {
      double phi[3] = {o[0][side][0][v], o[1][side][0][v], o[2][side][0][v]};
      double psi[3] = {o[0][side][1][v], o[1][side][1][v], o[2][side][1][v]};
      double chi_t;
      S[side][v] = tangential(P, phi, GAUSS_ETA[gp], &Dt[side][v], &chi_t);
      Dn[side][v] = o[1][side][1][v];
      ss[side][0][v] = o[1][side][2][v];
      side_second(phi, psi, chi_t, &ss[side][2][v], &ss[side][1][v]);
    }
    ok[side] = admissible(P, S[side]);
    if (!ok[side]) {
      ++guard;
      for (int v = 0; v < nv; ++v) {
        S[side][v] = g->W[gidx(g, v, cj[side], ci[side])]; Dn[side][v] = 0.0; Dt[side][v] = 0.0;
      }
    }
  }
  for (int q = 0; q < 3; ++q)
    for (int v = 0; v < nv; ++v)
      Sec[q][v] = (ok[0] && ok[1]) ? 0.5 * (ss[0][q][v] + ss[1][q][v]) : 0.0;
  return guard;
}

/* Per-face results for the stage (Gauss-averaged): F, dF/dt, the interface
 * state W(dt/2) and W(dt) of the BGK solution and the equilibrium second
 * time derivative W_tt. */
typedef struct {
  double *F[2], *Ft[2], *Wh[2], *Wf[2], *W2[2];   /* dir x / y: [nv][nfy][nfx] */
  int nfx[2], nfy[2];
  long long guard;
} faceres;

/* Computes all face quantities of a stage from the (ghost-filled) state. */
static void stage_faces(const ocfg *P, const gstate *g, double dt, faceres *fr) {
  int nv = P->nv, nx = P->nx, ny = P->ny;
  long long guard = 0;
  if (P->ndim == 1) {
    for (int f = 0; f <= nx; ++f) {
      int i = NG + f - 1;                 /* left cell of face f */
      double out[2][3][4], chi[2][4];
      normal_face(P, g, 0, i, 0, out, chi);
      double Wl[4], Wr[4], dl[4], dr[4], sxx[4];
      for (int v = 0; v < nv; ++v) {
        Wl[v] = out[0][0][v]; dl[v] = out[0][1][v] / P->dx;
        Wr[v] = out[1][0][v]; dr[v] = out[1][1][v] / P->dx;
        sxx[v] = 0.5 * (out[0][2][v] + out[1][2][v]) / (P->dx * P->dx);
      }
      int okl = admissible(P, Wl), okr = admissible(P, Wr);
      if (!okl) { ++guard; for (int v = 0; v < nv; ++v) { Wl[v] = g->W[gidx(g, v, 0, i)]; dl[v] = 0.0; } }
      if (!okr) { ++guard; for (int v = 0; v < nv; ++v) { Wr[v] = g->W[gidx(g, v, 0, i + 1)]; dr[v] = 0.0; } }
      if (!okl || !okr) for (int v = 0; v < nv; ++v) sxx[v] = 0.0;
      double F[4], Ft[4], Wh[4], Wf[4], W2[4];
      gks_point(P, Wl, Wr, dl, dr, NULL, NULL, sxx, NULL, NULL, dt, F, Ft, Wh, Wf, W2);
      for (int v = 0; v < nv; ++v) {
        size_t o = (size_t)v * (nx + 1) + f;
        fr->F[0][o] = F[v]; fr->Ft[0][o] = Ft[v];
        fr->Wh[0][o] = Wh[v]; fr->Wf[0][o] = Wf[v]; fr->W2[0][o] = W2[v];
      }
    }
    fr->guard += guard;
    return;
  }
  /* 2-D: dir 0 (x-faces) then dir 1 (y-faces) */
  for (int dir = 0; dir < 2; ++dir) {
    int nfn = (dir == 0) ? nx + 1 : ny + 1;   /* faces along the normal */
    int nt = (dir == 0) ? ny : nx;            /* rows along the tangent */
    double hn = (dir == 0) ? P->dx : P->dy;
    double ht = (dir == 0) ? P->dy : P->dx;
    long long gsum = 0;
#pragma omp parallel for schedule(static) reduction(+ : gsum)
    for (int t = 0; t < nt; ++t) {
      for (int f = 0; f < nfn; ++f) {
        /* normal reconstruction for rows t-1, t, t+1 */
        double out[3][2][3][4], chi[2][4];
        for (int dt_ = -1; dt_ <= 1; ++dt_) {
          int i, j;
          if (dir == 0) { i = NG + f - 1; j = NG + t + dt_; }
          else { i = NG + t + dt_; j = NG + f - 1; }
          normal_face(P, g, dir, i, j, out[dt_ + 1], chi);
        }
        /* own cells of the two sides in the centre row */
        int ci[2], cj[2];
        if (dir == 0) { ci[0] = NG + f - 1; ci[1] = NG + f; cj[0] = cj[1] = NG + t; }
        else { cj[0] = NG + f - 1; cj[1] = NG + f; ci[0] = ci[1] = NG + t; }
        double Fs[4] = {0, 0, 0, 0}, Fts[4] = {0, 0, 0, 0}, Whs[4] = {0, 0, 0, 0};
        double Wfs[4] = {0, 0, 0, 0}, W2s[4] = {0, 0, 0, 0};
        for (int gp = 0; gp < 2; ++gp) {
          double S[2][4], Dn[2][4], Dt[2][4], Sec[3][4];
          gsum += face_point(P, g, out, gp, ci, cj, S, Dn, Dt, Sec);
          /* rotate into the face frame: normal momentum first; physical units */
          double Wl[4], Wr[4], nl[4], nr[4], tl[4], tr[4], snn[4], snt[4], stt[4];
          int perm[4] = {0, 1, 2, 3};
          if (dir == 1) { perm[1] = 2; perm[2] = 1; }
          for (int v = 0; v < 4; ++v) {
            Wl[v] = S[0][perm[v]]; Wr[v] = S[1][perm[v]];
            nl[v] = Dn[0][perm[v]] / hn; nr[v] = Dn[1][perm[v]] / hn;
            tl[v] = Dt[0][perm[v]] / ht; tr[v] = Dt[1][perm[v]] / ht;
            snn[v] = Sec[0][perm[v]] / (hn * hn);
            snt[v] = Sec[1][perm[v]] / (hn * ht);
            stt[v] = Sec[2][perm[v]] / (ht * ht);
          }
          double F[4], Ft[4], Wh[4], Wf[4], W2[4];
          gks_point(P, Wl, Wr, nl, nr, tl, tr, snn, snt, stt, dt, F, Ft, Wh, Wf, W2);
          for (int v = 0; v < 4; ++v) {
            Fs[perm[v]] += 0.5 * F[v];
            Fts[perm[v]] += 0.5 * Ft[v];
            Whs[perm[v]] += 0.5 * Wh[v];
            Wfs[perm[v]] += 0.5 * Wf[v];
            W2s[perm[v]] += 0.5 * W2[v];
          }
        }
        int nfx = fr->nfx[dir];
        size_t base = (size_t)(dir == 0 ? t : f) * nfx + (dir == 0 ? f : t);
        size_t plane = (size_t)fr->nfx[dir] * fr->nfy[dir];
        for (int v = 0; v < 4; ++v) {
          fr->F[dir][v * plane + base] = Fs[v];
          fr->Ft[dir][v * plane + base] = Fts[v];
          fr->Wh[dir][v * plane + base] = Whs[v];
          fr->Wf[dir][v * plane + base] = Wfs[v];
          fr->W2[dir][v * plane + base] = W2s[v];
        }
      }
    }
    guard += gsum;
  }
  fr->guard += guard;
}

static int faceres_alloc(const ocfg *P, faceres *fr) {
  memset(fr, 0, sizeof *fr);
  fr->nfx[0] = P->nx + 1; fr->nfy[0] = P->ny;
  fr->nfx[1] = P->nx; fr->nfy[1] = P->ny + 1;
  int nd = P->ndim;
  for (int d = 0; d < nd; ++d) {
    size_t n = (size_t)fr->nfx[d] * fr->nfy[d] * P->nv;
    fr->F[d] = (double *)calloc(n, sizeof(double));
    fr->Ft[d] = (double *)calloc(n, sizeof(double));
    fr->Wh[d] = (double *)calloc(n, sizeof(double));
    fr->Wf[d] = (double *)calloc(n, sizeof(double));
    fr->W2[d] = (double *)calloc(n, sizeof(double));
    if (!fr->F[d] || !fr->Ft[d] || !fr->Wh[d] || !fr->Wf[d] || !fr->W2[d]) return -1;
  }
  return 0;
}
static void faceres_free(faceres *fr) {
  for (int d = 0; d < 2; ++d) {
    free(fr->F[d]); free(fr->Ft[d]); free(fr->Wh[d]); free(fr->Wf[d]); free(fr->W2[d]);
  }
}

/* L = -(1/|Omega|) sum faces F.n |Gamma| (Eq. (1)) and its time derivative. */
static void cell_terms(const ocfg *P, const faceres *fr, double *L, double *Lt) {
  int nv = P->nv, nx = P->nx, ny = P->ny;
  size_t ncell = (size_t)nx * ny;
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = (size_t)v * ncell + (size_t)j * nx + i;
        size_t px = (size_t)fr->nfx[0] * fr->nfy[0];
        size_t fxl = v * px + (size_t)j * fr->nfx[0] + i, fxh = fxl + 1;
        double l = -(fr->F[0][fxh] - fr->F[0][fxl]) / P->dx;
        double lt = -(fr->Ft[0][fxh] - fr->Ft[0][fxl]) / P->dx;
        if (P->ndim == 2) {
          size_t py = (size_t)fr->nfx[1] * fr->nfy[1];
          size_t fyl = v * py + (size_t)j * fr->nfx[1] + i, fyh = fyl + fr->nfx[1];
          l += -(fr->F[1][fyh] - fr->F[1][fyl]) / P->dy;
          lt += -(fr->Ft[1][fyh] - fr->Ft[1][fyl]) / P->dy;
        }
        L[c] = l; Lt[c] = lt;
      }
}

/* Cell-averaged gradients by the Gauss theorem, Eq. (2), from interface
 * values Wx (x-faces) and Wy (y-faces, 2-D), laid out like faceres. */
static void gauss_gradient(const ocfg *P, const faceres *fr, double *const Wface[2], double *G) {
  int nv = P->nv, nx = P->nx, ny = P->ny;
  size_t ncell = (size_t)nx * ny;
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = (size_t)v * ncell + (size_t)j * nx + i;
        size_t px = (size_t)fr->nfx[0] * fr->nfy[0];
        size_t fxl = v * px + (size_t)j * fr->nfx[0] + i, fxh = fxl + 1;
        G[c] = (Wface[0][fxh] - Wface[0][fxl]) / P->dx;
        if (P->ndim == 2) {
          size_t py = (size_t)fr->nfx[1] * fr->nfy[1];
          size_t fyl = v * py + (size_t)j * fr->nfx[1] + i, fyh = fyl + fr->nfx[1];
          G[(size_t)nv * ncell + c] = (Wface[1][fyh] - Wface[1][fyl]) / P->dy;
        }
      }
}

/* CFL time step (Sec. 6 uses CFL >= 0.5; reading of the 2-D form):
 * dt = CFL * min over cells of min(dx/(|U|+c), dy/(|V|+c)). */
static double cfl_dt(const ocfg *P, const double *W) {
  int nv = P->nv;
  size_t ncell = (size_t)P->nx * P->ny;
  double m = INFINITY;
  for (size_t c = 0; c < ncell; ++c) {
    double rho = W[c], U = W[ncell + c] / rho;
    double V = (nv == 4) ? W[2 * ncell + c] / rho : 0.0;
    double p = (P->gamma - 1.0) * (W[(nv - 1) * ncell + c] - 0.5 * rho * (U * U + V * V));
    double cs = sqrt(P->gamma * p / rho);
    double t = P->dx / (fabs(U) + cs);
    if (nv == 4) { double ty = P->dy / (fabs(V) + cs); if (ty < t) t = ty; }
    if (t < m) m = t;
  }
  return P->cfl * m;
}

/* ====================================================================== */
/* Exported entry points                                                   */
/* ====================================================================== */

int oracle_init(void) { return ops_ready ? OR_OK : (build_ops() ? OR_EINVAL : OR_OK); }

/* Linear-operator weights (for the polynomial-reproduction pins). */
int oracle_linear_weights(double *hval, double *hder) {
  if (oracle_init()) return OR_EINVAL;
  memcpy(hval, H_val, sizeof H_val);
  memcpy(hder, H_der, sizeof H_der);
  return OR_OK;
}

/* GENO at one face for one component: q, g = averages and h-scaled averaged
 * derivatives of cells j-1..j+2. out = (value_l, hder_l, chi_l, value_r,
 * hder_r, chi_r, h2der_l, h2der_r): h2der = h^2 * second derivative. */
int oracle_geno_face(const double *params, const double *q, const double *g, double *out) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, 1, 1, 1, 1.0, 1.0, params);
  double l[4], r[4];
  geno_face(&P, q, g, l, r);
  for (int k = 0; k < 3; ++k) { out[k] = l[k]; out[3 + k] = r[k]; }
  out[6] = l[3]; out[7] = r[3];
  return OR_OK;
}

/* Internals of GENO on one side, for the unit pins: dat = Q, G of cells
 * c-2..c+2 about the reconstructing cell (10 values), si = 0 left state,
 * 1 right state; qH, hqH the shared linear values. out = IS[3], p_k value[3],
 * h p_k'[3], omega[3], chi, q^L, h q^L', R, h R' (17 values). */
int oracle_geno_side_detail(const double *params, const double *dat, int si, double qH,
                            double hqH, double *out) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, 1, 1, 1, 1.0, 1.0, params);
  double xf = (si == 0) ? 0.5 : -0.5;
  double c[3][3], wt[3], wsum = 0.0;
  for (int k = 0; k < 3; ++k) {
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int m = 0; m < 10; ++m) s += SUB[si][k][q][m] * dat[m];
      c[k][q] = s;
    }
    out[k] = is_quadratic(c[k]);
    out[3 + k] = c[k][0] + c[k][1] * xf + c[k][2] * xf * xf;
    out[6 + k] = c[k][1] + 2.0 * c[k][2] * xf;
    wt[k] = P.d[k] / pow(out[k] + P.eps, P.rL);
    wsum += wt[k];
  }
  for (int k = 0; k < 3; ++k) out[9 + k] = wt[k] / wsum;
  double v, hd, h2, chi;
  geno_side(&P, dat, si, qH, hqH, 0.0, &v, &hd, &h2, &chi);
  out[12] = chi;
  out[13] = 0.0; out[14] = 0.0;
  for (int k = 0; k < 3; ++k) { out[13] += out[9 + k] * out[3 + k]; out[14] += out[9 + k] * out[6 + k]; }
  out[15] = v; out[16] = hd;
  return OR_OK;
}

/* Maxwellian moment table: out = mu[0..DU-1], mv[0..DV-1], mz[0..DZ-1]. */
int oracle_moments(double U, double V, double lam, double K, int half, int has_v, double *out) {
  mtab m; moments(U, V, lam, K, half, has_v, &m);
  memcpy(out, m.mu, sizeof m.mu);
  memcpy(out + DU, m.mv, sizeof m.mv);
  memcpy(out + DU + DV, m.mz, sizeof m.mz);
  return OR_OK;
}

/* GKS flux at npts points (face frame). ndim selects 1-D (3 vars, no
 * tangential data) or 2-D (4 vars). Arrays are [npts][nv]; sec is
 * [npts][3][nv]: physical second derivatives d_nn, d_nt, d_tt of the point
 * (1-D: d_nn only, the others ignored), or NULL for zero. Outputs F, dF/dt,
 * W(dt/2), W(dt) and the equilibrium W_tt. */
int oracle_gks_points(const double *params, int ndim, int npts, const double *Wl,
                      const double *Wr, const double *dnl, const double *dnr,
                      const double *dtl, const double *dtr, const double *sec, double dt,
                      double *F, double *Ft, double *Wh, double *Wf, double *Wtt) {
  if (ndim != 1 && ndim != 2) return OR_EINVAL;
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, 1, 1, 1.0, 1.0, params);
  int nv = P.nv;
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = 0; p < npts; ++p) {
    const double *s0 = sec ? sec + (size_t)p * 3 * nv : zero;
    const double *s1 = sec ? s0 + nv : zero, *s2 = sec ? s0 + 2 * nv : zero;
    gks_point(&P, Wl + p * nv, Wr + p * nv, dnl + p * nv, dnr + p * nv,
              ndim == 2 ? dtl + p * nv : NULL, ndim == 2 ? dtr + p * nv : NULL, s0, s1, s2, dt,
              F + p * nv, Ft + p * nv, Wh + p * nv, Wf + p * nv, Wtt + p * nv);
  }
  return OR_OK;
}

/* Normal GENO over all faces of direction dir (after filling ghost cells).
 * 1-D: faces f = 0..nx; 2-D x-faces: rows j = -1..ny (ny+2) x faces 0..nx;
 * y-faces: faces 0..ny x columns i = -1..nx (nx+2).
 * out: [side][quant(3)][var][rows][faces] (x) or [side][quant][var][faces][cols] (y),
 * quant = value, h d_n, h^2 d_nn;
 * chi: [side][var][...]. */
int oracle_normal_faces(const double *params, int ndim, int nx, int ny, double dx, double dy,
                        const double *W, const double *dW, int dir, double *out, double *chi) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  gstate g;
  if (gstate_alloc(&P, &g)) return OR_ENOMEM;
  gstate_load(&P, &g, W, dW);
  fill_ghosts(&P, &g);
  int nv = P.nv;
  int n0, n1;   /* outer (slow) and inner (fast) extents */
  if (ndim == 1) { n0 = 1; n1 = nx + 1; }
  else if (dir == 0) { n0 = ny + 2; n1 = nx + 1; }
  else { n0 = ny + 1; n1 = nx + 2; }
  size_t plane = (size_t)n0 * n1;
  for (int a = 0; a < n0; ++a)
    for (int b = 0; b < n1; ++b) {
      int i, j;
      if (ndim == 1) { i = NG + b - 1; j = 0; }
      else if (dir == 0) { i = NG + b - 1; j = NG + a - 1; }
      else { i = NG + b - 1; j = NG + a - 1; }
      double o[2][3][4], c[2][4];
      normal_face(&P, &g, ndim == 1 ? 0 : dir, i, j, o, c);
      for (int s = 0; s < 2; ++s)
        for (int v = 0; v < nv; ++v) {
          for (int q = 0; q < 3; ++q)
            out[(((size_t)s * 3 + q) * nv + v) * plane + (size_t)a * n1 + b] = o[s][q][v];
          chi[((size_t)s * nv + v) * plane + (size_t)a * n1 + b] = c[s][v];
        }
    }
  gstate_free(&g);
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* The paper's comparison of the nonlinear weights (Sec. 5): WENO-Z and     */
/* TENO weights on the same three sub-stencils, and the share of the linear */
/* reconstruction each keeps, chi = min_k w_k / d_k (for GENO: its path     */
/* function). d_k are the linear weights normalised to sum 1.               */
/* ---------------------------------------------------------------------- */
/* IS_k of the three sub-stencil quadratics of one side (as in geno_side). */
static void side_is(const double dat[10], int si, double IS[3]) {
  for (int k = 0; k < 3; ++k) {
    double c[3];
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int m = 0; m < 10; ++m) s += SUB[si][k][q][m] * dat[m];
      c[q] = s;
    }
    IS[k] = is_quadratic(c);
  }
}

/* WENO-Z: w~_k = d_k (1 + tau_Z / (IS_k + eps)), w = w~ / sum w~. tau_Z is
 * the difference of the two outer sub-stencils' indicators, |IS_1 - IS_3|
 * (reading: the paper leaves tau_Z to the stencil). Returns chi. */
static double wenoz_weights(const ocfg *P, const double IS[3], double w[3]) {
  double dsum = P->d[0] + P->d[1] + P->d[2], tz = fabs(IS[0] - IS[2]), ws = 0.0;
  for (int k = 0; k < 3; ++k) { w[k] = (P->d[k] / dsum) * (1.0 + tz / (IS[k] + P->eps)); ws += w[k]; }
  double chi = INFINITY;
  for (int k = 0; k < 3; ++k) {
    w[k] /= ws;
    double r = w[k] / (P->d[k] / dsum);
    if (r < chi) chi = r;
  }
  return chi;
}

/* TENO: scale separation gamma_k = (1/(IS_k + eps))^7 normalised; a
 * sub-stencil with gamma_k <= C_T is cut; w_k = delta_k d_k / sum delta d.
 * Returns chi (1 when no sub-stencil is cut, else 0). */
static double teno_weights(const ocfg *P, const double IS[3], double ct, double w[3]) {
  double g[3], gs = 0.0, ws = 0.0;
  for (int k = 0; k < 3; ++k) { g[k] = pow(1.0 / (IS[k] + P->eps), 7.0); gs += g[k]; }
  for (int k = 0; k < 3; ++k) { w[k] = (g[k] / gs > ct) ? P->d[k] : 0.0; ws += w[k]; }
  double chi = INFINITY;
  for (int k = 0; k < 3; ++k) {
    w[k] /= ws;
    double r = w[k] / (P->d[k] / (P->d[0] + P->d[1] + P->d[2]));
    if (r < chi) chi = r;
  }
  return chi;
}


/* Characteristic decomposition of the normal-direction flux Jacobian at the
 * Roe average of Wa and Wb (nv = 3 in 1-D, 4 in 2-D; dir 0 = x, 1 = y):
 * R (nv x nv, row-major, columns are right eigenvectors), L = R^-1 and the
 * speeds un - c, un, [un,] un + c. OR_EINVAL without a real sound speed. */
int oracle_roe_eigen(const double *params, int ndim, int dir, const double *Wa, const double *Wb,
                     double *R, double *L, double *lam) {
  ocfg P;
  cfg_from(&P, ndim, 1, 1, 1.0, 1.0, params);
  if (ndim == 1 && dir != 0) return OR_EINVAL;
  double Rm[4][4], Lm[4][4];
  if (roe_eigen(&P, dir, Wa, Wb, Rm, Lm)) return OR_EINVAL;
  const int nv = P.nv;
  for (int r = 0; r < nv; ++r)
    for (int k = 0; k < nv; ++k) { R[r * nv + k] = Rm[r][k]; L[r * nv + k] = Lm[r][k]; }
  /* speeds: each non-shear column has density entry 1, so its normal
   * momentum entry is its speed; the shear column moves with the entropy
   * column's speed un */
  const int in = 1 + dir;
  for (int k = 0; k < nv; ++k) lam[k] = Rm[in][(nv == 4 && k == 2) ? 1 : k];
  return OR_OK;
}

/* Weights of all three methods from given indicators IS[3]:
 * out = w_Z[3], chi_Z, w_T[3], chi_T, chi_GENO (IS^tau of the compact scheme). */
int oracle_weights(const double *params, const double *IS, double ct, double *out) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, 1, 1, 1, 1.0, 1.0, params);
  out[3] = wenoz_weights(&P, IS, out);
  out[7] = teno_weights(&P, IS, ct, out + 4);
  double ISH = IS[0], ISL = IS[0];
  for (int k = 1; k < 3; ++k) { if (IS[k] > ISH) ISH = IS[k]; if (IS[k] < ISL) ISL = IS[k]; }
  out[8] = path_function(&P, fabs((IS[1] + IS[2]) / 2.0 - IS[0]), ISH, ISL);
  return OR_OK;
}

/* chi of GENO, WENO-Z and TENO on every face-side of a direction (layout of
 * oracle_normal_faces' chi): out[method][side][var][...]. */
int oracle_linearity_faces(const double *params, int ndim, int nx, int ny, double dx, double dy,
                           const double *W, const double *dW, int dir, double ct, double *out) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  gstate g;
  if (gstate_alloc(&P, &g)) return OR_ENOMEM;
  gstate_load(&P, &g, W, dW);
  fill_ghosts(&P, &g);
  int nv = P.nv;
  int n0, n1;
  if (ndim == 1) { n0 = 1; n1 = nx + 1; }
  else if (dir == 0) { n0 = ny + 2; n1 = nx + 1; }
  else { n0 = ny + 1; n1 = nx + 2; }
  int d = ndim == 1 ? 0 : dir;
  size_t plane = (size_t)n0 * n1, mplane = 2 * (size_t)nv * plane;
  double h = (d == 0) ? P.dx : P.dy;
  for (int a = 0; a < n0; ++a)
    for (int b = 0; b < n1; ++b) {
      int i = NG + b - 1, j = ndim == 1 ? 0 : NG + a - 1;
      for (int v = 0; v < nv; ++v) {
        double q[4], gg[4];
        for (int m = -1; m <= 2; ++m) {
          int ii = (d == 0) ? i + m : i, jj = (d == 0) ? j : j + m;
          q[m + 1] = g.W[gidx(&g, v, jj, ii)];
          gg[m + 1] = h * g.dW[gidx(&g, d * nv + v, jj, ii)];
        }
        double dl[10] = {0}, dr[10] = {0};
        for (int m = 0; m < 4; ++m) {
          dl[2 * (m + 1)] = q[m]; dl[2 * (m + 1) + 1] = gg[m];
          dr[2 * m] = q[m]; dr[2 * m + 1] = gg[m];
        }
        for (int s = 0; s < 2; ++s) {
          double IS[3], w[9];
          side_is(s == 0 ? dl : dr, s, IS);
          oracle_weights(params, IS, ct, w);
          size_t o = ((size_t)s * nv + v) * plane + (size_t)a * n1 + b;
          out[0 * mplane + o] = w[8];
          out[1 * mplane + o] = w[3];
          out[2 * mplane + o] = w[7];
        }
      }
    }
  gstate_free(&g);
  return OR_OK;
}

/* Face states at the Gauss points after the tangential step and the
 * positivity guard (2-D), or at the face (1-D).
 * out (2-D): [side][gauss][quant][var][nfy][nfx], quant = value, h*d_n,
 * h*d_t, followed by the second derivatives of the points
 * [gauss][h_n^2 d_nn, h_n h_t d_nt, h_t^2 d_tt][var][nfy][nfx];
 * (1-D): [side][value, h*d_n][var][nf] followed by h^2 d_nn [var][nf].
 * Variables in the (x, y) frame. */
int oracle_face_states(const double *params, int ndim, int nx, int ny, double dx, double dy,
                       const double *W, const double *dW, int dir, double *out, long long *guard) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  gstate g;
  if (gstate_alloc(&P, &g)) return OR_ENOMEM;
  gstate_load(&P, &g, W, dW);
  fill_ghosts(&P, &g);
  int nv = P.nv;
  long long gcount = 0;
  if (ndim == 1) {
    size_t plane = (size_t)(nx + 1);
    for (int f = 0; f <= nx; ++f) {
      int i = NG + f - 1;
      double o[2][3][4], c[2][4];
      normal_face(&P, &g, 0, i, 0, o, c);
      int ok[2];
      for (int s = 0; s < 2; ++s) {
        double S[4];
        for (int v = 0; v < nv; ++v) S[v] = o[s][0][v];
        ok[s] = admissible(&P, S);
        if (!ok[s]) ++gcount;
        for (int v = 0; v < nv; ++v) {
          double val = ok[s] ? o[s][0][v] : g.W[gidx(&g, v, 0, i + s)];
          double dn = ok[s] ? o[s][1][v] : 0.0;
          out[(((size_t)s * 2 + 0) * nv + v) * plane + f] = val;
          out[(((size_t)s * 2 + 1) * nv + v) * plane + f] = dn;
        }
      }
      for (int v = 0; v < nv; ++v)
        out[((size_t)4 * nv + v) * plane + f] =
            (ok[0] && ok[1]) ? 0.5 * (o[0][2][v] + o[1][2][v]) : 0.0;
    }
  } else {
    int nfx = (dir == 0) ? nx + 1 : nx, nfy = (dir == 0) ? ny : ny + 1;
    size_t plane = (size_t)nfx * nfy;
    for (int a = 0; a < nfy; ++a)
      for (int b = 0; b < nfx; ++b) {
        int f = (dir == 0) ? b : a, t = (dir == 0) ? a : b;
        double o[3][2][3][4], c[2][4];
        for (int dt_ = -1; dt_ <= 1; ++dt_) {
          int i, j;
          if (dir == 0) { i = NG + f - 1; j = NG + t + dt_; }
          else { i = NG + t + dt_; j = NG + f - 1; }
          normal_face(&P, &g, dir, i, j, o[dt_ + 1], c);
        }
        int ci[2], cj[2];
        if (dir == 0) { ci[0] = NG + f - 1; ci[1] = NG + f; cj[0] = cj[1] = NG + t; }
        else { cj[0] = NG + f - 1; cj[1] = NG + f; ci[0] = ci[1] = NG + t; }
        for (int gp = 0; gp < 2; ++gp) {
          double S[2][4], Dn[2][4], Dt[2][4], Sec[3][4];
          gcount += face_point(&P, &g, o, gp, ci, cj, S, Dn, Dt, Sec);
          for (int s = 0; s < 2; ++s)
            for (int v = 0; v < nv; ++v) {
              size_t base = (((size_t)s * 2 + gp) * 3) * nv;
              out[(base + 0 * nv + v) * plane + (size_t)a * nfx + b] = S[s][v];
              out[(base + 1 * nv + v) * plane + (size_t)a * nfx + b] = Dn[s][v];
              out[(base + 2 * nv + v) * plane + (size_t)a * nfx + b] = Dt[s][v];
            }
          for (int q = 0; q < 3; ++q)
            for (int v = 0; v < nv; ++v) {
              size_t base = (size_t)12 * nv + ((size_t)gp * 3 + q) * nv;
              out[(base + v) * plane + (size_t)a * nfx + b] = Sec[q][v];
            }
        }
      }
  }
  if (guard) *guard = gcount;
  gstate_free(&g);
  return OR_OK;
}

/* nsteps full steps of the two-stage fourth-order method (S2O4) in place.
 * Cell averages (Eq. (1)), with L and its time derivative L_t from the
 * time-fitted interface fluxes:
 *   stage 1: W* = W + dt/2 L + dt^2/8 L_t,
 *   stage 2: W^{n+1} = W + dt L + dt^2/6 (L_t + 2 L_t*).
 * Cell-averaged gradients by the Gauss theorem (Eq. (2)) from the interface
 * values at the stage times. Reading (default): the same two-stage structure
 * applied to the interface values, whose time derivatives are those of the
 * BGK interface solution (through its states at dt/2 and dt, linear in t for
 * tau = 0) and the equilibrium second time derivative W_tt of each stage:
 *   W_face(t*) = W_int(dt/2) + dt^2/8 W_tt,
 *   W_face(t^{n+1}) = W_int(dt) + dt^2/6 (W_tt + 2 W_tt*).
 * Earlier reading (gupd = 1): the BGK interface state at dt/2 of each stage.
 * dt_hist: nsteps doubles (may be NULL). guard: positivity fall-backs.
 * fixed_dt > 0 overrides the CFL step. */
int oracle_step(const double *params, int ndim, int nx, int ny, double dx, double dy,
                double *W, double *dW, int nsteps, double fixed_dt, double *dt_hist,
                long long *guard) {
  if (oracle_init()) return OR_EINVAL;
  if (ndim != 1 && ndim != 2) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  int nv = P.nv;
  size_t ncell = (size_t)P.nx * P.ny;
  size_t nW = ncell * nv, nG = ncell * nv * ndim;
  double *L = malloc(nW * sizeof(double)), *Lt = malloc(nW * sizeof(double));
  double *Ws = malloc(nW * sizeof(double)), *Gs = malloc(nG * sizeof(double));
  double *R = malloc(nW * sizeof(double));
  gstate g; faceres fr;
  if (!L || !Lt || !Ws || !Gs || !R || gstate_alloc(&P, &g) || faceres_alloc(&P, &fr)) return OR_ENOMEM;
  /* interface values at the stage times, per direction */
  double *Wst[2] = {NULL, NULL}, *Wnx[2] = {NULL, NULL};
  for (int d = 0; d < ndim; ++d) {
    size_t n = (size_t)fr.nfx[d] * fr.nfy[d] * nv;
    Wst[d] = malloc(n * sizeof(double));
    Wnx[d] = malloc(n * sizeof(double));
    if (!Wst[d] || !Wnx[d]) return OR_ENOMEM;
  }
  for (int n = 0; n < nsteps; ++n) {
    double dt = fixed_dt > 0.0 ? fixed_dt : cfl_dt(&P, W);
    if (dt_hist) dt_hist[n] = dt;
    /* stage 1 */
    gstate_load(&P, &g, W, dW);
    fill_ghosts(&P, &g);
    stage_faces(&P, &g, dt, &fr);
    cell_terms(&P, &fr, L, Lt);
    for (size_t k = 0; k < nW; ++k) {
      Ws[k] = W[k] + 0.5 * dt * L[k] + dt * dt / 8.0 * Lt[k];
      R[k] = W[k] + dt * L[k] + dt * dt / 6.0 * Lt[k];
    }
    for (int d = 0; d < ndim; ++d) {
      size_t nf = (size_t)fr.nfx[d] * fr.nfy[d] * nv;
      for (size_t k = 0; k < nf; ++k) {
        if (P.gupd == 1) { Wst[d][k] = fr.Wh[d][k]; continue; }
        Wst[d][k] = fr.Wh[d][k] + dt * dt / 8.0 * fr.W2[d][k];
        Wnx[d][k] = fr.Wf[d][k] + dt * dt / 6.0 * fr.W2[d][k];
      }
    }
    gauss_gradient(&P, &fr, Wst, Gs);
    /* stage 2 */
    gstate_load(&P, &g, Ws, Gs);
    fill_ghosts(&P, &g);
    stage_faces(&P, &g, dt, &fr);
    cell_terms(&P, &fr, L, Lt);
    for (size_t k = 0; k < nW; ++k) W[k] = R[k] + dt * dt / 3.0 * Lt[k];
    for (int d = 0; d < ndim; ++d) {
      size_t nf = (size_t)fr.nfx[d] * fr.nfy[d] * nv;
      for (size_t k = 0; k < nf; ++k) {
        if (P.gupd == 1) Wnx[d][k] = fr.Wh[d][k];
        else Wnx[d][k] += dt * dt / 3.0 * fr.W2[d][k];
      }
    }
    gauss_gradient(&P, &fr, Wnx, dW);
  }
  if (guard) *guard = fr.guard;
  free(L); free(Lt); free(Ws); free(Gs); free(R);
  for (int d = 0; d < 2; ++d) { free(Wst[d]); free(Wnx[d]); }
  gstate_free(&g); faceres_free(&fr);
  return OR_OK;
}

/* One stage's face results (for unit parity of the flux over a grid) for
 * direction dir, each [nv][nfy][nfx]: F, dF/dt, W(dt/2), W(dt) and W_tt. */
int oracle_stage_faces(const double *params, int ndim, int nx, int ny, double dx, double dy,
                       const double *W, const double *dW, double dt, int dir,
                       double *F, double *Ft, double *Wh, double *Wf, double *Wtt) {
  if (oracle_init()) return OR_EINVAL;
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  gstate g; faceres fr;
  if (gstate_alloc(&P, &g) || faceres_alloc(&P, &fr)) return OR_ENOMEM;
  gstate_load(&P, &g, W, dW);
  fill_ghosts(&P, &g);
  stage_faces(&P, &g, dt, &fr);
  int d = (ndim == 1) ? 0 : dir;
  size_t n = (size_t)fr.nfx[d] * fr.nfy[d] * P.nv;
  memcpy(F, fr.F[d], n * sizeof(double));
  memcpy(Ft, fr.Ft[d], n * sizeof(double));
  memcpy(Wh, fr.Wh[d], n * sizeof(double));
  memcpy(Wf, fr.Wf[d], n * sizeof(double));
  memcpy(Wtt, fr.W2[d], n * sizeof(double));
  gstate_free(&g); faceres_free(&fr);
  return OR_OK;
}

/* CFL time step of a state (interior cells). */
double oracle_cfl_dt(const double *params, int ndim, int nx, int ny, double dx, double dy,
                     const double *W) {
  ocfg P; cfg_from(&P, ndim, nx, ny, dx, dy, params);
  return cfl_dt(&P, W);
}
