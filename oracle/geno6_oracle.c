/*
 * CPU FP64 oracle of the sixth-order non-compact finite-volume scheme with
 * GENO reconstruction in one dimension (Zhao & Xu, "A generalized ENO
 * reconstruction in compact GKS for compressible flow simulations", Sec. 4.1),
 * with the HLLC Riemann flux and the classical four-stage fourth-order
 * Runge-Kutta method named in Sec. 2.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library. It shares
 * no code, header, table or constant with the HIP library: every candidate
 * polynomial is obtained here, per call, by solving its cell-average system
 * by Gaussian elimination, and every smoothness indicator by integrating the
 * squared derivatives of that polynomial exactly.
 *
 * Paper passages followed:
 *   Sec. 3   Eq. (3)  blend R = chi q^H + (1 - chi) q^L
 *   Sec. 3.1 Eq. (4)  chi = tanh(C alpha) / tanh(C)
 *   Sec. 3.2 Eq. (5)  alpha from IS^tau, IS^H, IS^L with exponent r = 2
 *   Sec. 3.2 Eq. (6)  Jiang-Shu type indicators; Eq. (7) IS^H = Max{IS_k}
 *   Sec. 3.3 Eq. (8)  q^L = sum w_k p_k, w_k ~ d_k / (IS_k + eps)^2
 *            Eq. (9)  IS^L = Min{IS_k}
 *   Sec. 4.1          six-cell stencil S_0 and sub-stencils S_1..S_4,
 *                     R = chi p^5 + (1 - chi) sum w_k p_k, and
 *                     IS^tau = |(IS_1 + IS_3)/2 - IS_2|
 *   Sec. 2            HLLC flux and four-stage fourth-order Runge-Kutta
 * Readings where the paper defers to the literature or is silent:
 *   - p^5 and p_k are the polynomials whose cell averages over their stencil
 *     equal the data (degrees 5, 2, 2, 3, 3).
 *   - IS_k integrates over the target cell (cell j for the state left of
 *     x_{j+1/2}, cell j+1 for the state right of it) every derivative up to
 *     the polynomial's degree, scaled as in Eq. (6): sum_l h^(2l-1) *
 *     integral (d^l p / dx^l)^2 dx.
 *   - The right-side state mirrors every stencil about x_{j+1/2}.
 *   - The central sub-stencil boosted by C_0 = 8 in Eq. (8) is S_2 (the one
 *     centred on the target cell): d = (1, 8, 1, 1).
 *   - Variables are reconstructed component by component, either the
 *     conservative ones or (option) the characteristic ones: the stencil's
 *     states are projected on the left eigenvectors of the flux Jacobian at
 *     the Roe average of the two cells at the face, reconstructed, and
 *     mapped back with the right eigenvectors (a face whose Roe average has
 *     no real sound speed keeps the conservative variables).
 *   - A reconstructed state with rho <= 0, p <= 0 or a non-finite entry is
 *     replaced by the target cell's average (guard).
 *   - HLLC (Toro): wave speeds S_L = min(u_L - a_L, u_R - a_R),
 *     S_R = max(u_L + a_L, u_R + a_R); contact speed S* and star states of
 *     the standard HLLC solver.
 *   - dt = cfl dx / max over cells of (|u| + a), taken at the start of the
 *     step; classical Runge-Kutta stages with weights 1/6, 1/3, 1/3, 1/6.
 *   - Ghost cells: periodic images; transmissive = copy of the nearest
 *     interior cell; reflecting = mirror image with the momentum negated;
 *     fixed = given states (inflow or a fixed profile).
 *
 * Layout of every state array handed in: SoA [field][n], fields
 * (rho, rho U, rho E), interior cells only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define O6_OK 0
#define O6_EINVAL -1
#define O6_ENOMEM -2

enum { Q_GAMMA = 0, Q_C, Q_EPS, Q_D1, Q_D2, Q_D3, Q_D4, Q_CFL, Q_BCL, Q_BCH, Q_DTFIX, Q_CHAR,
       Q_GHOST,                /* 18 values: [end][ghost cell k][field] for fixed ends */
       Q_ISTAU = Q_GHOST + 18, /* 0: the printed IS^tau of Sec. 4.1, 1: the large-stencil one */
       Q_COUNT };

typedef struct {
  double gamma, C, eps, d[4], cfl, dt_fixed;
  int bc[2];   /* 0 periodic, 1 transmissive, 2 reflecting, 3 fixed states */
  int characteristic;   /* 0: conservative variables, 1: characteristic variables */
  int istau;            /* IS^tau: 0 printed (Sec. 4.1), 1 from p^5 (see geno_side) */
  double ghost[2][3][3];  /* fixed ends: [end][k][field], cell -1-k or n+k */
} cfg6;

static void cfg_load(cfg6 *c, const double *p) {
  c->gamma = p[Q_GAMMA]; c->C = p[Q_C]; c->eps = p[Q_EPS];
  for (int k = 0; k < 4; ++k) c->d[k] = p[Q_D1 + k];
  c->cfl = p[Q_CFL]; c->bc[0] = (int)p[Q_BCL]; c->bc[1] = (int)p[Q_BCH];
  c->dt_fixed = p[Q_DTFIX];
  c->characteristic = (int)p[Q_CHAR];
  c->istau = (int)p[Q_ISTAU];
  for (int e = 0; e < 2; ++e)
    for (int k = 0; k < 3; ++k)
      for (int f = 0; f < 3; ++f) c->ghost[e][k][f] = p[Q_GHOST + (e * 3 + k) * 3 + f];
}

/* ---------------------------------------------------------------------- */
/* Candidate polynomials from cell averages                                */
/* ---------------------------------------------------------------------- */
/* Local coordinate xi = (x - x_j) / h: the target cell is [-1/2, 1/2] and
 * cell j+m is [m - 1/2, m + 1/2]. p(xi) = sum_k a[k] xi^k. */

/* Dense Gaussian elimination with partial pivoting; A is n x n row-major. */
static int gauss_solve(int n, double *A, double *b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return O6_EINVAL;
    if (piv != c) {
      for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
      double t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
    b[r] = s / A[r * n + r];
  }
  return O6_OK;
}

/* Polynomial of degree n-1 whose averages over cells lo, lo+1, ..., lo+n-1
 * (offsets from the target cell) are avg[0..n-1]. */
static int poly_from_averages(const double *avg, int lo, int n, double *a) {
  double A[36], b[6];
  for (int m = 0; m < n; ++m) {
    double xl = lo + m - 0.5, xr = lo + m + 0.5;
    for (int k = 0; k < n; ++k)
      A[m * n + k] = (pow(xr, k + 1) - pow(xl, k + 1)) / (k + 1);  /* average of xi^k over the cell */
    b[m] = avg[m];
  }
  if (gauss_solve(n, A, b)) return O6_EINVAL;
  for (int k = 0; k < n; ++k) a[k] = b[k];
  return O6_OK;
}

static double poly_eval(const double *a, int n, double xi) {
  double s = 0.0;
  for (int k = n - 1; k >= 0; --k) s = s * xi + a[k];
  return s;
}

/* Eq. (6) on the target cell: sum over l = 1..lmax of the integral over
 * [-1/2, 1/2] of (d^l p / d xi^l)^2 (the powers of h cancel). The derivative
 * polynomial is squared term by term and integrated exactly. */
static double smoothness(const double *a, int n, int lmax) {
  double s = 0.0;
  for (int l = 1; l <= lmax; ++l) {
    double c[6] = {0, 0, 0, 0, 0, 0};   /* coefficients of the l-th derivative */
    for (int k = l; k < n; ++k) {
      double f = 1.0;
      for (int q = 0; q < l; ++q) f *= (double)(k - q);
      c[k - l] = f * a[k];
    }
    for (int i = 0; i < n - l; ++i)
      for (int k = 0; k < n - l; ++k) {
        int e = i + k;
        if (e % 2) continue;   /* odd powers integrate to zero on [-1/2, 1/2] */
        s += c[i] * c[k] * 2.0 * pow(0.5, e + 1) / (e + 1);
      }
  }
  return s;
}

/* ---------------------------------------------------------------------- */
/* GENO side state (Sec. 4.1)                                              */
/* ---------------------------------------------------------------------- */
/* u6 holds the averages of cells j-2..j+3 around the face x_{j+1/2}.
 * side 0: the state left of the face (target cell j, xi = +1/2);
 * side 1: the state right of it (target cell j+1, xi = -1/2, stencils
 * mirrored). detail (may be NULL) receives 16 numbers:
 *   [0] value, [1] chi, [2] alpha, [3] p^5 value, [4..7] IS_1..IS_4,
 *   [8..11] w_1..w_4, [12..15] p_1..p_4 values at the face. */
static int geno_side(const cfg6 *P, const double u6[6], int side, double *detail) {
  /* stencils as offsets from the target cell, for the left side */
  static const int LO[5] = {-2, -2, -1, -1, 0};   /* S_0, S_1, S_2, S_3, S_4 */
  static const int NC[5] = {6, 3, 3, 4, 4};
  const int tgt = side == 0 ? 2 : 3;               /* index of the target cell in u6 */
  const double xi = side == 0 ? 0.5 : -0.5;
  double val[5], IS[5];
  for (int s = 0; s < 5; ++s) {
    int lo = side == 0 ? LO[s] : -(LO[s] + NC[s] - 1);   /* mirror about the face */
    double avg[6], a[6];
    for (int m = 0; m < NC[s]; ++m) avg[m] = u6[tgt + lo + m];
    if (poly_from_averages(avg, lo, NC[s], a)) return O6_EINVAL;
    val[s] = poly_eval(a, NC[s], xi);
    IS[s] = s == 0 ? 0.0 : smoothness(a, NC[s], NC[s] - 1);
  }
  /* Eq. (7), (9) and the Sec. 4.1 indicator */
  double ISH = IS[1], ISL = IS[1];
  for (int k = 2; k <= 4; ++k) { ISH = fmax(ISH, IS[k]); ISL = fmin(ISL, IS[k]); }
  /* Sec. 4.1 prints IS^tau = |(IS_1 + IS_3)/2 - IS_2|, blind to a jump that
   * lies only in S_4 (the cells j..j+3 on the left side). Option istau = 1
   * takes instead, as Sec. 3 describes IS^tau (a higher-order indicator of
   * the large stencil) and Sec. 4.3 builds it on triangles, the difference
   * between the indicator of p^5 up to its fifth derivative and up to its
   * fourth, i.e. the integral of (d^5 p^5 / dxi^5)^2 over the target cell. */
  double IStau = fabs(0.5 * (IS[1] + IS[3]) - IS[2]);
  if (P->istau == 1) {
    const int lo0 = side == 0 ? LO[0] : -(LO[0] + NC[0] - 1);
    double avg[6], a[6];
    for (int m = 0; m < 6; ++m) avg[m] = u6[tgt + lo0 + m];
    if (poly_from_averages(avg, lo0, 6, a)) return O6_EINVAL;
    IStau = fabs(smoothness(a, 6, 5) - smoothness(a, 6, 4));
  }
  /* Eq. (5) with r = 2 and Eq. (4) */
  const double aH = 1.0 + pow(IStau / (ISH + P->eps), 2.0);
  const double aL = 1.0 + pow(IStau / (ISL + P->eps), 2.0);
  const double alpha = 2.0 * aH / (aH + aL);
  const double chi = tanh(P->C * alpha) / tanh(P->C);
  /* Eq. (8) with r^L = 2 */
  double wt[4], sw = 0.0;
  for (int k = 0; k < 4; ++k) { wt[k] = P->d[k] / pow(IS[k + 1] + P->eps, 2.0); sw += wt[k]; }
  double qL = 0.0;
  for (int k = 0; k < 4; ++k) { wt[k] /= sw; qL += wt[k] * val[k + 1]; }
  const double v = chi * val[0] + (1.0 - chi) * qL;
  if (detail) {
    detail[0] = v; detail[1] = chi; detail[2] = alpha; detail[3] = val[0];
    for (int k = 0; k < 4; ++k) {
      detail[4 + k] = IS[k + 1]; detail[8 + k] = wt[k]; detail[12 + k] = val[k + 1];
    }
  }
  return O6_OK;
}

/* ---------------------------------------------------------------------- */
/* Euler flux and HLLC (Toro's HLLC solver, reading of Sec. 2)             */
/* ---------------------------------------------------------------------- */
static double pressure(const cfg6 *P, const double *U) {
  return (P->gamma - 1.0) * (U[2] - 0.5 * U[1] * U[1] / U[0]);
}

static void euler_flux(const cfg6 *P, const double *U, double *F) {
  double u = U[1] / U[0], p = pressure(P, U);
  F[0] = U[1];
  F[1] = U[1] * u + p;
  F[2] = (U[2] + p) * u;
}

static void hllc(const cfg6 *P, const double *UL, const double *UR, double *F) {
  const double rl = UL[0], ul = UL[1] / rl, pl = pressure(P, UL), al = sqrt(P->gamma * pl / rl);
  const double rr = UR[0], ur = UR[1] / rr, pr = pressure(P, UR), ar = sqrt(P->gamma * pr / rr);
  const double SL = fmin(ul - al, ur - ar), SR = fmax(ul + al, ur + ar);
  double FL[3], FR[3];
  if (SL >= 0.0) { euler_flux(P, UL, F); return; }
  if (SR <= 0.0) { euler_flux(P, UR, F); return; }
  const double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur));
  if (Ss >= 0.0) {
    euler_flux(P, UL, FL);
    const double f = rl * (SL - ul) / (SL - Ss);
    const double Us[3] = {f, f * Ss, f * (UL[2] / rl + (Ss - ul) * (Ss + pl / (rl * (SL - ul))))};
    for (int v = 0; v < 3; ++v) F[v] = FL[v] + SL * (Us[v] - UL[v]);
  } else {
    euler_flux(P, UR, FR);
    const double f = rr * (SR - ur) / (SR - Ss);
    const double Us[3] = {f, f * Ss, f * (UR[2] / rr + (Ss - ur) * (Ss + pr / (rr * (SR - ur))))};
    for (int v = 0; v < 3; ++v) F[v] = FR[v] + SR * (Us[v] - UR[v]);
  }
}

static int admissible(const cfg6 *P, const double *U) {
  for (int v = 0; v < 3; ++v) if (!isfinite(U[v])) return 0;
  return U[0] > 0.0 && pressure(P, U) > 0.0;
}

/* ---------------------------------------------------------------------- */
/* Characteristic variables (reading: Roe average of the two cells at the  */
/* face, right eigenvectors of the Euler flux Jacobian there; the left     */
/* ones are their inverse, obtained here by Gaussian elimination)          */
/* ---------------------------------------------------------------------- */
/* Roe average of Ua, Ub: (u, H, c); right eigenvectors R (columns for the
 * speeds u - c, u, u + c, row-major R[row * 3 + col]) and L = R^-1. */
static int eigen(const cfg6 *P, const double *Ua, const double *Ub, double *R, double *L,
                 double *lam) {
  const double sa = sqrt(Ua[0]), sb = sqrt(Ub[0]);
  const double ua = Ua[1] / Ua[0], ub = Ub[1] / Ub[0];
  const double Ha = (Ua[2] + pressure(P, Ua)) / Ua[0], Hb = (Ub[2] + pressure(P, Ub)) / Ub[0];
  const double u = (sa * ua + sb * ub) / (sa + sb), H = (sa * Ha + sb * Hb) / (sa + sb);
  const double c2 = (P->gamma - 1.0) * (H - 0.5 * u * u);
  if (!(c2 > 0.0)) return O6_EINVAL;
  const double c = sqrt(c2);
  const double Rm[9] = {1.0, 1.0, 1.0,
                        u - c, u, u + c,
                        H - u * c, 0.5 * u * u, H + u * c};
  for (int i = 0; i < 9; ++i) R[i] = Rm[i];
  for (int col = 0; col < 3; ++col) {     /* L = R^-1, column by column */
    double A[9], b[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 9; ++i) A[i] = Rm[i];
    b[col] = 1.0;
    if (gauss_solve(3, A, b)) return O6_EINVAL;
    for (int r = 0; r < 3; ++r) L[r * 3 + col] = b[r];
  }
  if (lam) { lam[0] = u - c; lam[1] = u; lam[2] = u + c; }
  return O6_OK;
}

/* ---------------------------------------------------------------------- */
/* Ghost cells and face states                                             */
/* ---------------------------------------------------------------------- */
/* Value of field f at cell index i in [-3, n+3) from the interior array. */
static double cell(const cfg6 *P, const double *U, int n, int f, int i) {
  if (i >= 0 && i < n) return U[(size_t)f * n + i];
  const int lo = i < 0, bc = P->bc[lo ? 0 : 1];
  if (bc == 3) return P->ghost[lo ? 0 : 1][lo ? -i - 1 : i - n][f];
  if (bc == 0) return U[(size_t)f * n + (lo ? i + n : i - n)];
  if (bc == 1) return U[(size_t)f * n + (lo ? 0 : n - 1)];
  const int src = lo ? -i - 1 : 2 * n - 1 - i;
  return (f == 1 ? -1.0 : 1.0) * U[(size_t)f * n + src];
}

/* Face s in [0, n] lies between cells s-1 and s. Writes the two guarded
 * states, the HLLC flux and the path functions; returns the number of guard
 * replacements (0..2) or a negative error. */
static int face(const cfg6 *P, const double *U, int n, int s, double UL[3], double UR[3],
                double F[3], double chi[6]) {
  int guard = 0;
  double st[6][3];   /* the stencil's conservative states, cells s-3..s+2 */
  for (int m = 0; m < 6; ++m)
    for (int v = 0; v < 3; ++v) st[m][v] = cell(P, U, n, v, s - 3 + m);
  double R[9], L[9];
  /* a face whose Roe average has no real sound speed (non-physical cells)
     falls back to the conservative variables */
  const int ch = P->characteristic && eigen(P, st[2], st[3], R, L, NULL) == O6_OK;
  double wl[3], wr[3];
  for (int v = 0; v < 3; ++v) {
    double u6[6], det[16];
    for (int m = 0; m < 6; ++m)
      u6[m] = ch ? L[v * 3 + 0] * st[m][0] + L[v * 3 + 1] * st[m][1] + L[v * 3 + 2] * st[m][2]
                 : st[m][v];
    if (geno_side(P, u6, 0, det)) return O6_EINVAL;
    wl[v] = det[0]; if (chi) chi[v] = det[1];
    if (geno_side(P, u6, 1, det)) return O6_EINVAL;
    wr[v] = det[0]; if (chi) chi[3 + v] = det[1];
  }
  for (int v = 0; v < 3; ++v) {
    if (ch) {
      UL[v] = R[v * 3 + 0] * wl[0] + R[v * 3 + 1] * wl[1] + R[v * 3 + 2] * wl[2];
      UR[v] = R[v * 3 + 0] * wr[0] + R[v * 3 + 1] * wr[1] + R[v * 3 + 2] * wr[2];
    } else {
      UL[v] = wl[v];
      UR[v] = wr[v];
    }
  }
  if (!admissible(P, UL)) { for (int v = 0; v < 3; ++v) UL[v] = cell(P, U, n, v, s - 1); ++guard; }
  if (!admissible(P, UR)) { for (int v = 0; v < 3; ++v) UR[v] = cell(P, U, n, v, s); ++guard; }
  hllc(P, UL, UR, F);
  return guard;
}

/* L = -(F_{j+1/2} - F_{j-1/2}) / dx for every interior cell. */
static long long rhs(const cfg6 *P, const double *U, int n, double dx, double *L, double *Fbuf) {
  long long guard = 0;
  int bad = 0;
#pragma omp parallel for reduction(+ : guard) reduction(| : bad) schedule(static)
  for (int s = 0; s <= n; ++s) {
    double UL[3], UR[3], F[3];
    int g = face(P, U, n, s, UL, UR, F, NULL);
    if (g < 0) { bad = 1; continue; }
    guard += g;
    for (int v = 0; v < 3; ++v) Fbuf[(size_t)v * (n + 1) + s] = F[v];
  }
  if (bad) return -1;
  for (int v = 0; v < 3; ++v)
    for (int j = 0; j < n; ++j)
      L[(size_t)v * n + j] = -(Fbuf[(size_t)v * (n + 1) + j + 1] - Fbuf[(size_t)v * (n + 1) + j]) / dx;
  return guard;
}

static double cfl_dt(const cfg6 *P, const double *U, int n, double dx) {
  double smax = 0.0;
  for (int j = 0; j < n; ++j) {
    double W[3] = {U[j], U[(size_t)n + j], U[2 * (size_t)n + j]};
    double u = W[1] / W[0], a = sqrt(P->gamma * pressure(P, W) / W[0]);
    smax = fmax(smax, fabs(u) + a);
  }
  return P->cfl * dx / smax;
}

/* ---------------------------------------------------------------------- */
/* Exported entry points                                                   */
/* ---------------------------------------------------------------------- */
int o6_nparams(void) { return Q_COUNT; }

int o6_poly(const double *avg, int lo, int n, double *a) {
  if (n < 1 || n > 6) return O6_EINVAL;
  return poly_from_averages(avg, lo, n, a);
}

double o6_smoothness(const double *a, int n, int lmax) { return smoothness(a, n, lmax); }

int o6_side(const double *params, const double *u6, int side, double *detail) {
  cfg6 P; cfg_load(&P, params);
  return geno_side(&P, u6, side, detail);
}

/* Roe-averaged eigen-structure of the face between states Ua and Ub. */
int o6_eigen(const double *params, const double *Ua, const double *Ub, double *R, double *L,
             double *lam) {
  cfg6 P; cfg_load(&P, params);
  return eigen(&P, Ua, Ub, R, L, lam);
}

int o6_hllc(const double *params, const double *UL, const double *UR, double *F) {
  cfg6 P; cfg_load(&P, params);
  hllc(&P, UL, UR, F);
  return O6_OK;
}

/* Every face s = 0..n: UL, UR, F as [var][n+1]; chi as [side][var][n+1]
 * (NULL allowed). Returns the guard count or a negative error. */
long long o6_faces(const double *params, int n, const double *U, double *UL, double *UR,
                   double *F, double *chi) {
  cfg6 P; cfg_load(&P, params);
  if (n < 3) return O6_EINVAL;
  long long guard = 0;
  for (int s = 0; s <= n; ++s) {
    double l[3], r[3], f[3], c[6];
    int g = face(&P, U, n, s, l, r, f, c);
    if (g < 0) return g;
    guard += g;
    for (int v = 0; v < 3; ++v) {
      UL[(size_t)v * (n + 1) + s] = l[v];
      UR[(size_t)v * (n + 1) + s] = r[v];
      F[(size_t)v * (n + 1) + s] = f[v];
      if (chi) {
        chi[(size_t)v * (n + 1) + s] = c[v];
        chi[(size_t)(3 + v) * (n + 1) + s] = c[3 + v];
      }
    }
  }
  return guard;
}

long long o6_rhs(const double *params, int n, double dx, const double *U, double *L) {
  cfg6 P; cfg_load(&P, params);
  if (n < 3) return O6_EINVAL;
  double *Fb = malloc(sizeof(double) * 3 * (size_t)(n + 1));
  if (!Fb) return O6_ENOMEM;
  long long g = rhs(&P, U, n, dx, L, Fb);
  free(Fb);
  return g;
}

double o6_cfl_dt(const double *params, int n, double dx, const double *U) {
  cfg6 P; cfg_load(&P, params);
  return cfl_dt(&P, U, n, dx);
}

/* nsteps classical Runge-Kutta steps of U in place; dt from the CFL
 * condition at the start of each step unless dt_fixed > 0; dt_out (may be
 * NULL) receives each step's dt. Returns the guard count or a negative
 * error. */
long long o6_step(const double *params, int n, double dx, double *U, int nsteps, double *dt_out) {
  cfg6 P; cfg_load(&P, params);
  if (n < 3 || nsteps < 0) return O6_EINVAL;
  const size_t N = 3 * (size_t)n;
  double *k = malloc(sizeof(double) * N * 4), *Y = malloc(sizeof(double) * N),
         *Fb = malloc(sizeof(double) * 3 * (size_t)(n + 1));
  if (!k || !Y || !Fb) { free(k); free(Y); free(Fb); return O6_ENOMEM; }
  long long guard = 0;
  static const double C_IN[4] = {0.0, 0.5, 0.5, 1.0};      /* stage abscissae */
  static const double B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  for (int st = 0; st < nsteps; ++st) {
    const double dt = P.dt_fixed > 0.0 ? P.dt_fixed : cfl_dt(&P, U, n, dx);
    if (dt_out) dt_out[st] = dt;
    for (int s = 0; s < 4; ++s) {
      for (size_t q = 0; q < N; ++q) Y[q] = s == 0 ? U[q] : U[q] + C_IN[s] * dt * k[(size_t)(s - 1) * N + q];
      long long g = rhs(&P, Y, n, dx, k + (size_t)s * N, Fb);
      if (g < 0) { free(k); free(Y); free(Fb); return O6_EINVAL; }
      guard += g;
    }
    for (size_t q = 0; q < N; ++q)
      U[q] = U[q] + dt * (B[0] * k[q] + B[1] * k[N + q] + B[2] * k[2 * N + q] + B[3] * k[3 * N + q]);
  }
  free(k); free(Y); free(Fb);
  return guard;
}
