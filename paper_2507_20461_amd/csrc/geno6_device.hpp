// Device functions of the sixth-order non-compact scheme (Sec. 4.1): GENO
// side states on the six-cell stencil, the positivity guard and the HLLC
// flux. Templated on the scalar type D so that the same code runs on the
// device (double) and on the host with a counting type (operation counts).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace geno6 {

struct KP6 {
  double gamma;
  double C;          // path-function steepness (Eq. (4))
  double inv_tanhC;  // 1 / tanh(C)
  double t2_cut;     // 2 (1 - A) / A, A = 19.8 / C: alpha >= A when (IS^tau / y)^2 is below it
  double eps;        // indicator floor (Eq. (5), (8))
  double d[4];       // linear weights of S_1..S_4 (Eq. (8))
  double cfl;
  double dt_fixed;
  int characteristic;   // reconstruct characteristic fields (0 or 1)
};

// Candidate values at the face and indicators of both states at the face
// x_{j+1/2}; u[0..5] are the averages of cells j-2..j+3. The coefficients
// follow from the cell-average conditions of each candidate in
// xi = (x - x_t)/h about its target cell t (j for the left state, j+1 for
// the right one, whose stencils are the mirror images about the face):
//   S_1 {j-2, j-1, j}   face value (2 u0 - 7 u1 + 11 u2) / 6
//   S_2 {j-1, j, j+1}   face value (-u1 + 5 u2 + 2 u3) / 6
//   S_3 {j-1..j+2}      face value (-u1 + 7 u2 + 7 u3 - u4) / 12
//   S_4 {j..j+3}        face value (3 u2 + 13 u3 - 5 u4 + u5) / 12
// and Eq. (6) on the target cell, with p = sum a_k xi^k:
//   quadratic: IS = a1^2 + 13/3 a2^2
//   cubic:     IS = (a1 + a3/4)^2 + 13/3 a2^2 + 781/20 a3^2
// (the integrals over [-1/2, 1/2] of the squared first, second and third
// derivatives, completed to squares). Everything is written in the first
// differences d_i = u_i - u_{i-1} (i = 1..5) and the second differences
// D_a = d_2 - d_1, D_b = d_3 - d_2, D_c = d_4 - d_3, D_d = d_5 - d_4, which
// the two states share. Left state (2 a1 and 2 a2 of S_1, S_2; 6 (a1 +
// a3/4), 2 a2, 6 a3 of S_3, S_4):
//   S_1: D_a + 2 d_2, D_a;   S_2: -(d_2 + d_3), D_b
//   S_3: 2 d_2 + 5 d_3 - d_4, D_b, D_c - D_b
//   S_4: 11 d_3 - 7 d_4 + 2 d_5, 2 D_c - D_d, D_d - D_c
// face values u2 + (5 d_2 - 2 d_1)/6, u2 + (d_2 + 2 d_3)/6,
// p_3 = (7 (u2 + u3) - u1 - u4)/12, u3 + (d_5 - 3 d_3 - 4 d_4)/12.
// The right state is the same with d_i -> -d_{6-i} and D_a <-> D_d,
// D_b <-> D_c (signs inside squares dropped):
//   S_1: D_d - 2 d_4, D_d;   S_2: d_3 + d_4, D_c
//   S_3: 2 d_4 + 5 d_3 - d_2, D_c, D_b - D_c (the square of S_3's a3 is
//        the left state's)
//   S_4: 11 d_3 - 7 d_2 + 2 d_1, 2 D_b - D_a, D_a - D_b
// face values u3 + (2 d_5 - 5 d_4)/6, u3 - (d_4 + 2 d_3)/6, p_3,
// u2 + (3 d_3 + 4 d_2 - d_1)/12.
template <typename D>
struct Cand {
  D v1, v2, v4;        // face values of p_1, p_2, p_4 (p_3 is shared by both sides)
  D IS[4];
};

template <typename D>
__host__ __device__ __forceinline__ void candidates(const D (&u)[6], Cand<D>& L, Cand<D>& R, D& p5,
                                                   D& p3) {
  const D sixth = D(1.0 / 6.0), twelfth = D(1.0 / 12.0);
  const D k13 = D(13.0 / 12.0), k36 = D(1.0 / 36.0), k781 = D(781.0 / 720.0), q = D(0.25);
  const D d1 = u[1] - u[0], d2 = u[2] - u[1], d3 = u[3] - u[2], d4 = u[4] - u[3], d5 = u[5] - u[4];
  const D Da = d2 - d1, Db = d3 - d2, Dc = d4 - d3, Dd = d5 - d4;
  p5 = (u[0] + u[5] - D(8.0) * (u[1] + u[4]) + D(37.0) * (u[2] + u[3])) * D(1.0 / 60.0);
  p3 = (D(7.0) * (u[2] + u[3]) - u[1] - u[4]) * twelfth;
  // 13/3 a2^2 terms of the four second differences and the shared a3 term of S_3
  const D Ka = k13 * Da * Da, Kb = k13 * Db * Db, Kc = k13 * Dc * Dc, Kd = k13 * Dd * Dd;
  const D c3 = Dc - Db;
  const D P3 = k781 * c3 * c3;
  // left state
  L.v1 = u[2] + (D(5.0) * d2 - D(2.0) * d1) * sixth;
  L.v2 = u[2] + (d2 + D(2.0) * d3) * sixth;
  L.v4 = u[3] + (d5 - D(3.0) * d3 - D(4.0) * d4) * twelfth;
  const D l1 = Da + D(2.0) * d2, l2 = d2 + d3;
  const D l3 = D(2.0) * d2 + D(5.0) * d3 - d4;
  const D l4a = D(11.0) * d3 - D(7.0) * d4 + D(2.0) * d5, l4b = D(2.0) * Dc - Dd, l4c = Dd - Dc;
  L.IS[0] = Ka + q * l1 * l1;
  L.IS[1] = Kb + q * l2 * l2;
  L.IS[2] = Kb + P3 + k36 * l3 * l3;
  L.IS[3] = k36 * l4a * l4a + k13 * l4b * l4b + k781 * l4c * l4c;
  // right state
  R.v1 = u[3] + (D(2.0) * d5 - D(5.0) * d4) * sixth;
  R.v2 = u[3] - (d4 + D(2.0) * d3) * sixth;
  R.v4 = u[2] + (D(3.0) * d3 + D(4.0) * d2 - d1) * twelfth;
  const D r1 = Dd - D(2.0) * d4, r2 = d3 + d4;
  const D r3 = D(2.0) * d4 + D(5.0) * d3 - d2;
  const D r4a = D(11.0) * d3 - D(7.0) * d2 + D(2.0) * d1, r4b = D(2.0) * Db - Da, r4c = Da - Db;
  R.IS[0] = Kd + q * r1 * r1;
  R.IS[1] = Kc + q * r2 * r2;
  R.IS[2] = Kc + P3 + k36 * r3 * r3;
  R.IS[3] = k36 * r4a * r4a + k13 * r4b * r4b + k781 * r4c * r4c;
}

// Path function (Eq. (4), (5) with r = 2, Eq. (7), (9) and the Sec. 4.1
// IS^tau). alpha = 2 aH / (aH + aL), aH = 1 + t^2/x^2, aL = 1 + t^2/y^2
// (x = IS^H + eps, y = IS^L + eps) is the fraction num / den with
// num = 2 y^2 (x^2 + t^2), den = 2 x^2 y^2 + t^2 (x^2 + y^2). tanh(z) for
// z >= 0 is (1 - e)/(1 + e), e = exp(-2z); for z = C alpha >= 19.8,
// e < 2^-54 and both tanh(z) and tanh(C) (C >= z) round to 1, so chi is 1
// exactly: that case is recognised without the division, as
// C num >= 19.8 den (near the threshold both branches give 1).
template <typename D>
__host__ __device__ __forceinline__ D path_chi6(const D (&IS)[4], const KP6& k) {
  using std::fabs;
  using std::fmax;
  using std::fmin;
  const D ISH = fmax(fmax(IS[0], IS[1]), fmax(IS[2], IS[3]));
  const D ISL = fmin(fmin(IS[0], IS[1]), fmin(IS[2], IS[3]));
  const D t = fabs(D(0.5) * (IS[0] + IS[2]) - IS[1]);
  const D x = ISH + D(k.eps), y = ISL + D(k.eps);
  const D x2 = x * x, y2 = y * y, t2 = t * t;
  // alpha >= A = 19.8 / C already holds when t^2 / y^2 <= 2 (1 - A) / A
  // (then 2 (1 + t^2/x^2) >= A (2 + t^2/x^2 + t^2/y^2) for any x >= y): a
  // cheaper sufficient test with the same outcome, chi = 1
  if (t2 <= D(k.t2_cut) * y2) return D(1.0);
  const D num = D(2.0) * y2 * (x2 + t2);
  const D den = D(2.0) * x2 * y2 + t2 * (x2 + y2);
  if (!(D(k.C) * num < D(19.8) * den)) return D(1.0);
  using std::exp;
  const D z = D(k.C) * (num / den);
  const D e = exp(D(-2.0) * z);
  return (D(1.0) - e) / (D(1.0) + e) * D(k.inv_tanhC);
}

// Eq. (8) with r^L = 2: q^L = sum_k d_k v_k / a_k / sum_k d_k / a_k,
// a_k = (IS_k + eps)^2, formed with one division by multiplying through by
// a_1 a_2 a_3 a_4.
template <typename D>
__host__ __device__ __forceinline__ D low_order6(const D (&IS)[4], D v1, D v2, D v3, D v4,
                                                 const KP6& k) {
  const D e = D(k.eps);
  const D a1 = (IS[0] + e) * (IS[0] + e), a2 = (IS[1] + e) * (IS[1] + e);
  const D a3 = (IS[2] + e) * (IS[2] + e), a4 = (IS[3] + e) * (IS[3] + e);
  const D a12 = a1 * a2, a34 = a3 * a4;
  const D w1 = D(k.d[0]) * (a2 * a34), w2 = D(k.d[1]) * (a1 * a34);
  const D w3 = D(k.d[2]) * (a12 * a4), w4 = D(k.d[3]) * (a12 * a3);
  return (w1 * v1 + w2 * v2 + w3 * v3 + w4 * v4) / (w1 + w2 + w3 + w4);
}

// GENO state of one side: c from candidates() on the side's stencil, p5 and
// p3 the face values of the quintic and of the S_3 cubic (the same
// polynomials for both sides). chi_out receives the path function.
template <typename D>
__host__ __device__ __forceinline__ D side6(const Cand<D>& c, D p5, D p3, const KP6& k,
                                           D& chi_out) {
  const D chi = path_chi6(c.IS, k);
  chi_out = chi;
  if (chi == D(1.0)) return p5;
  const D qL = low_order6(c.IS, c.v1, c.v2, p3, c.v4, k);
  return chi * p5 + (D(1.0) - chi) * qL;
}

// rho > 0 and p > 0 (as rho E - m^2/2 > 0, rho > 0) with finite entries.
template <typename D>
__host__ __device__ __forceinline__ bool admissible6(const D* W) {
  using std::isfinite;
  return isfinite(W[0]) && isfinite(W[1]) && isfinite(W[2]) && W[0] > D(0.0) &&
         W[0] * W[2] - D(0.5) * W[1] * W[1] > D(0.0);
}

// HLLC flux (Toro's solver) with S_L = min(u_L - a_L, u_R - a_R),
// S_R = max(u_L + a_L, u_R + a_R), contact speed
// S* = (p_R - p_L + m_L (S_L - u_L) - m_R (S_R - u_R)) /
//      (rho_L (S_L - u_L) - rho_R (S_R - u_R)),
// star state of side K: f (1, S*, E_K/rho_K + (S* - u_K)(S* + p_K /
// (rho_K (S_K - u_K)))), f = rho_K (S_K - u_K)/(S_K - S*),
// F = F_K + S_K (U*_K - U_K) with K = L for S* >= 0, else R; F_L for
// S_L >= 0, F_R for S_R <= 0. The star side is chosen by selects, so a
// wave takes no branch. Three divisions: 1/(rho_L rho_R) gives both
// reciprocal densities, one for S*, and q = 1/((S_K - u_K)(S_K - S*))
// gives f = rho_K (S_K - u_K)^2 q and p_K/(rho_K (S_K - u_K)) =
// p_K (S_K - S*) q / rho_K.
template <typename D>
__host__ __device__ __forceinline__ void hllc6(const D* UL, const D* UR, D gamma, D* F) {
  using std::fmax;
  using std::fmin;
  using std::sqrt;
  const D irr_l = D(1.0) / (UL[0] * UR[0]);
  const D irl = UR[0] * irr_l, irr = UL[0] * irr_l;
  const D ul = UL[1] * irl, ur = UR[1] * irr;
  const D gm1 = gamma - D(1.0);
  const D pl = gm1 * (UL[2] - D(0.5) * UL[1] * ul), pr = gm1 * (UR[2] - D(0.5) * UR[1] * ur);
  const D al = sqrt(gamma * pl * irl), ar = sqrt(gamma * pr * irr);
  const D SL = fmin(ul - al, ur - ar), SR = fmax(ul + al, ur + ar);
  const D dl = SL - ul, dr = SR - ur;
  const D Ss = (pr - pl + UL[1] * dl - UR[1] * dr) / (UL[0] * dl - UR[0] * dr);
  const bool left = Ss >= D(0.0);
  const D rK = left ? UL[0] : UR[0], mK = left ? UL[1] : UR[1], EK = left ? UL[2] : UR[2];
  const D uK = left ? ul : ur, pK = left ? pl : pr, irK = left ? irl : irr;
  const D SK = left ? SL : SR, dK = left ? dl : dr;
  const D gap = SK - Ss;
  const D q = D(1.0) / (dK * gap);
  const D f = rK * dK * dK * q;
  const D Es = f * (EK * irK + (Ss - uK) * (Ss + pK * gap * q * irK));
  const D FK0 = mK, FK1 = mK * uK + pK, FK2 = (EK + pK) * uK;
  const D Fs0 = FK0 + SK * (f - rK), Fs1 = FK1 + SK * (f * Ss - mK), Fs2 = FK2 + SK * (Es - EK);
  const bool sup_l = SL >= D(0.0), sup_r = SR <= D(0.0);
  const D FL0 = UL[1], FL1 = UL[1] * ul + pl, FL2 = (UL[2] + pl) * ul;
  const D FR0 = UR[1], FR1 = UR[1] * ur + pr, FR2 = (UR[2] + pr) * ur;
  F[0] = sup_l ? FL0 : (sup_r ? FR0 : Fs0);
  F[1] = sup_l ? FL1 : (sup_r ? FR1 : Fs1);
  F[2] = sup_l ? FL2 : (sup_r ? FR2 : Fs2);
}

// Roe average of the two cells at a face and the eigenvectors of the Euler
// flux Jacobian there, for the speeds u - c, u, u + c: right eigenvectors
// (columns) (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c); left
// ones (rows of the inverse), with b1 = (gamma - 1)/c^2, b2 = b1 u^2 / 2:
// ((b2 + u/c)/2, -(b1 u + 1/c)/2, b1/2), (1 - b2, b1 u, -b1),
// ((b2 - u/c)/2, -(b1 u - 1/c)/2, b1/2). Returns false when the average has
// no real sound speed (the face then keeps the conservative variables).
template <typename D>
struct Eig {
  D u, c, H;
  D L[3][3];
};

template <typename D>
__host__ __device__ __forceinline__ bool roe_eigen(const D* Wa, const D* Wb, D gamma, Eig<D>& e) {
  using std::sqrt;
  const D sa = sqrt(Wa[0]), sb = sqrt(Wb[0]);
  const D isa = D(1.0) / sa, isb = D(1.0) / sb, iss = D(1.0) / (sa + sb);
  const D gm1 = gamma - D(1.0);
  // sqrt(rho) u = m / sqrt(rho); sqrt(rho) H = (E + p) / sqrt(rho)
  const D pa = gm1 * (Wa[2] - D(0.5) * Wa[1] * Wa[1] * isa * isa);
  const D pb = gm1 * (Wb[2] - D(0.5) * Wb[1] * Wb[1] * isb * isb);
  e.u = (Wa[1] * isa + Wb[1] * isb) * iss;
  e.H = ((Wa[2] + pa) * isa + (Wb[2] + pb) * isb) * iss;
  const D c2 = gm1 * (e.H - D(0.5) * e.u * e.u);
  if (!(c2 > D(0.0))) return false;
  e.c = sqrt(c2);
  const D ic = D(1.0) / e.c;
  const D b1 = gm1 * ic * ic, b2 = D(0.5) * b1 * e.u * e.u, uc = e.u * ic;
  e.L[0][0] = D(0.5) * (b2 + uc);
  e.L[0][1] = D(-0.5) * (b1 * e.u + ic);
  e.L[0][2] = D(0.5) * b1;
  e.L[1][0] = D(1.0) - b2;
  e.L[1][1] = b1 * e.u;
  e.L[1][2] = -b1;
  e.L[2][0] = D(0.5) * (b2 - uc);
  e.L[2][1] = D(-0.5) * (b1 * e.u - ic);
  e.L[2][2] = D(0.5) * b1;
  return true;
}

// W = R w with the right eigenvectors of e.
template <typename D>
__host__ __device__ __forceinline__ void from_characteristic(const Eig<D>& e, const D* w, D* W) {
  const D uc = e.u * e.c;
  W[0] = w[0] + w[1] + w[2];
  W[1] = (e.u - e.c) * w[0] + e.u * w[1] + (e.u + e.c) * w[2];
  W[2] = (e.H - uc) * w[0] + D(0.5) * e.u * e.u * w[1] + (e.H + uc) * w[2];
}

// GENO states of the three fields of one face: get(v, m) returns field v of
// cell j-2+m (m = 0..5) around the face x_{j+1/2}.
template <typename D, typename Get>
__host__ __device__ __forceinline__ void reconstruct6(const Get& get, const KP6& k, D* WL, D* WR,
                                                      D* chi) {
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const D u[6] = {get(v, 0), get(v, 1), get(v, 2), get(v, 3), get(v, 4), get(v, 5)};
    Cand<D> cl, cr;
    D p5, p3;
    candidates(u, cl, cr, p5, p3);
    D xl, xr;
    WL[v] = side6(cl, p5, p3, k, xl);
    WR[v] = side6(cr, p5, p3, k, xr);
    if (chi) {
      chi[v] = xl;
      chi[3 + v] = xr;
    }
  }
}

// One face: get(v, m) returns the average of cell j-2+m (m = 0..5) of
// conservative variable v around the face x_{j+1/2} (a functor, so that a
// caller can read each variable's stencil from LDS when it is needed and
// hold only one in registers). CHAR: reconstruct characteristic fields
// (with the conservative fallback of roe_eigen). Writes the guarded states
// WL, WR, the flux F and (chi != nullptr) the six path functions
// [side * 3 + v]; returns the number of guarded sides.
template <typename D, bool CHAR, typename Get>
__host__ __device__ __forceinline__ int face6(const Get& get, const KP6& k, D* WL, D* WR, D* F,
                                              D* chi) {
  bool done = false;
  if constexpr (CHAR) {
    const D Wa[3] = {get(0, 2), get(1, 2), get(2, 2)}, Wb[3] = {get(0, 3), get(1, 3), get(2, 3)};
    Eig<D> e;
    if (roe_eigen(Wa, Wb, D(k.gamma), e)) {
      const auto getw = [&](int v, int m) {
        return e.L[v][0] * get(0, m) + e.L[v][1] * get(1, m) + e.L[v][2] * get(2, m);
      };
      D wl[3], wr[3];
      reconstruct6<D>(getw, k, wl, wr, chi);
      from_characteristic(e, wl, WL);
      from_characteristic(e, wr, WR);
      done = true;
    }
  }
  if (!done) reconstruct6<D>(get, k, WL, WR, chi);
  // guard by selects (no branch: a wave rarely has a guarded lane, and the
  // branch would cost register copies on every path)
  const bool okl = admissible6(WL), okr = admissible6(WR);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    WL[v] = okl ? WL[v] : get(v, 2);
    WR[v] = okr ? WR[v] : get(v, 3);
  }
  hllc6(WL, WR, D(k.gamma), F);
  return (okl ? 0 : 1) + (okr ? 0 : 1);
}

}  // namespace geno6
