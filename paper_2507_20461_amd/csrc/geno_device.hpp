// Device functions of the GENO reconstruction (Zhao & Xu, Sec. 3 and Sec. 4.2)
// for gfx950. Scalar per-thread code: one thread owns one face-row (normal
// step) or one (face, side, variable) (tangential step) and keeps every
// intermediate in registers.
//
// Templated on the arithmetic type R of the reconstruction (double, float)
// and on the type D of the smoothness indicators (always double on the GPU:
// eps = 1e-15 and IS^2 ~ 1e-30 are out of FP32 range, and the indicators of
// the normal step are formed from the float64 cell data, because rounding
// nearly constant data to float32 leaves steps of one unit in the last place
// whose indicators, ~1e-15 |q|^2, would read as discontinuities). The
// functions are host+device so that the same code can be instantiated with an
// operation-counting type on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#define GENO_HD __host__ __device__ __forceinline__

namespace geno {

// Constants seen by the kernels (filled on the host from geno_params).
struct KParams {
  double C;       // path-function steepness, Eq. (4)
  double tanhC;   // tanh(C)
  double eps;     // Eq. (5) and Eq. (8)
  double d1, d2, d3;  // linear weights of S_1, S_2, S_3 (Eq. (8))
  double gamma;
  double K;       // internal degrees of freedom of the BGK model
  double tc1, tc2;    // collision time coefficients
  double cfl;
  double dt_fixed;    // > 0: fixed time step instead of the CFL condition
  double eps_ulps;    // float32 data: eps floor in units of 2^-24 of the stencil magnitude
  double gate_thr;    // learned gate: a prediction >= gate_thr sets chi = 1
  int gate;           // learned gate enabled
  int charvars;       // reconstruct characteristic variables in the normal step
  int fuse;           // 2-D steps: normal step inside the face kernels (host side)
};

// Path function chi = tanh(C alpha)/tanh(C) (Eq. (4)) of the ultimate
// smoothness indicator alpha = 2 alpha^H/(alpha^H + alpha^L) with
// alpha^{H,L} = 1 + (IS^tau/(IS^{H,L} + eps))^2 (Eq. (5), r = 2). alpha is
// evaluated over the common denominator (IS^H+eps)^2 (IS^L+eps)^2 so that a
// single division remains. tanh(x) rounds to 1 in float64 for x > 19.1, so
// once C alpha > 19.8 chi is tanh(C)^-1 exactly; that test is made on the
// numerator and denominator of alpha, without the division (near the
// threshold both ways give tanh(x) = 1).
template <typename D>
GENO_HD D path_chi(D IStau, D ISH, D ISL, D eps, const KParams& k) {
  const D a = ISH + eps, b = ISL + eps, t2 = IStau * IStau;
  const D a2 = a * a, b2 = b * b;
  const D num = (a2 + t2) * b2;
  const D den = num + (b2 + t2) * a2;
  D th;
  if (D(2.0 * k.C) * num > D(19.8) * den) {
    th = D(1.0);
  } else {
    const D alpha = 2.0 * num / den;
    th = tanh(k.C * alpha);
  }
  return (k.tanhC == 1.0) ? th : th / k.tanhC;
}

// eps of Eq. (5) and (8). With float32 reconstruction data (the mixed form)
// the absolute 1e-15 lies below the data's own rounding: float32 face values,
// and the gradients formed from differences of them, carry rounding of a few
// to ~10 units in the last place of |q| (2^-24 |q|) from the few dozen
// operations that produce them, and indicators of that noise (>= 4e-15 |q|^2)
// would read as discontinuities. There eps is raised by
// (eps_ulps 2^-24 qmax)^2, qmax the largest |value| of the stencil; float64
// data keep the plain eps.
template <typename R, typename D>
GENO_HD D eps_of(D qmax, const KParams& k) {
  if constexpr (std::is_same<R, float>::value) {
    const D f = D(k.eps_ulps * (1.0 / 16777216.0)) * qmax;
    return k.eps + f * f;
  } else {
    (void)qmax;
    return D(k.eps);
  }
}

// Linear high-order reconstruction p^7 on S_0 = {j-1, j, j+1, j+2} (Sec. 4.2)
// at x_{j+1/2}: value and h * derivative (linear_p7) and h^2 * second
// derivative (linear_p7_d2) of the degree-7 polynomial whose cell averages
// and averaged h-scaled derivatives match those of the four cells. Written
// in symmetric pairs so that the mirrored evaluation is exact (the second
// derivative is even under the mirror).
template <typename R>
GENO_HD void linear_p7(R Qm, R Q0, R Q1, R Q2, R Gm, R G0, R G1, R G2, R& qH, R& hqH) {
  qH = (R(5.0) * (Qm + Q2) + R(37.0) * (Q0 + Q1)) * R(1.0 / 84.0) +
       ((Gm - G2) + R(17.0) * (G0 - G1)) * R(1.0 / 70.0);
  hqH = R(7.0) * (Q2 - Qm) * R(1.0 / 54.0) + R(2.5) * (Q1 - Q0) -
        ((Gm + G2) * R(1.0 / 36.0) + R(11.0) * (G0 + G1) * R(1.0 / 12.0));
}
template <typename R>
GENO_HD R linear_p7_d2(R Qm, R Q0, R Q1, R Q2, R Gm, R G0, R G1, R G2) {
  return ((Q0 + Q1) - (Qm + Q2)) + (R(9.0) * (G1 - G0) + (G2 - Gm)) * R(0.25);
}

// GENO value and h * derivative at the face on the right of cell j (the
// left state), Eq. (3), (7)-(9), (13)-(14). Sub-stencil quadratics
// p_k(xi) = a_k + B_k xi + C_k xi^2 in xi = (x - x_j)/h:
//   S_1 = {j-1, j} with the averaged derivative of j-1,
//   S_2 = {j-1, j, j+1}, S_3 = {j, j+1, j+2};
// IS_k = B_k^2 + 13/3 C_k^2 (Jiang-Shu form of Eq. (6) on cell j);
// IS^H = max, IS^L = min, IS^tau = |(IS_2 + IS_3)/2 - IS_1|; ENO weights
// d_k/(IS_k + eps)^2 normalised (Eq. (8)), evaluated over a common
// denominator. When chi == 1 exactly the low-order part carries weight 0 and
// is not formed. Returns true on the low-order branch (chi < 1).
// Coefficients B_k, C_k of the three sub-stencil quadratics of one side and
// their indicators IS_k (Jiang-Shu form of Eq. (6) on cell j).
template <typename D>
struct SideQuads {
  D B1, C1, B2, C2, B3, C3, IS1, IS2, IS3;
};

template <typename D>
GENO_HD SideQuads<D> side_quads(D Qm, D Q0, D Q1, D Q2, D Gm) {
  SideQuads<D> s;
  s.B1 = D(2.0) * (Q0 - Qm) - Gm;
  s.C1 = (Q0 - Qm) - Gm;
  s.B2 = D(0.5) * (Q1 - Qm);
  s.C2 = D(0.5) * (Q1 - D(2.0) * Q0 + Qm);
  s.B3 = D(0.5) * (D(4.0) * Q1 - D(3.0) * Q0 - Q2);
  s.C3 = D(0.5) * (Q0 - D(2.0) * Q1 + Q2);
  const D c13 = D(13.0 / 3.0);
  s.IS1 = s.B1 * s.B1 + c13 * (s.C1 * s.C1);
  s.IS2 = s.B2 * s.B2 + c13 * (s.C2 * s.C2);
  s.IS3 = s.B3 * s.B3 + c13 * (s.C3 * s.C3);
  return s;
}

template <typename R, typename D>
GENO_HD bool geno_side(D Qm, D Q0, D Q1, D Q2, D Gm, R qH, R hqH, R h2qH, const KParams& k,
                       R& val, R& hder, R& h2der, D& chi) {
  const SideQuads<D> sq = side_quads<D>(Qm, Q0, Q1, Q2, Gm);
  const D Bd1 = sq.B1, Cd1 = sq.C1, Bd2 = sq.B2, Cd2 = sq.C2, Bd3 = sq.B3, Cd3 = sq.C3;
  const D IS1 = sq.IS1, IS2 = sq.IS2, IS3 = sq.IS3;
  const D ISH = fmax(IS1, fmax(IS2, IS3));
  const D ISL = fmin(IS1, fmin(IS2, IS3));
  const D IStau = fabs(0.5 * (IS2 + IS3) - IS1);
  const D eps = eps_of<R, D>(fmax(fmax(fabs(Qm), fabs(Q0)), fmax(fabs(Q1), fabs(Q2))), k);
  chi = path_chi<D>(IStau, ISH, ISL, eps, k);
  if (chi == 1.0) {
    val = qH;
    hder = hqH;
    h2der = h2qH;
    return false;
  }
  D e1 = IS1 + eps, e2 = IS2 + eps, e3 = IS3 + eps;
  e1 = e1 * e1;
  e2 = e2 * e2;
  e3 = e3 * e3;
  const D w1 = k.d1 * (e2 * e3), w2 = k.d2 * (e1 * e3), w3 = k.d3 * (e1 * e2);
  const D inv = 1.0 / (w1 + w2 + w3);
  const R o1 = R(w1 * inv), o2 = R(w2 * inv), o3 = R(w3 * inv);
  const R B1 = R(Bd1), C1 = R(Cd1), B2 = R(Bd2), C2 = R(Cd2), B3 = R(Bd3), C3 = R(Cd3);
  const R q0 = R(Q0), s6 = R(1.0 / 6.0);
  const R p1 = q0 + R(0.5) * B1 + s6 * C1;
  const R p2 = q0 + R(0.5) * B2 + s6 * C2;
  const R p3 = q0 + R(0.5) * B3 + s6 * C3;
  const R qL = o1 * p1 + o2 * p2 + o3 * p3;
  const R hqL = o1 * (B1 + C1) + o2 * (B2 + C2) + o3 * (B3 + C3);
  // second derivatives of the quadratics: h^2 p_k'' = 2 C_k
  const R h2qL = R(2.0) * (o1 * C1 + o2 * C2 + o3 * C3);
  const R x = R(chi), xm = R(1.0 - chi);
  val = x * qH + xm * qL;
  hder = x * hqH + xm * hqL;
  h2der = x * h2qH + xm * h2qL;
  return true;
}

// Both states at face j+1/2 for one component from cells j-1..j+2 (data in
// the indicator type D, the linear part evaluated in R). The right state
// (cell j+1) is the left-state formula applied to the data reflected about
// the face: Q~_m = Q_{1-m}, G~_m = -G_{1-m}; its derivative changes sign, its
// second derivative does not. A side marked skip (by the learned gate) takes
// chi = 1, the linear reconstruction, without its indicators. h2: the mean of
// the two sides' h^2 * second derivatives (the time stepping of the gradients
// uses the mean). Returns the number of sides on the low-order branch.
template <typename R, typename D>
GENO_HD int geno_face(D Qm, D Q0, D Q1, D Q2, D Gm, D G0, D G1, D G2, const KParams& k, R& vl,
                      R& dl, D& xl, R& vr, R& dr, D& xr, R& h2, bool skipL = false,
                      bool skipR = false) {
  R qH, hqH;
  linear_p7<R>(R(Qm), R(Q0), R(Q1), R(Q2), R(Gm), R(G0), R(G1), R(G2), qH, hqH);
  const R h2qH = linear_p7_d2<R>(R(Qm), R(Q0), R(Q1), R(Q2), R(Gm), R(G0), R(G1), R(G2));
  int n = 0;
  R sl, sr;
  if (skipL) {
    vl = qH;
    dl = hqH;
    sl = h2qH;
    xl = D(1.0);
  } else {
    n += geno_side<R, D>(Qm, Q0, Q1, Q2, Gm, qH, hqH, h2qH, k, vl, dl, sl, xl);
  }
  if (skipR) {
    vr = qH;
    dr = hqH;
    sr = h2qH;
    xr = D(1.0);
  } else {
    R dm;
    n += geno_side<R, D>(Q2, Q1, Q0, Qm, -G2, qH, -hqH, h2qH, k, vr, dm, sr, xr);
    dr = -dm;
  }
  h2 = R(0.5) * (sl + sr);
  return n;
}

// The paper's comparison (Sec. 5): the share of the linear reconstruction
// that WENO-Z and TENO weights on the same three sub-stencils keep,
// chi = min_k w_k / d_k, d_k the linear weights normalised to sum 1.
// WENO-Z: w~_k = d_k (1 + tau_Z / (IS_k + eps)), tau_Z = |IS_1 - IS_3| (the
// two outer sub-stencils).
template <typename D>
GENO_HD D wenoz_chi(D IS1, D IS2, D IS3, const KParams& k) {
  const D dsum = D(k.d1) + D(k.d2) + D(k.d3);
  const D d[3] = {D(k.d1) / dsum, D(k.d2) / dsum, D(k.d3) / dsum};
  const D IS[3] = {IS1, IS2, IS3};
  const D tz = fabs(IS1 - IS3);
  D w[3], ws = D(0.0);
  for (int q = 0; q < 3; ++q) {
    w[q] = d[q] * (D(1.0) + tz / (IS[q] + D(k.eps)));
    ws = ws + w[q];
  }
  D chi = (w[0] / ws) / d[0];
  for (int q = 1; q < 3; ++q) chi = fmin(chi, (w[q] / ws) / d[q]);
  return chi;
}

// TENO: scale separation gamma_k = (1/(IS_k + eps))^7 normalised; a
// sub-stencil with gamma_k <= ct is cut (weight 0), the others keep their
// linear weights renormalised. chi is 1 when none is cut, else 0.
template <typename D>
GENO_HD D teno_chi(D IS1, D IS2, D IS3, D ct, const KParams& k) {
  const D IS[3] = {IS1, IS2, IS3};
  D g[3], gs = D(0.0);
  for (int q = 0; q < 3; ++q) {
    const D x = D(1.0) / (IS[q] + D(k.eps));
    const D x2 = x * x;
    g[q] = x2 * x2 * x2 * x;
    gs = gs + g[q];
  }
  for (int q = 0; q < 3; ++q)
    if (!(g[q] / gs > ct)) return D(0.0);
  return D(1.0);
}

// Gauss points of a face: +-1/(2 sqrt 3) of its length about its centre.
#define GENO_ETA 0.28867513459481288225

// Tangential step to the two Gauss points of a face (2-D; the paper's
// structured scheme is 1-D, so this is the reading used here). phm, ph0,
// php: face averages of one side and component on rows t-1, t, t+1. The
// high-order candidate is the quadratic through the three averages (value
// ph0 +- eta s_c, h * slope s_c +- eta D2 since eta^2 = 1/12); the low-order
// one the ENO combination (d = 1, r^L = 2) of the slopes s_- and s_+; the two
// are blended by the path function with IS_+- = s_+-^2, IS^H = max,
// IS^L = min, IS^tau = |IS_+ - IS_-|. Point 0 is at -eta, point 1 at +eta.
// chi_t: the blend weight; h^2 * the second tangential derivative of the
// blend is chi_t D2 (d2_out = D2; the low-order candidate is linear).
// Returns true on the low-order branch.
template <typename R, typename D>
GENO_HD bool tangential(R phm, R ph0, R php, const KParams& k, R& v0, R& v1, R& t0, R& t1,
                        R& chi_t, R& d2_out) {
  const R sm = ph0 - phm, sp = php - ph0;
  const R sc = R(0.5) * (sm + sp), d2 = sp - sm;
  const D ISm = D(sm * sm), ISp = D(sp * sp);
  const D eps = eps_of<R, D>(D(fmax(fmax(fabs(phm), fabs(ph0)), fabs(php))), k);
  const D chi = path_chi<D>(fabs(ISp - ISm), fmax(ISm, ISp), fmin(ISm, ISp), eps, k);
  const R eta = R(GENO_ETA);
  R s, th0, th1;
  bool low = false;
  if (chi == 1.0) {
    s = sc;
    th0 = sc - eta * d2;
    th1 = sc + eta * d2;
  } else {
    low = true;
    D em = ISm + eps, ep = ISp + eps;
    em = em * em;
    ep = ep * ep;
    // weights 1/(IS_-+eps)^2 and 1/(IS_++eps)^2 over a common denominator
    const D inv = 1.0 / (ep + em);
    const R wm = R(ep * inv), wp = R(em * inv);
    const R sL = wm * sm + wp * sp;
    const R x = R(chi), xm = R(1.0 - chi);
    s = x * sc + xm * sL;
    th0 = x * (sc - eta * d2) + xm * sL;
    th1 = x * (sc + eta * d2) + xm * sL;
  }
  v0 = ph0 - eta * s;
  v1 = ph0 + eta * s;
  t0 = th0;
  t1 = th1;
  chi_t = R(chi);
  d2_out = d2;
  return low;
}

// Point state admissible for the flux: finite, rho > 0, p > 0.
template <int NV, typename R>
GENO_HD bool admissible(const R* W, double gamma) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (!isfinite(W[v])) return false;
  if (!(W[0] > R(0.0))) return false;
  R ke = W[1] * W[1];
  if constexpr (NV == 4) ke = ke + W[2] * W[2];
  // p = (gamma - 1)(rhoE - |m|^2 / (2 rho)) > 0  <=>  rho rhoE - |m|^2 / 2 > 0 (rho > 0)
  (void)gamma;
  return W[0] * W[NV - 1] - R(0.5) * ke > R(0.0);
}

// Characteristic fields of the 2-D Euler flux Jacobian along a face normal,
// at the Roe average of the two cells at the face, in the normal frame
// (rho, rho un, rho ut, rho E). Right eigenvectors (columns) for the speeds
// un - c, un, un (shear) and un + c:
//   (1, un - c, ut, H - un c), (1, un, ut, q^2/2), (0, 0, 1, ut),
//   (1, un + c, ut, H + un c),  q^2 = un^2 + ut^2,
// and their inverse in closed form, with b1 = (gamma - 1)/c^2, b2 = b1 q^2/2:
//   ((b2 + un/c)/2, -(b1 un + 1/c)/2, -b1 ut/2, b1/2),
//   (1 - b2, b1 un, b1 ut, -b1), (-ut, 0, 1, 0),
//   ((b2 - un/c)/2, -(b1 un - 1/c)/2, -b1 ut/2, b1/2).
struct Eig2 {
  double un, ut, c, H, q2;
  double L[4][4];
};

// false when the average has no real sound speed (the face then keeps the
// conservative variables)
GENO_HD bool roe_eigen2(const double* Wa, const double* Wb, double gamma, Eig2& e) {
  const double sa = sqrt(Wa[0]), sb = sqrt(Wb[0]);
  const double isa = 1.0 / sa, isb = 1.0 / sb, iss = 1.0 / (sa + sb);
  const double gm1 = gamma - 1.0;
  const double pa = gm1 * (Wa[3] - 0.5 * (Wa[1] * Wa[1] + Wa[2] * Wa[2]) * isa * isa);
  const double pb = gm1 * (Wb[3] - 0.5 * (Wb[1] * Wb[1] + Wb[2] * Wb[2]) * isb * isb);
  // sqrt(rho) u = m / sqrt(rho); sqrt(rho) H = (E + p) / sqrt(rho)
  e.un = (Wa[1] * isa + Wb[1] * isb) * iss;
  e.ut = (Wa[2] * isa + Wb[2] * isb) * iss;
  e.H = ((Wa[3] + pa) * isa + (Wb[3] + pb) * isb) * iss;
  e.q2 = e.un * e.un + e.ut * e.ut;
  const double c2 = gm1 * (e.H - 0.5 * e.q2);
  if (!(c2 > 0.0)) return false;
  e.c = sqrt(c2);
  const double ic = 1.0 / e.c;
  const double b1 = gm1 * ic * ic, b2 = 0.5 * b1 * e.q2, uc = e.un * ic;
  e.L[0][0] = 0.5 * (b2 + uc);
  e.L[0][1] = -0.5 * (b1 * e.un + ic);
  e.L[0][2] = -0.5 * b1 * e.ut;
  e.L[0][3] = 0.5 * b1;
  e.L[1][0] = 1.0 - b2;
  e.L[1][1] = b1 * e.un;
  e.L[1][2] = b1 * e.ut;
  e.L[1][3] = -b1;
  e.L[2][0] = -e.ut;
  e.L[2][1] = 0.0;
  e.L[2][2] = 1.0;
  e.L[2][3] = 0.0;
  e.L[3][0] = 0.5 * (b2 - uc);
  e.L[3][1] = -0.5 * (b1 * e.un - ic);
  e.L[3][2] = e.L[0][2];
  e.L[3][3] = e.L[0][3];
  return true;
}

// W = R w (normal frame) with the right eigenvectors of e.
GENO_HD void from_characteristic2(const Eig2& e, const double* w, double* W) {
  const double uc = e.un * e.c, s = w[0] + w[1] + w[3];
  W[0] = s;
  W[1] = (e.un - e.c) * w[0] + e.un * w[1] + (e.un + e.c) * w[3];
  W[2] = e.ut * s + w[2];
  W[3] = (e.H - uc) * w[0] + 0.5 * e.q2 * w[1] + e.ut * w[2] + (e.H + uc) * w[3];
}

}  // namespace geno
