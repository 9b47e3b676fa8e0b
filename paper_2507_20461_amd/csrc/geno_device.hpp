// Device functions of the GENO reconstruction (Zhao & Xu, Sec. 3 and Sec. 4.2)
// for gfx950. Scalar per-thread code: one thread owns one face (or one
// face-row) and keeps every intermediate in registers.
#pragma once

#include <hip/hip_runtime.h>

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
};

// Path function chi = tanh(C alpha)/tanh(C) (Eq. (4)) of the ultimate
// smoothness indicator alpha = 2 alpha^H/(alpha^H + alpha^L) with
// alpha^{H,L} = 1 + (IS^tau/(IS^{H,L} + eps))^2 (Eq. (5), r = 2). alpha is
// evaluated over the common denominator (IS^H+eps)^2 (IS^L+eps)^2 so that a
// single division remains. tanh(x) rounds to 1 for x > 19.8 (its distance to
// 1 is below 1e-17), so the call is skipped there.
__device__ __forceinline__ double path_chi(double IStau, double ISH, double ISL,
                                           const KParams& k) {
  const double a = ISH + k.eps, b = ISL + k.eps, t2 = IStau * IStau;
  const double a2 = a * a, b2 = b * b;
  const double num = (a2 + t2) * b2;
  const double alpha = 2.0 * num / (num + (b2 + t2) * a2);
  const double x = k.C * alpha;
  const double th = (x > 19.8) ? 1.0 : tanh(x);
  return (k.tanhC == 1.0) ? th : th / k.tanhC;
}

// Linear high-order reconstruction p^7 on S_0 = {j-1, j, j+1, j+2} (Sec. 4.2)
// at x_{j+1/2}: value and h * derivative of the degree-7 polynomial whose cell
// averages and averaged h-scaled derivatives match those of the four cells.
// Written in symmetric pairs so that the mirrored evaluation is exact.
__device__ __forceinline__ void linear_p7(double Qm, double Q0, double Q1, double Q2, double Gm,
                                          double G0, double G1, double G2, double& qH,
                                          double& hqH) {
  qH = (5.0 * (Qm + Q2) + 37.0 * (Q0 + Q1)) * (1.0 / 84.0) +
       ((Gm - G2) + 17.0 * (G0 - G1)) * (1.0 / 70.0);
  hqH = 7.0 * (Q2 - Qm) * (1.0 / 54.0) + 2.5 * (Q1 - Q0) -
        ((Gm + G2) * (1.0 / 36.0) + 11.0 * (G0 + G1) * (1.0 / 12.0));
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
// is not formed.
__device__ __forceinline__ void geno_side(double Qm, double Q0, double Q1, double Q2, double Gm,
                                          double qH, double hqH, const KParams& k,
                                          double& val, double& hder, double& chi) {
  const double B1 = 2.0 * (Q0 - Qm) - Gm, C1 = (Q0 - Qm) - Gm;
  const double B2 = 0.5 * (Q1 - Qm), C2 = 0.5 * (Q1 - 2.0 * Q0 + Qm);
  const double B3 = 0.5 * (4.0 * Q1 - 3.0 * Q0 - Q2), C3 = 0.5 * (Q0 - 2.0 * Q1 + Q2);
  const double c13 = 13.0 / 3.0;
  const double IS1 = B1 * B1 + c13 * (C1 * C1);
  const double IS2 = B2 * B2 + c13 * (C2 * C2);
  const double IS3 = B3 * B3 + c13 * (C3 * C3);
  const double ISH = fmax(IS1, fmax(IS2, IS3));
  const double ISL = fmin(IS1, fmin(IS2, IS3));
  const double IStau = fabs(0.5 * (IS2 + IS3) - IS1);
  chi = path_chi(IStau, ISH, ISL, k);
  if (chi == 1.0) {
    val = qH;
    hder = hqH;
    return;
  }
  double e1 = IS1 + k.eps, e2 = IS2 + k.eps, e3 = IS3 + k.eps;
  e1 *= e1;
  e2 *= e2;
  e3 *= e3;
  const double w1 = k.d1 * (e2 * e3), w2 = k.d2 * (e1 * e3), w3 = k.d3 * (e1 * e2);
  const double inv = 1.0 / (w1 + w2 + w3);
  const double s6 = 1.0 / 6.0;
  const double p1 = Q0 + 0.5 * B1 + s6 * C1;
  const double p2 = Q0 + 0.5 * B2 + s6 * C2;
  const double p3 = Q0 + 0.5 * B3 + s6 * C3;
  const double qL = (w1 * p1 + w2 * p2 + w3 * p3) * inv;
  const double hqL = (w1 * (B1 + C1) + w2 * (B2 + C2) + w3 * (B3 + C3)) * inv;
  val = chi * qH + (1.0 - chi) * qL;
  hder = chi * hqH + (1.0 - chi) * hqL;
}

// Both states at face j+1/2 for one component from cells j-1..j+2. The right
// state (cell j+1) is the left-state formula applied to the data reflected
// about the face: Q~_m = Q_{1-m}, G~_m = -G_{1-m}; its derivative changes sign.
__device__ __forceinline__ void geno_face(double Qm, double Q0, double Q1, double Q2, double Gm,
                                          double G0, double G1, double G2, const KParams& k,
                                          double& vl, double& dl, double& xl, double& vr,
                                          double& dr, double& xr) {
  double qH, hqH;
  linear_p7(Qm, Q0, Q1, Q2, Gm, G0, G1, G2, qH, hqH);
  geno_side(Qm, Q0, Q1, Q2, Gm, qH, hqH, k, vl, dl, xl);
  double dm;
  geno_side(Q2, Q1, Q0, Qm, -G2, qH, -hqH, k, vr, dm, xr);
  dr = -dm;
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
__device__ __forceinline__ void tangential(double phm, double ph0, double php, const KParams& k,
                                           double& v0, double& v1, double& t0, double& t1) {
  const double sm = ph0 - phm, sp = php - ph0;
  const double sc = 0.5 * (sm + sp), d2 = sp - sm;
  const double ISm = sm * sm, ISp = sp * sp;
  const double chi = path_chi(fabs(ISp - ISm), fmax(ISm, ISp), fmin(ISm, ISp), k);
  double s, th0, th1;
  if (chi == 1.0) {
    s = sc;
    th0 = sc - GENO_ETA * d2;
    th1 = sc + GENO_ETA * d2;
  } else {
    double em = ISm + k.eps, ep = ISp + k.eps;
    em *= em;
    ep *= ep;
    // weights 1/(IS_-+eps)^2 and 1/(IS_++eps)^2 over a common denominator
    const double sL = (ep * sm + em * sp) / (ep + em);
    s = chi * sc + (1.0 - chi) * sL;
    th0 = chi * (sc - GENO_ETA * d2) + (1.0 - chi) * sL;
    th1 = chi * (sc + GENO_ETA * d2) + (1.0 - chi) * sL;
  }
  v0 = ph0 - GENO_ETA * s;
  v1 = ph0 + GENO_ETA * s;
  t0 = th0;
  t1 = th1;
}

}  // namespace geno
