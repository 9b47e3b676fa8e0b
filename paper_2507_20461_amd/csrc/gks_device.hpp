// Gas-kinetic interface flux at one point of a face for gfx950 (the BGK
// interface solution of the high-order GKS family; the paper defers its
// details to the literature, Sec. 2).
//
// Distribution at the face point (time t from the start of the step,
// e = exp(-t/tau)):
//   f = (1 - e) g_c + ((t + tau) e - tau)(abar u + bbar v) g_c
//       + (t - tau (1 - e)) Abar g_c
//       + e sum_{s = l (u > 0), r (u < 0)} g_s [1 - (t + tau)(a_s u + b_s v) - tau A_s]
// g_c: Maxwellian of W_c = sum_s rho_s <psi>_s (half-space moments);
// a, b: micro-slopes of the normal / tangential derivatives; abar, bbar of
// the averaged derivatives over g_c; A: time slopes from the compatibility
// condition.
//
// Identities used to avoid moment sums where a closed form exists: for any
// Maxwellian g of state W and micro-slope a of a change dW,
//   rho <u (a.psi) psi> = J_x(W) dW   (Euler flux Jacobian),
// hence rho_c <u Abar psi>_c = J_x(W_c) W_t with W_t = -(J_x Wbar_n + J_y Wbar_t),
// rho_c <(abar u + bbar v) psi>_c = -W_t and rho_c <Abar psi>_c = W_t.
// With tau = 0 the solution reduces exactly to F = F_Euler(W_c),
// dF/dt = J_x(W_c) W_t and W(t) = W_c + t W_t.
// The time stepping of the gradients also needs the equilibrium's second
// time derivative at the point, W_tt = -d_x (J_x W_t) - d_y (J_y W_t) of the
// Euler equations (the moments of the BGK equilibrium), weighted by
// second_order_weight (1 for smooth data, 0 at a jump of the state or slope),
// formed here from the Hessians of the Euler fluxes:
//   (W_t)_x = -(F''[W_x, W_x] + J_x W_xx + G''[W_x, W_y] + J_y W_xy),
//   (W_t)_y = -(F''[W_x, W_y] + J_x W_xy + G''[W_y, W_y] + J_y W_yy),
//   W_tt = -(F''[W_x, W_t] + J_x (W_t)_x + G''[W_y, W_t] + J_y (W_t)_y),
// with the averaged first and second derivatives of the point.
//
// Templated on the arithmetic type R (double; float in the mixed form) and
// host+device so that an operation-counting type can be substituted.
#pragma once

#include <hip/hip_runtime.h>

#include "geno_device.hpp"

namespace gks {

using geno::KParams;

// Type of the time-fit scalars: float64 when the point arithmetic is float32
// (the fit differences of the time integrals cancel to O(dt^2)), otherwise the
// arithmetic type itself.
template <typename R>
struct Wide {
  using type = R;
};
template <>
struct Wide<float> {
  using type = double;
};

// primitive variables; ir = 1/rho; lam = rho/(2p) only after with_lam()
template <typename R>
struct Prim {
  R rho, ir, U, V, p, lam;
};

template <int NV, typename R>
GENO_HD Prim<R> prim(const R* W, double gamma) {
  Prim<R> q;
  q.rho = W[0];
  q.ir = R(1.0) / W[0];
  q.U = W[1] * q.ir;
  if constexpr (NV == 4) q.V = W[2] * q.ir;
  else q.V = R(0.0);
  R ke = q.U * q.U;
  if constexpr (NV == 4) ke = ke + q.V * q.V;
  q.p = R(gamma - 1.0) * (W[NV - 1] - R(0.5) * q.rho * ke);
  q.lam = R(0.0);
  return q;
}

template <typename R>
GENO_HD void with_lam(Prim<R>& q) {
  q.lam = q.rho / (R(2.0) * q.p);
}

// Euler flux along the first velocity component (face frame).
template <int NV, typename R>
GENO_HD void euler_flux(const R* W, const Prim<R>& q, R* F) {
  F[0] = W[1];
  F[1] = W[1] * q.U + q.p;
  if constexpr (NV == 4) F[2] = W[2] * q.U;
  F[NV - 1] = q.U * (W[NV - 1] + q.p);
}

// J_x(W) dW and J_y(W) dW of the Euler fluxes (face frame: x normal).
template <int NV, typename R>
GENO_HD void jac_x(const R* W, const Prim<R>& q, const R* d, double gamma, R* out) {
  const R ir = q.ir;
  const R dU = (d[1] - q.U * d[0]) * ir;
  R dp;
  if constexpr (NV == 4) {
    dp = R(gamma - 1.0) *
         (d[3] - q.U * d[1] - q.V * d[2] + R(0.5) * (q.U * q.U + q.V * q.V) * d[0]);
    out[2] = d[2] * q.U + W[2] * dU;
  } else {
    dp = R(gamma - 1.0) * (d[2] - q.U * d[1] + R(0.5) * q.U * q.U * d[0]);
  }
  out[0] = d[1];
  out[1] = d[1] * q.U + W[1] * dU + dp;
  out[NV - 1] = dU * (W[NV - 1] + q.p) + q.U * (d[NV - 1] + dp);
}

template <typename R>
GENO_HD void jac_y(const R* W, const Prim<R>& q, const R* d, double gamma, R* out) {
  const R ir = q.ir;
  const R dV = (d[2] - q.V * d[0]) * ir;
  const R dp = R(gamma - 1.0) *
               (d[3] - q.U * d[1] - q.V * d[2] + R(0.5) * (q.U * q.U + q.V * q.V) * d[0]);
  out[0] = d[2];
  out[1] = d[1] * q.V + W[1] * dV;
  out[2] = d[2] * q.V + W[2] * dV + dp;
  out[3] = dV * (W[3] + q.p) + q.V * (d[3] + dp);
}

// F''[b, d]: the Hessian of the Euler flux along x (face frame) applied to
// two changes b, d of the state (symmetric in b and d). With the velocity
// and pressure changes bU = (b_1 - U b_0)/rho, bp = (gamma - 1)(b_E - U b_1 -
// V b_2 + |U|^2/2 b_0) (same for d) and H = (rho E + p)/rho:
//   (0, rho ((3 - gamma) bU dU - (gamma - 1) bV dV), rho (bU dV + dU bV),
//    bU (d_E + dp - H d_0) + dU (b_E + bp - H b_0) - U (gamma - 1) rho (bU dU + bV dV)).
template <int NV, typename R>
GENO_HD void hess_x(const R* W, const Prim<R>& q, const R* b, const R* d, double gamma, R* out) {
  const R gm = R(gamma - 1.0);
  const R H = (W[NV - 1] + q.p) * q.ir;
  const R bU = (b[1] - q.U * b[0]) * q.ir, dU = (d[1] - q.U * d[0]) * q.ir;
  R bp, dp, s;
  if constexpr (NV == 4) {
    const R bV = (b[2] - q.V * b[0]) * q.ir, dV = (d[2] - q.V * d[0]) * q.ir;
    const R k2 = R(0.5) * (q.U * q.U + q.V * q.V);
    bp = gm * (b[3] - q.U * b[1] - q.V * b[2] + k2 * b[0]);
    dp = gm * (d[3] - q.U * d[1] - q.V * d[2] + k2 * d[0]);
    s = bU * dU + bV * dV;
    out[1] = q.rho * (R(3.0 - gamma) * (bU * dU) - gm * (bV * dV));
    out[2] = q.rho * (bU * dV + dU * bV);
  } else {
    const R k2 = R(0.5) * q.U * q.U;
    bp = gm * (b[2] - q.U * b[1] + k2 * b[0]);
    dp = gm * (d[2] - q.U * d[1] + k2 * d[0]);
    s = bU * dU;
    out[1] = q.rho * (R(3.0 - gamma) * s);
  }
  out[0] = R(0.0);
  out[NV - 1] = bU * (d[NV - 1] + dp - H * d[0]) + dU * (b[NV - 1] + bp - H * b[0]) -
                q.U * (gm * q.rho * s);
}

// G''[b, d]: the same for the flux along y (2-D).
template <typename R>
GENO_HD void hess_y(const R* W, const Prim<R>& q, const R* b, const R* d, double gamma, R* out) {
  const R gm = R(gamma - 1.0);
  const R H = (W[3] + q.p) * q.ir;
  const R bU = (b[1] - q.U * b[0]) * q.ir, dU = (d[1] - q.U * d[0]) * q.ir;
  const R bV = (b[2] - q.V * b[0]) * q.ir, dV = (d[2] - q.V * d[0]) * q.ir;
  const R k2 = R(0.5) * (q.U * q.U + q.V * q.V);
  const R bp = gm * (b[3] - q.U * b[1] - q.V * b[2] + k2 * b[0]);
  const R dp = gm * (d[3] - q.U * d[1] - q.V * d[2] + k2 * d[0]);
  const R s = bU * dU + bV * dV;
  out[0] = R(0.0);
  out[1] = q.rho * (bV * dU + dV * bU);
  out[2] = q.rho * (R(3.0 - gamma) * (bV * dV) - gm * (bU * dU));
  out[3] = bV * (d[3] + dp - H * d[0]) + dV * (b[3] + bp - H * b[0]) - q.V * (gm * q.rho * s);
}

// Equilibrium second time derivative W_tt at state W (face frame) from the
// first derivatives dx, dy, the time derivative Wt and the second
// derivatives sxx, sxy, syy (2-D; 1-D uses dx, Wt and sxx only).
template <int NV, typename R>
GENO_HD void second_time(const R* W, const Prim<R>& q, const R* dx, const R* dy, const R* Wt,
                         const R* sxx, const R* sxy, const R* syy, double gamma, R* Wtt) {
  R a[NV], b[NV], tx[NV];
  hess_x<NV, R>(W, q, dx, dx, gamma, a);
  jac_x<NV, R>(W, q, sxx, gamma, b);
#pragma unroll
  for (int v = 0; v < NV; ++v) tx[v] = -(a[v] + b[v]);
  if constexpr (NV == 4) {
    R ty[NV];
    hess_y<R>(W, q, dx, dy, gamma, a);
    jac_y<R>(W, q, sxy, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) tx[v] = tx[v] - (a[v] + b[v]);
    hess_x<NV, R>(W, q, dx, dy, gamma, a);
    jac_x<NV, R>(W, q, sxy, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) ty[v] = -(a[v] + b[v]);
    hess_y<R>(W, q, dy, dy, gamma, a);
    jac_y<R>(W, q, syy, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) ty[v] = ty[v] - (a[v] + b[v]);
    // W_tt = -(F''[W_x, W_t] + J_x (W_t)_x + G''[W_y, W_t] + J_y (W_t)_y)
    hess_x<NV, R>(W, q, dx, Wt, gamma, a);
    jac_x<NV, R>(W, q, tx, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) Wtt[v] = -(a[v] + b[v]);
    hess_y<R>(W, q, dy, Wt, gamma, a);
    jac_y<R>(W, q, ty, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) Wtt[v] = Wtt[v] - (a[v] + b[v]);
  } else {
    (void)dy;
    (void)sxy;
    (void)syy;
    hess_x<NV, R>(W, q, dx, Wt, gamma, a);
    jac_x<NV, R>(W, q, tx, gamma, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) Wtt[v] = -(a[v] + b[v]);
  }
}

// Micro-slope a with <a psi> = w over the Maxwellian (U, V, lam), closed form
// of the 4x4 (3x3 in 1-D) moment system.
template <int NV, typename R>
GENO_HD void micro_slope(const Prim<R>& q, double K, const R* w, R* a) {
  const R il = R(1.0) / q.lam;
  const R l2 = R(2.0) * q.lam;
  if constexpr (NV == 4) {
    const R B = q.U * q.U + q.V * q.V + R(0.5 * (K + 2.0)) * il;
    const R R4 = R(2.0) * w[3] - B * w[0];
    const R R3 = w[2] - q.V * w[0];
    const R R2 = w[1] - q.U * w[0];
    a[3] = q.lam * q.lam * R(4.0 / (K + 2.0)) * (R4 - R(2.0) * q.U * R2 - R(2.0) * q.V * R3);
    a[2] = l2 * R3 - q.V * a[3];
    a[1] = l2 * R2 - q.U * a[3];
    a[0] = w[0] - q.U * a[1] - q.V * a[2] - R(0.5) * a[3] * B;
  } else {
    const R B = q.U * q.U + R(0.5 * (K + 1.0)) * il;
    const R R3 = R(2.0) * w[2] - B * w[0];
    const R R2 = w[1] - q.U * w[0];
    a[2] = q.lam * q.lam * R(4.0 / (K + 1.0)) * (R3 - R(2.0) * q.U * R2);
    a[1] = l2 * R2 - q.U * a[2];
    a[0] = w[0] - q.U * a[1] - R(0.5) * a[2] * B;
  }
}

// Moments of a Maxwellian normalised by its density: u^n (n <= 6) over the
// whole space or one half-space, v^m (m <= 5) over the whole space, and the
// internal energy moments <xi^2>, <xi^4>.
template <typename R>
struct Mom {
  R u[7];
  R v[6];
  R x2, x4;
};

// Fills u[2..6], v[*] and the xi moments from u[0], u[1].
template <int NV, typename R>
GENO_HD void fill_moments(Mom<R>& m, const Prim<R>& q, double K) {
  const R h = R(0.5) / q.lam;
#pragma unroll
  for (int n = 0; n < 5; ++n) m.u[n + 2] = q.U * m.u[n + 1] + R(n + 1) * h * m.u[n];
  m.v[0] = R(1.0);
  if constexpr (NV == 4) {
    m.v[1] = q.V;
#pragma unroll
    for (int n = 0; n < 4; ++n) m.v[n + 2] = q.V * m.v[n + 1] + R(n + 1) * h * m.v[n];
  } else {
#pragma unroll
    for (int n = 1; n < 6; ++n) m.v[n] = R(0.0);
  }
  m.x2 = R(K) * h;
  m.x4 = R(K * (K + 2.0)) * h * h;
}

// <u^i v^j psi> into out (NV components); ZX adds a factor xi^2.
template <int NV, int ZX, typename R>
GENO_HD void mom_psi(const Mom<R>& m, int i, int j, R* out) {
  const R z0 = ZX ? m.x2 : R(1.0), z1 = ZX ? m.x4 : m.x2;
  const R g = m.u[i] * m.v[j];
  out[0] = ZX ? g * z0 : g;
  out[1] = ZX ? m.u[i + 1] * m.v[j] * z0 : m.u[i + 1] * m.v[j];
  if constexpr (NV == 4) {
    out[2] = ZX ? m.u[i] * m.v[j + 1] * z0 : m.u[i] * m.v[j + 1];
    const R s = m.u[i + 2] * m.v[j] + m.u[i] * m.v[j + 2];
    out[3] = R(0.5) * ((ZX ? s * z0 : s) + g * z1);
  } else {
    out[2] = R(0.5) * ((ZX ? m.u[i + 2] * z0 : m.u[i + 2]) + m.u[i] * z1);
  }
}

// <u^i v^j (a.psi) psi>, psi = (1, u, [v,] (u^2 [+ v^2] + xi^2)/2).
template <int NV, typename R>
GENO_HD void mom_a(const Mom<R>& m, const R* a, int i, int j, R* out) {
  R t0[NV], t1[NV], t2[NV], t3[NV], t4[NV], t5[NV];
  mom_psi<NV, 0>(m, i, j, t0);
  mom_psi<NV, 0>(m, i + 1, j, t1);
  mom_psi<NV, 0>(m, i + 2, j, t3);
  mom_psi<NV, 1>(m, i, j, t5);
  if constexpr (NV == 4) {
    mom_psi<NV, 0>(m, i, j + 1, t2);
    mom_psi<NV, 0>(m, i, j + 2, t4);
  }
  const R aE = R(0.5) * a[NV - 1];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    R s = a[0] * t0[k] + a[1] * t1[k];
    if constexpr (NV == 4) s = s + a[2] * t2[k] + aE * (t3[k] + t4[k] + t5[k]);
    else s = s + aE * (t3[k] + t5[k]);
    out[k] = s;
  }
}

// Weight phi of the second-order term of the interface value at a point
// with side states Wl, Wr (primitives pl, pr) and physical normal
// derivatives nl, nr: r is the largest of the jumps between the sides
// relative to their scale (pressure and density |a_l - a_r| / (a_l + a_r);
// the velocity components over the sum of the sound speeds) and of the
// jumps of the normal derivatives over the distance a sound wave covers in
// dt (dt c |d_l - d_r| over the variable's scale: the density sum, that sum
// times c for the momenta, the energy sum; c the mean sound speed);
// phi = 1 for r <= r1 = 1e-2, 1 - x^2 with x = (r - r1) / (r0 - r1) up to
// r0 = 1e-1, 0 beyond. A shock or contact (and the foot of a shock, where
// the states agree but the slopes do not) gives r of order one, resolved
// data r far below r1; phi is continuous, and flat (exactly 1) over the
// whole range of smooth data, where the scheme's rounding sensitivity is
// that of the unweighted term.
template <int NV, typename R>
GENO_HD R second_order_weight(const Prim<R>& pl, const Prim<R>& pr, const R* Wl, const R* Wr,
                              const R* nl, const R* nr, R dt, const KParams& k) {
  const R cl = sqrt(R(k.gamma) * pl.p * pl.ir), cr = sqrt(R(k.gamma) * pr.p * pr.ir);
  const R ic = R(1.0) / (cl + cr);
  R r = fabs(pl.p - pr.p) / (pl.p + pr.p);
  r = fmax(r, fabs(pl.rho - pr.rho) / (pl.rho + pr.rho));
  r = fmax(r, fabs(pl.U - pr.U) * ic);
  if constexpr (NV == 4) r = fmax(r, fabs(pl.V - pr.V) * ic);
  const R rs = pl.rho + pr.rho, dc = dt * R(0.5) * (cl + cr);
  r = fmax(r, dc * fabs(nl[0] - nr[0]) / rs);
#pragma unroll
  for (int v = 1; v < NV - 1; ++v) r = fmax(r, dt * fabs(nl[v] - nr[v]) / rs);
  r = fmax(r, dc * fabs(nl[NV - 1] - nr[NV - 1]) / (fabs(Wl[NV - 1]) + fabs(Wr[NV - 1])));
  constexpr double r1 = 1e-2, r0 = 1e-1;
  if (r <= R(r1)) return R(1.0);
  const R x = (r - R(r1)) * R(1.0 / (r0 - r1));
  return x < R(1.0) ? R(1.0) - x * x : R(0.0);
}

// Kinds of gas-kinetic point, returned by point_flux.
enum { PT_EQUAL = 0, PT_FAST = 1, PT_SLOW = 2 };

// Results at one point: F, dF/dt (time fit of the integrals over dt/2 and
// dt), the interface state W(dt/2) and W(dt) of the solution, and the
// equilibrium second time derivative W_tt.
template <int NV, typename R>
struct PointOut {
  R F[NV], Ft[NV], Wh[NV], Wf[NV], Wtt[NV];
};

// Point flux. Wl, Wr: states (face frame, normal momentum first); nl, nr,
// tl, tr: physical normal / tangential derivatives (tl, tr unused in 1-D);
// snn, snt, stt: physical second derivatives of the point (normal-normal,
// normal-tangential, tangential-tangential; snt, stt unused in 1-D). Writes
// the point's results into o (F only if want_F). Returns PT_SLOW if the
// collision time is positive, else PT_EQUAL for equal states and PT_FAST
// otherwise. With FULL = false a PT_SLOW point is not evaluated and o is not
// written (the caller hands the face to the full path).
template <int NV, bool FULL, typename R>
GENO_HD int point_flux(const R* Wl, const R* Wr, const R* nl, const R* nr, const R* tl,
                        const R* tr, const R* snn, const R* snt, const R* stt,
                        typename Wide<R>::type dt_w, const KParams& k, bool want_F,
                        PointOut<NV, R>& o) {
  using D = typename Wide<R>::type;
  const double g = k.gamma, K = k.K;
  Prim<R> pl = prim<NV, R>(Wl, g), pr = prim<NV, R>(Wr, g);
  const R dt = R(dt_w);
  R tau = R(k.tc1) * dt + R(k.tc2) * dt * fabs(pl.p - pr.p) / (pl.p + pr.p);
  if constexpr (std::is_same<R, float>::value) {
    // float32 states: a pressure difference within eps_ulps units of 2^-24
    // of the pressures is rounding noise; the tau > 0 solution differs from
    // the tau = C1 dt one by terms of order that ratio times the (equally
    // small) relative state difference or h |grad W| / |W|, below the
    // float32 resolution, so that limit is taken
    if (fabs(pl.p - pr.p) <= R(k.eps_ulps * (1.0 / 16777216.0)) * (pl.p + pr.p))
      tau = R(k.tc1) * dt;
  }
  const bool slow = tau > R(0.0);
  if (!FULL && slow) return PT_SLOW;
  // interface equilibrium W_c = rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0}.
  // Equal states give W_c = W_l exactly (the two half-space moments add up
  // to the full ones), so the half-space moments are only formed when the
  // states differ or the full solution needs them.
  bool same = true;
#pragma unroll
  for (int v = 0; v < NV; ++v) same = same && (Wl[v] == Wr[v]);
  R lu0 = R(0), lu1 = R(0), ru0 = R(0), ru1 = R(0);
  R Wc[NV];
  if (same && !slow) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wc[v] = Wl[v];
  } else {
    with_lam(pl);
    with_lam(pr);
    const R sl = sqrt(pl.lam), sr = sqrt(pr.lam);
    const R tl0 = R(0.5) * erfc(-sl * pl.U), tr0 = R(0.5) * erfc(sr * pr.U);
    const R isp = R(0.28209479177387814347);  // 1 / (2 sqrt(pi))
    const R tl1 = exp(-pl.lam * pl.U * pl.U) * isp / sl;
    const R tr1 = exp(-pr.lam * pr.U * pr.U) * isp / sr;
    lu0 = tl0;
    lu1 = pl.U * tl0 + tl1;
    ru0 = tr0;
    ru1 = pr.U * tr0 - tr1;
    const R hl = R(0.5) / pl.lam, hr = R(0.5) / pr.lam;
    const R lu2 = pl.U * lu1 + hl * lu0, ru2 = pr.U * ru1 + hr * ru0;
    Wc[0] = pl.rho * lu0 + pr.rho * ru0;
    Wc[1] = pl.rho * lu1 + pr.rho * ru1;
    if constexpr (NV == 4) {
      Wc[2] = pl.rho * pl.V * lu0 + pr.rho * pr.V * ru0;
      Wc[3] = R(0.5) * (pl.rho * (lu2 + (pl.V * pl.V + hl + R(K) * hl) * lu0) +
                        pr.rho * (ru2 + (pr.V * pr.V + hr + R(K) * hr) * ru0));
    } else {
      Wc[2] = R(0.5) * (pl.rho * (lu2 + R(K) * hl * lu0) + pr.rho * (ru2 + R(K) * hr * ru0));
    }
  }
  Prim<R> pc = pl;
  if (!(same && !slow)) {
    pc = prim<NV, R>(Wc, g);
    with_lam(pc);
  }
  // averaged derivatives and the equilibrium time derivative
  R dn[NV], dtn[NV], Wt[NV], tmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    dn[v] = R(0.5) * (nl[v] + nr[v]);
    if constexpr (NV == 4) dtn[v] = R(0.5) * (tl[v] + tr[v]);
    else dtn[v] = R(0.0);
  }
  jac_x<NV, R>(Wc, pc, dn, g, Wt);
  if constexpr (NV == 4) {
    jac_y<R>(Wc, pc, dtn, g, tmp);
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = -(Wt[v] + tmp[v]);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = -Wt[v];
  }
  R Fe[NV], JW[NV];
  euler_flux<NV, R>(Wc, pc, Fe);
  jac_x<NV, R>(Wc, pc, Wt, g, JW);
  // the second-order term of the interface value: phi W_tt of the
  // equilibrium, phi = 1 where the two sides reconstruct the same state and
  // slope (smooth data) and 0 at a discontinuity (second_order_weight)
  const R phi = second_order_weight<NV, R>(pl, pr, Wl, Wr, nl, nr, dt, k);
  if (phi > R(0.0)) {
    second_time<NV, R>(Wc, pc, dn, dtn, Wt, snn, snt, stt, g, o.Wtt);
    if (phi < R(1.0))
#pragma unroll
      for (int v = 0; v < NV; ++v) o.Wtt[v] = phi * o.Wtt[v];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) o.Wtt[v] = R(0.0);
  }
  const R h = R(0.5) * dt;
  if (!slow) {
    // tau = 0: exact limits of the time integrals
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (want_F) o.F[v] = Fe[v];
      o.Ft[v] = JW[v];
      o.Wh[v] = Wc[v] + h * Wt[v];
      o.Wf[v] = Wc[v] + dt * Wt[v];
    }
    return same ? PT_EQUAL : PT_FAST;
  }
  if constexpr (FULL) {
    // ---- tau > 0 ----
    // time integrals over [0, d] of the weights of the solution, d = dt/2, dt
    const D dd = dt_w, td = D(tau), hh = D(0.5) * dd;
    const D xh = hh / td;
    const D eh = exp(-xh), emh = -expm1(-xh);
    const D ef = eh * eh, emf = emh * (D(2.0) - emh);
    const D tt = td * td;
    const D c1h = hh - td * emh, c1f = dd - td * emf;
    const D c5h = D(2.0) * tt - td * (hh + D(2.0) * td) * eh;
    const D c5f = D(2.0) * tt - td * (dd + D(2.0) * td) * ef;
    const D c2h = c5h - td * hh, c2f = c5f - td * dd;
    const D c3h = D(0.5) * hh * hh - td * hh + tt * emh;
    const D c3f = D(0.5) * dd * dd - td * dd + tt * emf;
    const D c4h = td * emh, c4f = td * emf;
    const D c6h = tt * emh, c6f = tt * emf;
    // fit F(t) = F + t dF/dt to the two integrals
    const D idt = D(1.0) / dd, idt2 = D(4.0) * idt * idt;
    const R f1 = R((D(4.0) * c1h - c1f) * idt), g1 = R((c1f - D(2.0) * c1h) * idt2);
    const R f2 = R((D(4.0) * c2h - c2f) * idt), g2 = R((c2f - D(2.0) * c2h) * idt2);
    const R f3 = R((D(4.0) * c3h - c3f) * idt), g3 = R((c3f - D(2.0) * c3h) * idt2);
    const R f4 = R((D(4.0) * c4h - c4f) * idt), g4 = R((c4f - D(2.0) * c4h) * idt2);
    const R f5 = R((D(4.0) * c5h - c5f) * idt), g5 = R((c5f - D(2.0) * c5h) * idt2);
    const R f6 = R((D(4.0) * c6h - c6f) * idt), g6 = R((c6f - D(2.0) * c6h) * idt2);
    // interface state at d = dt/2 and dt: weights em, (d + tau) e - tau and
    // d - tau em of the equilibrium part; e (1, -(d + tau), -tau) of each side
    const R k1h = R(emh), k2h = R((hh + td) * eh - td), k3h = R(hh - td * emh), k4h = R(hh + td);
    const R k1f = R(emf), k2f = R((dd + td) * ef - td), k3f = R(dd - td * emf), k4f = R(dd + td);
    const R ehr = R(eh), efr = R(ef);

    // equilibrium part: <u (abar u + bbar v) psi>_c needs the moments of g_c
    {
      Mom<R> mc;
      mc.u[0] = R(1.0);
      mc.u[1] = pc.U;
      fill_moments<NV, R>(mc, pc, K);
      R wv[NV], ab[NV], X2[NV];
      const R irc = pc.ir;
#pragma unroll
      for (int v = 0; v < NV; ++v) wv[v] = dn[v] * irc;
      micro_slope<NV, R>(pc, K, wv, ab);
      mom_a<NV, R>(mc, ab, 2, 0, X2);
      if constexpr (NV == 4) {
        R bb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) wv[v] = dtn[v] * irc;
        micro_slope<NV, R>(pc, K, wv, bb);
        mom_a<NV, R>(mc, bb, 1, 1, tmp);
#pragma unroll
        for (int v = 0; v < NV; ++v) X2[v] = X2[v] + tmp[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R x2 = pc.rho * X2[v];
        if (want_F) o.F[v] = f1 * Fe[v] + f2 * x2 + f3 * JW[v];
        o.Ft[v] = g1 * Fe[v] + g2 * x2 + g3 * JW[v];
        o.Wh[v] = k1h * Wc[v] + (k3h - k2h) * Wt[v];
        o.Wf[v] = k1f * Wc[v] + (k3f - k2f) * Wt[v];
      }
    }
    // non-equilibrium part, one side at a time
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const Prim<R>& ps = side ? pr : pl;
      const R* Ws = side ? Wr : Wl;
      const R* ns = side ? nr : nl;
      const R* ts = side ? tr : tl;
      Mom<R> ms;
      ms.u[0] = side ? ru0 : lu0;
      ms.u[1] = side ? ru1 : lu1;
      fill_moments<NV, R>(ms, ps, K);
      const R irs = ps.ir;
      R wv[NV], as[NV], bs[NV], As[NV], Ws_t[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) wv[v] = ns[v] * irs;
      micro_slope<NV, R>(ps, K, wv, as);
      jac_x<NV, R>(Ws, ps, ns, g, Ws_t);
      if constexpr (NV == 4) {
#pragma unroll
        for (int v = 0; v < NV; ++v) wv[v] = ts[v] * irs;
        micro_slope<NV, R>(ps, K, wv, bs);
        jac_y<R>(Ws, ps, ts, g, tmp);
#pragma unroll
        for (int v = 0; v < NV; ++v) Ws_t[v] = -(Ws_t[v] + tmp[v]) * irs;
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Ws_t[v] = -Ws_t[v] * irs;
      }
      micro_slope<NV, R>(ps, K, Ws_t, As);
      R U1[NV], Xs[NV], Ys[NV], P0[NV], Zs[NV], A0[NV];
      mom_psi<NV, 0>(ms, 1, 0, U1);  // <u psi>
      mom_a<NV, R>(ms, as, 2, 0, Xs);  // <u^2 (a.psi) psi>
      mom_a<NV, R>(ms, As, 1, 0, Ys);  // <u (A.psi) psi>
      mom_psi<NV, 0>(ms, 0, 0, P0);  // <psi>
      mom_a<NV, R>(ms, as, 1, 0, Zs);  // <u (a.psi) psi>
      mom_a<NV, R>(ms, As, 0, 0, A0);  // <(A.psi) psi>
      if constexpr (NV == 4) {
        mom_a<NV, R>(ms, bs, 1, 1, tmp);  // <u v (b.psi) psi>
#pragma unroll
        for (int v = 0; v < NV; ++v) Xs[v] = Xs[v] + tmp[v];
        mom_a<NV, R>(ms, bs, 0, 1, tmp);  // <v (b.psi) psi>
#pragma unroll
        for (int v = 0; v < NV; ++v) Zs[v] = Zs[v] + tmp[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R r = ps.rho;
        if (want_F) o.F[v] = o.F[v] + r * (f4 * U1[v] - f5 * Xs[v] - f6 * Ys[v]);
        o.Ft[v] = o.Ft[v] + r * (g4 * U1[v] - g5 * Xs[v] - g6 * Ys[v]);
        o.Wh[v] = o.Wh[v] + ehr * r * (P0[v] - k4h * Zs[v] - tau * A0[v]);
        o.Wf[v] = o.Wf[v] + efr * r * (P0[v] - k4f * Zs[v] - tau * A0[v]);
      }
    }
  }
  return PT_SLOW;
}

}  // namespace gks
