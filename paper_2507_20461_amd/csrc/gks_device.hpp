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
#pragma once

#include <hip/hip_runtime.h>

#include "geno_device.hpp"

namespace gks {

using geno::KParams;

template <int NV>
struct Prim {
  double rho, U, V, p, lam;
};

template <int NV>
__device__ __forceinline__ Prim<NV> prim(const double* W, double gamma) {
  Prim<NV> q;
  q.rho = W[0];
  const double ir = 1.0 / W[0];
  q.U = W[1] * ir;
  q.V = (NV == 4) ? W[2] * ir : 0.0;
  q.p = (gamma - 1.0) * (W[NV - 1] - 0.5 * q.rho * (q.U * q.U + q.V * q.V));
  q.lam = q.rho / (2.0 * q.p);
  return q;
}

// Euler flux along the first velocity component (face frame).
template <int NV>
__device__ __forceinline__ void euler_flux(const double* W, const Prim<NV>& q, double* F) {
  F[0] = W[1];
  F[1] = W[1] * q.U + q.p;
  if constexpr (NV == 4) F[2] = W[2] * q.U;
  F[NV - 1] = q.U * (W[NV - 1] + q.p);
}

// J_x(W) dW and J_y(W) dW of the Euler fluxes (face frame: x normal).
template <int NV>
__device__ __forceinline__ void jac_x(const double* W, const Prim<NV>& q, const double* d,
                                      double gamma, double* out) {
  const double ir = 1.0 / q.rho;
  const double dU = (d[1] - q.U * d[0]) * ir;
  double dp;
  if constexpr (NV == 4) {
    dp = (gamma - 1.0) * (d[3] - q.U * d[1] - q.V * d[2] + 0.5 * (q.U * q.U + q.V * q.V) * d[0]);
    out[2] = d[2] * q.U + W[2] * dU;
  } else {
    dp = (gamma - 1.0) * (d[2] - q.U * d[1] + 0.5 * q.U * q.U * d[0]);
  }
  out[0] = d[1];
  out[1] = d[1] * q.U + W[1] * dU + dp;
  out[NV - 1] = dU * (W[NV - 1] + q.p) + q.U * (d[NV - 1] + dp);
}

__device__ __forceinline__ void jac_y(const double* W, const Prim<4>& q, const double* d,
                                      double gamma, double* out) {
  const double ir = 1.0 / q.rho;
  const double dV = (d[2] - q.V * d[0]) * ir;
  const double dp =
      (gamma - 1.0) * (d[3] - q.U * d[1] - q.V * d[2] + 0.5 * (q.U * q.U + q.V * q.V) * d[0]);
  out[0] = d[2];
  out[1] = d[1] * q.V + W[1] * dV;
  out[2] = d[2] * q.V + W[2] * dV + dp;
  out[3] = dV * (W[3] + q.p) + q.V * (d[3] + dp);
}

// Micro-slope a with <a psi> = w over the Maxwellian (U, V, lam), closed form
// of the 4x4 (3x3 in 1-D) moment system.
template <int NV>
__device__ __forceinline__ void micro_slope(const Prim<NV>& q, double K, const double* w,
                                            double* a) {
  const double il = 1.0 / q.lam;
  if constexpr (NV == 4) {
    const double B = q.U * q.U + q.V * q.V + 0.5 * (K + 2.0) * il;
    const double R4 = 2.0 * w[3] - B * w[0];
    const double R3 = w[2] - q.V * w[0];
    const double R2 = w[1] - q.U * w[0];
    a[3] = 4.0 * q.lam * q.lam / (K + 2.0) * (R4 - 2.0 * q.U * R2 - 2.0 * q.V * R3);
    a[2] = 2.0 * q.lam * R3 - q.V * a[3];
    a[1] = 2.0 * q.lam * R2 - q.U * a[3];
    a[0] = w[0] - q.U * a[1] - q.V * a[2] - 0.5 * a[3] * B;
  } else {
    const double B = q.U * q.U + 0.5 * (K + 1.0) * il;
    const double R3 = 2.0 * w[2] - B * w[0];
    const double R2 = w[1] - q.U * w[0];
    a[2] = 4.0 * q.lam * q.lam / (K + 1.0) * (R3 - 2.0 * q.U * R2);
    a[1] = 2.0 * q.lam * R2 - q.U * a[2];
    a[0] = w[0] - q.U * a[1] - 0.5 * a[2] * B;
  }
}

// Moments of a Maxwellian normalised by its density: u^n (n <= 6) over the
// whole space or one half-space, v^m (m <= 5) over the whole space, and the
// internal energy moments <xi^2>, <xi^4>.
template <int NV>
struct Mom {
  double u[7];
  double v[6];
  double x2, x4;
};

// Fills u[2..6], v[*] and the xi moments from u[0], u[1].
template <int NV>
__device__ __forceinline__ void fill_moments(Mom<NV>& m, const Prim<NV>& q, double K) {
  const double h = 0.5 / q.lam;
#pragma unroll
  for (int n = 0; n < 5; ++n) m.u[n + 2] = q.U * m.u[n + 1] + (n + 1) * h * m.u[n];
  m.v[0] = 1.0;
  if constexpr (NV == 4) {
    m.v[1] = q.V;
#pragma unroll
    for (int n = 0; n < 4; ++n) m.v[n + 2] = q.V * m.v[n + 1] + (n + 1) * h * m.v[n];
  } else {
#pragma unroll
    for (int n = 1; n < 6; ++n) m.v[n] = 0.0;
  }
  m.x2 = K * h;
  m.x4 = K * (K + 2.0) * h * h;
}

// <u^i v^j psi> into out (NV components); zx = 0 / 1 adds a factor xi^2.
template <int NV>
__device__ __forceinline__ void mom_psi(const Mom<NV>& m, int i, int j, int zx, double* out) {
  const double z0 = zx ? m.x2 : 1.0, z1 = zx ? m.x4 : m.x2;
  const double g = m.u[i] * m.v[j];
  out[0] = g * z0;
  out[1] = m.u[i + 1] * m.v[j] * z0;
  if constexpr (NV == 4) {
    out[2] = m.u[i] * m.v[j + 1] * z0;
    out[3] = 0.5 * ((m.u[i + 2] * m.v[j] + m.u[i] * m.v[j + 2]) * z0 + g * z1);
  } else {
    out[2] = 0.5 * (m.u[i + 2] * z0 + m.u[i] * z1);
  }
}

// <u^i v^j (a.psi) psi>, psi = (1, u, [v,] (u^2 [+ v^2] + xi^2)/2).
template <int NV>
__device__ __forceinline__ void mom_a(const Mom<NV>& m, const double* a, int i, int j,
                                      double* out) {
  double t0[NV], t1[NV], t2[NV], t3[NV], t4[NV], t5[NV];
  mom_psi<NV>(m, i, j, 0, t0);
  mom_psi<NV>(m, i + 1, j, 0, t1);
  mom_psi<NV>(m, i + 2, j, 0, t3);
  mom_psi<NV>(m, i, j, 1, t5);
  if constexpr (NV == 4) {
    mom_psi<NV>(m, i, j + 1, 0, t2);
    mom_psi<NV>(m, i, j + 2, 0, t4);
  }
  const double aE = 0.5 * a[NV - 1];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = a[0] * t0[k] + a[1] * t1[k];
    if constexpr (NV == 4) s += a[2] * t2[k] + aE * (t3[k] + t4[k] + t5[k]);
    else s += aE * (t3[k] + t5[k]);
    out[k] = s;
  }
}

// Point flux. Wl, Wr: states (face frame, normal momentum first); nl, nr,
// tl, tr: physical normal / tangential derivatives (tl, tr unused in 1-D).
// Accumulates w * F, w * dF/dt and w * W(dt/2) into F, Ft, Wi (F may be
// skipped with want_F = false).
template <int NV>
__device__ __forceinline__ void point_flux(const double* Wl, const double* Wr, const double* nl,
                                           const double* nr, const double* tl, const double* tr,
                                           double dt, const KParams& k, double w, bool want_F,
                                           double* F, double* Ft, double* Wi) {
  const double g = k.gamma, K = k.K;
  const Prim<NV> pl = prim<NV>(Wl, g), pr = prim<NV>(Wr, g);
  // half-space u^0, u^1 moments of both sides
  const double sl = sqrt(pl.lam), sr = sqrt(pr.lam);
  const double tl0 = 0.5 * erfc(-sl * pl.U), tr0 = 0.5 * erfc(sr * pr.U);
  const double isp = 0.28209479177387814347;  // 1 / (2 sqrt(pi))
  const double tl1 = exp(-pl.lam * pl.U * pl.U) * isp / sl;
  const double tr1 = exp(-pr.lam * pr.U * pr.U) * isp / sr;
  const double lu0 = tl0, lu1 = pl.U * tl0 + tl1;
  const double ru0 = tr0, ru1 = pr.U * tr0 - tr1;
  const double hl = 0.5 / pl.lam, hr = 0.5 / pr.lam;
  const double lu2 = pl.U * lu1 + hl * lu0, ru2 = pr.U * ru1 + hr * ru0;
  // interface equilibrium W_c = rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0}
  double Wc[NV];
  Wc[0] = pl.rho * lu0 + pr.rho * ru0;
  Wc[1] = pl.rho * lu1 + pr.rho * ru1;
  if constexpr (NV == 4) {
    Wc[2] = pl.rho * pl.V * lu0 + pr.rho * pr.V * ru0;
    Wc[3] = 0.5 * (pl.rho * (lu2 + (pl.V * pl.V + hl + K * hl) * lu0) +
                   pr.rho * (ru2 + (pr.V * pr.V + hr + K * hr) * ru0));
  } else {
    Wc[2] = 0.5 * (pl.rho * (lu2 + K * hl * lu0) + pr.rho * (ru2 + K * hr * ru0));
  }
  const Prim<NV> pc = prim<NV>(Wc, g);
  // averaged derivatives and the equilibrium time derivative
  double dn[NV], dtn[NV], Wt[NV], tmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    dn[v] = 0.5 * (nl[v] + nr[v]);
    dtn[v] = (NV == 4) ? 0.5 * (tl[v] + tr[v]) : 0.0;
  }
  jac_x<NV>(Wc, pc, dn, g, Wt);
  if constexpr (NV == 4) {
    jac_y(Wc, *reinterpret_cast<const Prim<4>*>(&pc), dtn, g, tmp);
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = -(Wt[v] + tmp[v]);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = -Wt[v];
  }
  double Fe[NV], JW[NV];
  euler_flux<NV>(Wc, pc, Fe);
  jac_x<NV>(Wc, pc, Wt, g, JW);

  const double tau = k.tc1 * dt + k.tc2 * dt * fabs(pl.p - pr.p) / (pl.p + pr.p);
  const double h = 0.5 * dt;
  if (!(tau > 0.0)) {
    // tau = 0: exact limits of the time integrals
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (want_F) F[v] += w * Fe[v];
      Ft[v] += w * JW[v];
      Wi[v] += w * (Wc[v] + h * Wt[v]);
    }
    return;
  }
  // ---- tau > 0 ----
  // time integrals over [0, d] of the weights of the solution, d = dt/2, dt
  const double xh = h / tau;
  const double eh = exp(-xh), emh = -expm1(-xh);
  const double ef = eh * eh, emf = emh * (2.0 - emh);
  const double tt = tau * tau;
  const double c1h = h - tau * emh, c1f = dt - tau * emf;
  const double c5h = 2.0 * tt - tau * (h + 2.0 * tau) * eh;
  const double c5f = 2.0 * tt - tau * (dt + 2.0 * tau) * ef;
  const double c2h = c5h - tau * h, c2f = c5f - tau * dt;
  const double c3h = 0.5 * h * h - tau * h + tt * emh, c3f = 0.5 * dt * dt - tau * dt + tt * emf;
  const double c4h = tau * emh, c4f = tau * emf;
  const double c6h = tt * emh, c6f = tt * emf;
  // least-squares-free fit F(t) = F + t dF/dt to the two integrals
  const double idt = 1.0 / dt, idt2 = 4.0 * idt * idt;
  const double f1 = (4.0 * c1h - c1f) * idt, g1 = (c1f - 2.0 * c1h) * idt2;
  const double f2 = (4.0 * c2h - c2f) * idt, g2 = (c2f - 2.0 * c2h) * idt2;
  const double f3 = (4.0 * c3h - c3f) * idt, g3 = (c3f - 2.0 * c3h) * idt2;
  const double f4 = (4.0 * c4h - c4f) * idt, g4 = (c4f - 2.0 * c4h) * idt2;
  const double f5 = (4.0 * c5h - c5f) * idt, g5 = (c5f - 2.0 * c5h) * idt2;
  const double f6 = (4.0 * c6h - c6f) * idt, g6 = (c6f - 2.0 * c6h) * idt2;
  // interface state at dt/2
  const double k1 = emh, k2 = (h + tau) * eh - tau, k3 = h - tau * emh, k4 = h + tau;

  // equilibrium part: <u (abar u + bbar v) psi>_c needs the moments of g_c
  {
    Mom<NV> mc;
    mc.u[0] = 1.0;
    mc.u[1] = pc.U;
    fill_moments<NV>(mc, pc, K);
    double wv[NV], ab[NV], X2[NV];
    const double irc = 1.0 / pc.rho;
#pragma unroll
    for (int v = 0; v < NV; ++v) wv[v] = dn[v] * irc;
    micro_slope<NV>(pc, K, wv, ab);
    mom_a<NV>(mc, ab, 2, 0, X2);
    if constexpr (NV == 4) {
      double bb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) wv[v] = dtn[v] * irc;
      micro_slope<NV>(pc, K, wv, bb);
      mom_a<NV>(mc, bb, 1, 1, tmp);
#pragma unroll
      for (int v = 0; v < NV; ++v) X2[v] += tmp[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double x2 = pc.rho * X2[v];
      if (want_F) F[v] += w * (f1 * Fe[v] + f2 * x2 + f3 * JW[v]);
      Ft[v] += w * (g1 * Fe[v] + g2 * x2 + g3 * JW[v]);
      Wi[v] += w * (k1 * Wc[v] + (k3 - k2) * Wt[v]);
    }
  }
  // non-equilibrium part, one side at a time
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const Prim<NV>& ps = side ? pr : pl;
    const double* Ws = side ? Wr : Wl;
    const double* ns = side ? nr : nl;
    const double* ts = side ? tr : tl;
    Mom<NV> ms;
    ms.u[0] = side ? ru0 : lu0;
    ms.u[1] = side ? ru1 : lu1;
    fill_moments<NV>(ms, ps, K);
    const double irs = 1.0 / ps.rho;
    double wv[NV], as[NV], bs[NV], As[NV], Ws_t[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wv[v] = ns[v] * irs;
    micro_slope<NV>(ps, K, wv, as);
    jac_x<NV>(Ws, ps, ns, g, Ws_t);
    if constexpr (NV == 4) {
#pragma unroll
      for (int v = 0; v < NV; ++v) wv[v] = ts[v] * irs;
      micro_slope<NV>(ps, K, wv, bs);
      jac_y(Ws, *reinterpret_cast<const Prim<4>*>(&ps), ts, g, tmp);
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws_t[v] = -(Ws_t[v] + tmp[v]) * irs;
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws_t[v] = -Ws_t[v] * irs;
    }
    micro_slope<NV>(ps, K, Ws_t, As);
    double U1[NV], Xs[NV], Ys[NV], P0[NV], Zs[NV], A0[NV];
    mom_psi<NV>(ms, 1, 0, 0, U1);   // <u psi>
    mom_a<NV>(ms, as, 2, 0, Xs);    // <u^2 (a.psi) psi>
    mom_a<NV>(ms, As, 1, 0, Ys);    // <u (A.psi) psi>
    mom_psi<NV>(ms, 0, 0, 0, P0);   // <psi>
    mom_a<NV>(ms, as, 1, 0, Zs);    // <u (a.psi) psi>
    mom_a<NV>(ms, As, 0, 0, A0);    // <(A.psi) psi>
    if constexpr (NV == 4) {
      mom_a<NV>(ms, bs, 1, 1, tmp);  // <u v (b.psi) psi>
#pragma unroll
      for (int v = 0; v < NV; ++v) Xs[v] += tmp[v];
      mom_a<NV>(ms, bs, 0, 1, tmp);  // <v (b.psi) psi>
#pragma unroll
      for (int v = 0; v < NV; ++v) Zs[v] += tmp[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double r = ps.rho;
      if (want_F) F[v] += w * r * (f4 * U1[v] - f5 * Xs[v] - f6 * Ys[v]);
      Ft[v] += w * r * (g4 * U1[v] - g5 * Xs[v] - g6 * Ys[v]);
      Wi[v] += w * eh * r * (P0[v] - k4 * Zs[v] - tau * A0[v]);
    }
  }
}

}  // namespace gks
