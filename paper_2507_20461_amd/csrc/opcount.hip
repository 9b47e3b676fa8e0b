// Floating-point operation counts of the device functions, obtained by
// executing the same templates on the host with a counting scalar type.
//
// Convention: every add, subtract, multiply, divide and square root counts
// one operation, and so does each call of an elementary function (exp,
// expm1, erfc, tanh); negation, absolute value, min/max and comparisons are
// not counted. The counts are those of the formulas as the kernels evaluate
// them (constants folded at compile time are not counted).
#include <hip/hip_runtime.h>

#include <cmath>

#include "geno6.h"
#include "geno6_device.hpp"
#include "geno_device.hpp"
#include "geno_gks.h"
#include "gks_device.hpp"

namespace opcount {

long long g_ops = 0;

// counting double
struct C {
  double v;
  C() : v(0.0) {}
  C(double x) : v(x) {}  // NOLINT: implicit from constants
  explicit operator double() const { return v; }
};

inline C operator+(C a, C b) { ++g_ops; return C(a.v + b.v); }
inline C operator-(C a, C b) { ++g_ops; return C(a.v - b.v); }
inline C operator*(C a, C b) { ++g_ops; return C(a.v * b.v); }
inline C operator/(C a, C b) { ++g_ops; return C(a.v / b.v); }
inline C operator-(C a) { return C(-a.v); }
inline bool operator>(C a, C b) { return a.v > b.v; }
inline bool operator<(C a, C b) { return a.v < b.v; }
inline bool operator>=(C a, C b) { return a.v >= b.v; }
inline bool operator<=(C a, C b) { return a.v <= b.v; }
inline bool operator==(C a, C b) { return a.v == b.v; }
inline C sqrt(C a) { ++g_ops; return C(std::sqrt(a.v)); }
inline C exp(C a) { ++g_ops; return C(std::exp(a.v)); }
inline C expm1(C a) { ++g_ops; return C(std::expm1(a.v)); }
inline C erfc(C a) { ++g_ops; return C(std::erfc(a.v)); }
inline C tanh(C a) { ++g_ops; return C(std::tanh(a.v)); }
inline C fabs(C a) { return C(std::fabs(a.v)); }
inline C fmax(C a, C b) { return C(std::fmax(a.v, b.v)); }
inline C fmin(C a, C b) { return C(std::fmin(a.v, b.v)); }
inline bool isfinite(C a) { return std::isfinite(a.v); }

template <typename F>
long long count(F f) {
  g_ops = 0;
  f();
  return g_ops;
}

geno::KParams params(int ndim, double gamma) {
  geno::KParams k;
  k.C = 20.0;
  k.tanhC = std::tanh(20.0);
  k.eps = 1e-15;
  k.d1 = 1.0;
  k.d2 = 8.0;
  k.d3 = 1.0;
  k.gamma = gamma;
  k.K = ndim == 1 ? (3.0 - gamma) / (gamma - 1.0) : (4.0 - 2.0 * gamma) / (gamma - 1.0);
  k.tc1 = 0.0;
  k.tc2 = 1.0;
  k.cfl = 0.5;
  k.dt_fixed = 0.0;
  k.eps_ulps = 0.0;
  k.gate_thr = 1.0;
  k.gate = 0;
  k.charvars = 0;
  return k;
}

}  // namespace opcount

int geno_op_costs_impl(int ndim, double gamma, int nkinds, int nclass, double* costs) {
  using opcount::C;
  using opcount::count;
  const geno::KParams k = opcount::params(ndim, gamma);
  for (int i = 0; i < nkinds * nclass; ++i) costs[i] = 0.0;
  auto set = [&](int kind, int cls, double v) {
    if (kind < nkinds && cls < nclass) costs[kind * nclass + cls] = v;
  };
  // normal GENO: linear part per variable and face, one side on its two branches
  const long long lin = count([&] {
    C qH, hqH;
    geno::linear_p7<C>(1.0, 1.1, 1.2, 1.3, 0.1, 0.1, 0.1, 0.1, qH, hqH);
    (void)geno::linear_p7_d2<C>(1.0, 1.1, 1.2, 1.3, 0.1, 0.1, 0.1, 0.1);
  });
  // one side, plus its half of the mean second derivative (1 add, 1 mul
  // per face: counted as one per side)
  const long long side_hi = 1 + count([&] {   // linear data: IS_tau = 0, chi = 1 without tanh
    C v, d, d2, x;
    geno::geno_side<C, C>(1.0, 1.1, 1.2, 1.3, 0.1, 1.15, 0.1, 0.0, k, v, d, d2, x);
  });
  const long long side_lo = 1 + count([&] {   // a step: chi < 1, low-order part formed
    C v, d, d2, x;
    geno::geno_side<C, C>(0.0, 0.0, 1.0, 1.0, 0.0, 0.5, 0.0, 0.0, k, v, d, d2, x);
  });
  // tangential step of one side and variable, with its second tangential
  // and cross derivatives (2 mul, 1 sub, 1 mul) and their mean over the
  // sides (1 add, 1 mul each, per side: 2)
  const long long tan_hi = 6 + count([&] {
    C v0, v1, t0, t1, ct, d2;
    geno::tangential<C, C>(1.0, 1.1, 1.2, k, v0, v1, t0, t1, ct, d2);
  });
  const long long tan_lo = 6 + count([&] {
    C v0, v1, t0, t1, ct, d2;
    geno::tangential<C, C>(0.0, 0.0, 1.0, k, v0, v1, t0, t1, ct, d2);
  });
  const int nv = ndim == 2 ? 4 : 3;
  const long long adm = count([&] {
    C w[4] = {1.0, 0.1, 0.2, 2.5};
    if (nv == 4) (void)geno::admissible<4, C>(w, gamma);
    else (void)geno::admissible<3, C>(w, gamma);
  });
  // gas-kinetic point: tau = 0 with equal states, tau = 0 with different
  // states of equal pressure (a contact; the values are exact in binary so
  // that both pressures round alike), tau > 0
  long long pequal = 0, pfast = 0, pslow = 0;
  if (ndim == 2) {
    C Wl[4] = {1.0, 0.25, -0.125, 2.5390625}, Wr[4] = {0.5, 0.125, -0.0625, 2.51953125};
    C Wr2[4] = {0.8, 0.1, 0.1, 2.0};
    C n[4] = {0.1, 0.2, 0.3, 0.4}, t[4] = {0.2, 0.1, 0.0, -0.1};
    C s1[4] = {0.3, -0.2, 0.1, 0.4}, s2[4] = {0.1, 0.1, -0.3, 0.2}, s3[4] = {-0.2, 0.3, 0.1, 0.1};
    // the point plus its share of the stage-1 outputs (Gauss weight and
    // the two interface-value combinations: 4 per variable)
    pequal = 16 + count([&] {
      gks::PointOut<4, C> o;
      gks::point_flux<4, true, C>(Wl, Wl, n, n, t, t, s1, s2, s3, C(1e-3), k, true, o);
    });
    pfast = 16 + count([&] {
      gks::PointOut<4, C> o;
      gks::point_flux<4, true, C>(Wl, Wr, n, n, t, t, s1, s2, s3, C(1e-3), k, true, o);
    });
    pslow = 16 + count([&] {
      gks::PointOut<4, C> o;
      gks::point_flux<4, true, C>(Wl, Wr2, n, n, t, t, s1, s2, s3, C(1e-3), k, true, o);
    });
  } else {
    C Wl[3] = {1.0, 0.25, 2.53125}, Wr[3] = {0.5, 0.125, 2.515625}, Wr2[3] = {0.8, 0.1, 2.0};
    C n[3] = {0.1, 0.2, 0.3}, s1[3] = {0.3, -0.2, 0.1};
    // plus the two interface-value combinations (2 per variable)
    pequal = 6 + count([&] {
      gks::PointOut<3, C> o;
      gks::point_flux<3, true, C>(Wl, Wl, n, n, nullptr, nullptr, s1, nullptr, nullptr, C(1e-3),
                                  k, true, o);
    });
    pfast = 6 + count([&] {
      gks::PointOut<3, C> o;
      gks::point_flux<3, true, C>(Wl, Wr, n, n, nullptr, nullptr, s1, nullptr, nullptr, C(1e-3),
                                  k, true, o);
    });
    pslow = 6 + count([&] {
      gks::PointOut<3, C> o;
      gks::point_flux<3, true, C>(Wl, Wr2, n, n, nullptr, nullptr, s1, nullptr, nullptr, C(1e-3),
                                  k, true, o);
    });
  }
  if (ndim == 2) {
    // face-row entry of one variable: h*gradient scaling (4), linear part,
    // two sides
    const double row = 4 + lin + 2 * side_hi;
    for (int kind : {GENO_K_NORMAL_X, GENO_K_NORMAL_Y}) {
      set(kind, GENO_W_UNITS, row);
      set(kind, GENO_W_LOW, (double)(side_lo - side_hi));
      // a gated side skips its indicators (work counted with the unit)
      set(kind, GENO_W_GATED, -(double)side_hi);
    }
    // face: 8 tangential steps, 4 guard checks, derivative scaling (per
    // point: 16 first and 12 second derivatives) and the Gauss average of
    // 16 outputs (a weight and an addition each)
    const double face = 8.0 * tan_hi + 4.0 * adm + 2.0 * 28.0 + 32.0;
    for (int kind : {GENO_K_FACES_X, GENO_K_FACES_Y, GENO_K_SLOW}) {
      set(kind, GENO_W_UNITS, face);
      set(kind, GENO_W_LOW, (double)(tan_lo - tan_hi));
      set(kind, GENO_W_EQUAL, (double)pequal);
      set(kind, GENO_W_FAST, (double)pfast);
      set(kind, GENO_W_SLOW, (double)pslow);
    }
    // update per cell and variable: stage 1 L (5), L_t (5), gradients at the
    // stage time (4), W* (7), R (6); stage 2 L_t (5), gradients of W_tt* (4)
    // and of the stage-1 end-of-step values (4), their combination (4), W
    // (2), and per cell dt^2/3 (2) and the CFL bound (17)
    set(GENO_K_UPDATE_1, GENO_W_UNITS, 4.0 * 27.0);
    set(GENO_K_UPDATE_2, GENO_W_UNITS, 4.0 * 19.0 + 19.0);
    set(GENO_K_INIT, GENO_W_UNITS, 17.0);
  } else {
    const double face = 3.0 * (4 + lin + 2 * side_hi) + 2.0 * adm + 6.0;
    set(GENO_K_FACES_1D, GENO_W_UNITS, face);
    set(GENO_K_FACES_1D, GENO_W_LOW, (double)(side_lo - side_hi));
    set(GENO_K_FACES_1D, GENO_W_EQUAL, (double)pequal);
    set(GENO_K_FACES_1D, GENO_W_FAST, (double)pfast);
    set(GENO_K_FACES_1D, GENO_W_SLOW, (double)pslow);
    set(GENO_K_UPDATE_1, GENO_W_UNITS, 3.0 * 19.0);
    set(GENO_K_UPDATE_2, GENO_W_UNITS, 3.0 * 10.0 + 13.0);
    set(GENO_K_INIT, GENO_W_UNITS, 11.0);
  }
  return 0;
}

// Sixth-order non-compact scheme: a face with linear data (every side keeps
// chi = 1 without the exponential or the low-order part), the extra work of
// one side whose chi < 1, and the per-cell flux difference and stage update
// (2 per variable for L, on average 5 per variable for the four stage
// combinations, and the wave speed of the last stage, 9 operations, once in
// four stages: 3 * 7 + 2 = 23).
extern "C" int geno6_op_costs(double* costs) {
  using opcount::C;
  using opcount::count;
  if (!costs) return GENO_EINVAL;
  geno6::KP6 k;
  k.gamma = 1.4;
  k.C = 20.0;
  k.inv_tanhC = 1.0 / std::tanh(20.0);
  k.t2_cut = 2.0 * (1.0 - 19.8 / 20.0) / (19.8 / 20.0);
  k.eps = 1e-15;
  k.d[0] = 1.0;
  k.d[1] = 8.0;
  k.d[2] = 1.0;
  k.d[3] = 1.0;
  k.cfl = 0.5;
  k.dt_fixed = 0.0;
  k.characteristic = 0;
  // linear data of an admissible subsonic state (rho, rho u, rho E)
  const long long face_lin = count([&] {
    C u[3][6], WL[3], WR[3], F[3];
    for (int m = 0; m < 6; ++m) {
      u[0][m] = 1.0 + 0.01 * m;
      u[1][m] = 0.1 + 0.01 * m;
      u[2][m] = 2.5 + 0.01 * m;
    }
    const auto get = [&](int v, int m) { return u[v][m]; };
    (void)geno6::face6<C, false>(get, k, WL, WR, F, nullptr);
  });
  geno6::Cand<C> cl, cr, sl, sr;
  C p5, p3;
  const C lin[6] = {1.0, 1.1, 1.2, 1.3, 1.4, 1.5}, step[6] = {1.0, 1.0, 1.0, 5.0, 5.0, 5.0};
  geno6::candidates<C>(lin, cl, cr, p5, p3);
  geno6::candidates<C>(step, sl, sr, p5, p3);
  const long long side_lin = count([&] {
    C x;
    (void)geno6::side6<C>(cl, C(1.25), C(1.25), k, x);
  });
  const long long side_low = count([&] {
    C x;
    (void)geno6::side6<C>(sl, C(3.0), C(3.0), k, x);
  });
  costs[0] = (double)face_lin;
  costs[1] = (double)(side_low - side_lin);
  costs[2] = 23.0;
  return GENO_OK;
}
