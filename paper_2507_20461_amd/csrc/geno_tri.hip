// Fourth-order compact GENO reconstruction on triangular meshes (Sec. 4.3
// with Sec. 3): the mesh layer that turns the geometry into per-cell
// operator tables (host, once per mesh), and the reconstruction kernel.
//
// Everything about the polynomials is expressed in the scaled coordinates
// xi = (x - x_j)/h, eta = (y - y_j)/h of the target cell (h^2 = |Omega_j|),
// with the cubic candidate written as
//   p^3 = Q_j + sum_alpha a_alpha (phi_alpha - m_alpha),
// phi_alpha the nine monomials xi^a eta^b of degree 1..3 in the order
// (1,0) (0,1) (2,0) (1,1) (0,2) (3,0) (2,1) (1,2) (0,3), m_alpha their
// averages on Omega_j (so the cell average is exact). In these coordinates
// h^{2|l|-2} int (D^l p)^2 dx = mean over Omega_j of (d^l p / d xi^l)^2, so
//   IS~^H = mean over Omega_j of the squared first and second derivatives
//           (Dunavant's degree-4 rule on the cell, exact for them),
//   IS^tau = 36 a_30^2 + 4 a_21^2 + 4 a_12^2 + 36 a_03^2 (third derivatives
//            of a cubic are constants),  IS^H = IS~^H + IS^tau,
// and for p_k = Q_j + b_k . (xi, eta): IS_k = |b_k|^2. The kernel forms the
// means m_alpha with the same rule; the table holds what depends on the
// neighbours (stencil, least-squares operators) and the scaled vertices.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "geno_tri.h"
#include "gks_device.hpp"

namespace geno_err {
int fail(int code, const char* fmt, ...);
}

namespace {

using geno_err::fail;

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(GENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int NA = 9;        // coefficients of the cubic candidate
constexpr int ND = 17;       // entries of its data vector
// Table entries per cell, stored in pairs: entries 2p and 2p+1 of cell c
// are the two doubles of pair p at pair index p * n + c (16-byte aligned),
// so that one 16-byte load per lane brings two entries and a wave's load
// spans 64 consecutive cells. Every region starts on an even entry.
constexpr int E_IDX = 0;                  // 9 stencil cells (3 edge neighbours, 6 second level)
constexpr int E_H = 9;                    // h
constexpr int NAP = NA + 1;               // operator column padded to pairs
constexpr int E_M = 10;                   // least-squares operator [ND][NAP] (column i of P, padded)
constexpr int E_L = E_M + ND * NAP;       // linear candidates [3][2][3]
constexpr int E_V = E_L + 18;             // scaled vertices (xi, eta) x 3
// geometry of the flux and update: area, d = 4 area / perimeter, then per
// edge e (vertex e to e+1): outward unit normal (2), length, neighbour, the
// neighbour's index of the same edge, 1 if this cell owns the edge (the
// smaller (cell, edge) pair of its two sides) else 0
constexpr int E_G = E_V + 6;
constexpr int E_GE = E_G + 2;             // per-edge block of 6
// the owned (cell, edge) pairs as codes 3 cell + edge, edge-major (all owned
// edges 0 by cell, then edges 1, then 2), in list slots k = 0 .. 2n - 1 at
// entry E_OWN + k / n of cell slot k % n; unused slots -1 (a periodic mesh
// of n cells has 3n/2 edges)
constexpr int E_OWN = E_GE + 18;
constexpr int E_N = E_OWN + 2;
static_assert(E_M % 2 == 0 && E_L % 2 == 0 && E_V % 2 == 0 && E_G % 2 == 0 && E_OWN % 2 == 0 &&
                  E_N % 2 == 0,
              "table regions start on pairs");

// host index of entry e of cell c in a table of n cells
inline size_t tab_index(int e, size_t c, size_t n) { return ((size_t)(e >> 1) * n + c) * 2 + (e & 1); }


// averages over a triangle of the nine monomials and of
// their xi- and eta-derivatives, all at once, by the rule exact for degree
// <= 3 (vertices 1/20, edge midpoints 2/15, centroid 9/20)
void tri_avgs(const double (&t)[3][2], double (&m)[NA], double (&mx)[NA], double (&my)[NA]) {
  double P[7][2], Wq[7];
  for (int v = 0; v < 3; ++v) {
    const int w = (v + 1) % 3;
    P[v][0] = t[v][0];
    P[v][1] = t[v][1];
    Wq[v] = 1.0 / 20.0;
    P[3 + v][0] = 0.5 * (t[v][0] + t[w][0]);
    P[3 + v][1] = 0.5 * (t[v][1] + t[w][1]);
    Wq[3 + v] = 2.0 / 15.0;
  }
  P[6][0] = (t[0][0] + t[1][0] + t[2][0]) / 3.0;
  P[6][1] = (t[0][1] + t[1][1] + t[2][1]) / 3.0;
  Wq[6] = 9.0 / 20.0;
  for (int q = 0; q < NA; ++q) m[q] = mx[q] = my[q] = 0.0;
  for (int g = 0; g < 7; ++g) {
    const double x = P[g][0], y = P[g][1], xx = x * x, xy = x * y, yy = y * y;
    const double ph[NA] = {x, y, xx, xy, yy, xx * x, xx * y, x * yy, yy * y};
    const double px[NA] = {1.0, 0.0, 2.0 * x, y, 0.0, 3.0 * xx, 2.0 * xy, yy, 0.0};
    const double py[NA] = {0.0, 1.0, 0.0, x, 2.0 * y, 0.0, xx, 2.0 * xy, 3.0 * yy};
    for (int q = 0; q < NA; ++q) {
      m[q] += Wq[g] * ph[q];
      mx[q] += Wq[g] * px[q];
      my[q] += Wq[g] * py[q];
    }
  }
}

// Least-squares operator P = A^+ (NA x ND) of the ND x NA matrix A (full
// column rank) by Householder QR: A = Q R, P = R^-1 Q^T. Returns false if a
// diagonal of R is below 1e-12 of the largest.
bool pinv(const double (&A)[ND][NA], double (&P)[NA][ND]) {
  double R[ND][NA], Qt[ND][ND];
  std::memcpy(R, A, sizeof R);
  for (int i = 0; i < ND; ++i)
    for (int j = 0; j < ND; ++j) Qt[i][j] = i == j ? 1.0 : 0.0;
  for (int k = 0; k < NA; ++k) {
    double nrm = 0.0;
    for (int i = k; i < ND; ++i) nrm += R[i][k] * R[i][k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = R[k][k] > 0.0 ? -nrm : nrm;
    double v[ND] = {};
    for (int i = k; i < ND; ++i) v[i] = R[i][k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < ND; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = 0; j < NA; ++j) {
      double s = 0.0;
      for (int i = k; i < ND; ++i) s += v[i] * R[i][j];
      s = 2.0 * s / vv;
      for (int i = k; i < ND; ++i) R[i][j] -= s * v[i];
    }
    for (int j = 0; j < ND; ++j) {
      double s = 0.0;
      for (int i = k; i < ND; ++i) s += v[i] * Qt[i][j];
      s = 2.0 * s / vv;
      for (int i = k; i < ND; ++i) Qt[i][j] -= s * v[i];
    }
  }
  double rmax = 0.0;
  for (int k = 0; k < NA; ++k) rmax = std::fmax(rmax, std::fabs(R[k][k]));
  for (int k = 0; k < NA; ++k)
    if (!(std::fabs(R[k][k]) > 1e-12 * rmax)) return false;
  // back substitution R[0:NA, :] X = Qt[0:NA, :]
  for (int j = 0; j < ND; ++j)
    for (int k = NA - 1; k >= 0; --k) {
      double s = Qt[k][j];
      for (int q = k + 1; q < NA; ++q) s -= R[k][q] * P[q][j];
      P[k][j] = s / R[k][k];
    }
  return true;
}

struct TriK {
  double C, inv_tanhC, eps, d[3];
};

// One wave per variable over 64 consecutive cells: a work-group of NV waves
// covers 64 cells, its waves read the same table lines (the repeats hit the
// caches) and every load and store of a wave spans 64 consecutive cells.
// Per lane: the cubic's coefficients from the 17 data entries, the
// indicators, the path function, the ENO weights and the blended states at
// the six edge Gauss points.
template <int NV>
__global__ void __launch_bounds__(256) k_tri(int n, const double* __restrict__ ops,
                                             const double* __restrict__ W,
                                             const double* __restrict__ dW,
                                             double* __restrict__ out, double* __restrict__ chi,
                                             double* __restrict__ sec, TriK k) {
  const int v = (int)(threadIdx.x >> 6);
  const int c = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
  if (c >= n) return;
  const size_t sn = (size_t)n;
  const double2* op2 = reinterpret_cast<const double2*>(ops) + c;
  // entries [e0, e0 + 2 np) of this cell, np pair loads
  auto region = [&](int e0, int np, double* r) {
#pragma unroll
    for (int p = 0; p < np; ++p) {
      const double2 x = op2[(size_t)((e0 >> 1) + p) * sn];
      r[2 * p] = x.x;
      r[2 * p + 1] = x.y;
    }
  };
  double ih[10];
  region(E_IDX, 5, ih);
  int idx[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) idx[i] = (int)ih[i];
  const double h = ih[E_H];
  const double wc = W[v * sn + c];
  // entry i of the data vector
  auto data = [&](int i) -> double {
    if (i < 9) return W[v * sn + idx[i]] - wc;
    if (i < 11) return h * dW[((i - 9) * NV + v) * sn + c];
    const int kk = (i - 11) >> 1, dir = (i - 11) & 1;
    return h * dW[(dir * NV + v) * sn + idx[kk]];
  };
  double av[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) av[q] = 0.0;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const double d = data(i);
    {
      double m[NAP];
      region(E_M + i * NAP, NAP / 2, m);
#pragma unroll
      for (int q = 0; q < NA; ++q) av[q] = fma(m[q], d, av[q]);
    }
  }
  const double IStau = 36.0 * av[5] * av[5] + 4.0 * av[6] * av[6] + 4.0 * av[7] * av[7] +
                       36.0 * av[8] * av[8];
  double vv[6], vx[3], vy[3], mean[NA];
  region(E_V, 3, vv);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    vx[r] = vv[2 * r];
    vy[r] = vv[2 * r + 1];
  }
  // means of the monomials and IS~^H by Dunavant's degree-4 rule on the cell
  double Q = 0.0;
#pragma unroll
  for (int q = 0; q < NA; ++q) mean[q] = 0.0;
  {
    const double A2[2] = {0.445948490915965, 0.091576213509771};
    const double W2[2] = {0.223381589678011, 0.109951743655322};
#pragma unroll
    for (int gq = 0; gq < 2; ++gq)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double b0 = r == 0 ? 1.0 - 2.0 * A2[gq] : A2[gq];
        const double b1 = r == 1 ? 1.0 - 2.0 * A2[gq] : A2[gq];
        const double b2 = r == 2 ? 1.0 - 2.0 * A2[gq] : A2[gq];
        const double X = b0 * vx[0] + b1 * vx[1] + b2 * vx[2], Y = b0 * vy[0] + b1 * vy[1] + b2 * vy[2];
        const double XX = X * X, XY = X * Y, YY = Y * Y, w = W2[gq];
        const double ph[NA] = {X, Y, XX, XY, YY, XX * X, XX * Y, X * YY, YY * Y};
#pragma unroll
        for (int q = 0; q < NA; ++q) mean[q] = fma(w, ph[q], mean[q]);
        const double dx = av[0] + 2.0 * av[2] * X + av[3] * Y + 3.0 * av[5] * XX + 2.0 * av[6] * XY + av[7] * YY;
        const double dy = av[1] + av[3] * X + 2.0 * av[4] * Y + av[6] * XX + 2.0 * av[7] * XY + 3.0 * av[8] * YY;
        const double dxx = 2.0 * av[2] + 6.0 * av[5] * X + 2.0 * av[6] * Y;
        const double dxy = av[3] + 2.0 * av[6] * X + 2.0 * av[7] * Y;
        const double dyy = 2.0 * av[4] + 2.0 * av[7] * X + 6.0 * av[8] * Y;
        Q = fma(w, dx * dx + dy * dy + dxx * dxx + dxy * dxy + dyy * dyy, Q);
      }
  }
  double Lk[18];
  region(E_L, 9, Lk);
  const double ISH = Q + IStau;
  double b[3][2], IS[3];
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const double e0 = data(kk), e1 = data(11 + 2 * kk), e2 = data(12 + 2 * kk);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int o = (kk * 2 + r) * 3;
      b[kk][r] = Lk[o] * e0 + Lk[o + 1] * e1 + Lk[o + 2] * e2;
    }
    IS[kk] = b[kk][0] * b[kk][0] + b[kk][1] * b[kk][1];
  }
  const double ISL = IS[0] + IS[1] + IS[2] - fmin(IS[0], fmin(IS[1], IS[2])) -
                     fmax(IS[0], fmax(IS[1], IS[2]));
  const double xH = IStau / (ISH + k.eps), xL = IStau / (ISL + k.eps);
  const double aH = 1.0 + xH * xH * xH, aL = 1.0 + xL * xL * xL;
  const double alpha = 2.0 * aH / (aH + aL);
  const double x = tanh(k.C * alpha) * k.inv_tanhC;
  double w[3], ws = 0.0;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const double e = IS[kk] + k.eps;
    w[kk] = k.d[kk] / (e * e);
    ws += w[kk];
  }
  const double iw = 1.0 / ws;
  double gLx = 0.0, gLy = 0.0;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    w[kk] *= iw;
    gLx = fma(w[kk], b[kk][0], gLx);
    gLy = fma(w[kk], b[kk][1], gLy);
  }
  if (chi) chi[v * sn + c] = x;
  const double xm = 1.0 - x;

  const double t0 = 0.5 - 0.5 / 1.7320508075688772935, t1 = 0.5 + 0.5 / 1.7320508075688772935;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int e1 = (e + 1) % 3;
#pragma unroll
    for (int gp = 0; gp < 2; ++gp) {
      const double tt = gp == 0 ? t0 : t1;
      const double X = vx[e] + tt * (vx[e1] - vx[e]), Y = vy[e] + tt * (vy[e1] - vy[e]);
      const double XX = X * X, XY = X * Y, YY = Y * Y;
      const double ph[NA] = {X, Y, XX, XY, YY, XX * X, XX * Y, X * YY, YY * Y};
      const double px[NA] = {1.0, 0.0, 2.0 * X, Y, 0.0, 3.0 * XX, 2.0 * XY, YY, 0.0};
      const double py[NA] = {0.0, 1.0, 0.0, X, 2.0 * Y, 0.0, XX, 2.0 * XY, 3.0 * YY};
      double p3 = wc, p3x = 0.0, p3y = 0.0;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        p3 = fma(av[q], ph[q] - mean[q], p3);
        p3x = fma(av[q], px[q], p3x);
        p3y = fma(av[q], py[q], p3y);
      }
      double pL = wc;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) pL = fma(w[kk], b[kk][0] * X + b[kk][1] * Y, pL);
      const int pt = 2 * e + gp;
      out[((pt * 3 + 0) * NV + v) * sn + c] = x * p3 + xm * pL;
      out[((pt * 3 + 1) * NV + v) * sn + c] = x * p3x + xm * gLx;
      out[((pt * 3 + 2) * NV + v) * sn + c] = x * p3y + xm * gLy;
      if (sec) {
        // h^2 d2/dx2, d2/dxdy, d2/dy2 of the blend: chi times the cubic's
        // (in the scaled coordinates; the linear candidates have none)
        sec[((pt * 3 + 0) * NV + v) * sn + c] = x * (2.0 * av[2] + 6.0 * av[5] * X + 2.0 * av[6] * Y);
        sec[((pt * 3 + 1) * NV + v) * sn + c] = x * (av[3] + 2.0 * av[6] * X + 2.0 * av[7] * Y);
        sec[((pt * 3 + 2) * NV + v) * sn + c] = x * (2.0 * av[4] + 2.0 * av[7] * X + 6.0 * av[8] * Y);
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Compact GKS step on the mesh (Sec. 4.3 with Eq. (1)-(2)), conserved
// variables (rho, rho u, rho v, rho E), [4][n] averages and [2][4][n]
// averaged gradients. Per stage: the reconstruction above (values, gradients
// and second derivatives at the edge Gauss points), the edge kernel (one
// thread per owned edge: both Gauss points' gas-kinetic solutions in the
// frame of the owner's outward normal, rotated back and averaged) and the
// cell kernel (Eq. (1) and the Gauss-theorem gradients of Eq. (2) over the
// three edges, the two-stage fourth-order combination).
// ---------------------------------------------------------------------------
struct TriCtrl {
  double dt;
  unsigned long long guard;
  unsigned long long nonfinite;
};

// entry e of cell c of the table
__device__ __forceinline__ double tab_at(const double* __restrict__ ops, int e, int c, size_t n) {
  return ops[((size_t)(e >> 1) * n + (size_t)c) * 2 + (e & 1)];
}

// momentum components of a per-variable vector into the frame (n, t),
// t = (-n_y, n_x), and back
__device__ __forceinline__ void to_frame(double* q, double nx, double ny) {
  const double a = q[1] * nx + q[2] * ny, b = -q[1] * ny + q[2] * nx;
  q[1] = a;
  q[2] = b;
}
__device__ __forceinline__ void from_frame(double* q, double nx, double ny) {
  const double a = q[1] * nx - q[2] * ny, b = q[1] * ny + q[2] * nx;
  q[1] = a;
  q[2] = b;
}

// local dt bound of a cell: d / (|u| + c)
__device__ __forceinline__ double tri_tmin(const double* w, double d, double gamma) {
  const double rho = w[0], u = w[1] / rho, v = w[2] / rho;
  const double p = (gamma - 1.0) * (w[3] - 0.5 * rho * (u * u + v * v));
  const double t = d / (sqrt(u * u + v * v) + sqrt(gamma * p / rho));
  return t > 0.0 ? t : 0.0;
}

__device__ __forceinline__ void tri_block_min(double t, double* part) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t = fmin(t, __shfl_xor(t, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// start of a call: cleared counters and the CFL partials of the state
__global__ void __launch_bounds__(256) k_tri_init(int n, const double* __restrict__ ops,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ part, TriCtrl* ctrl,
                                                  double gamma) {
  const int c = (int)(blockIdx.x * 256 + threadIdx.x);
  if (c == 0) {
    ctrl->guard = 0;
    ctrl->nonfinite = 0;
  }
  double t = INFINITY;
  if (c < n) {
    double w[4];
    for (int v = 0; v < 4; ++v) w[v] = W[(size_t)v * n + c];
    t = tri_tmin(w, tab_at(ops, E_G + 1, c, (size_t)n), gamma);
  }
  tri_block_min(t, part);
}

// dt of the step (one work-group): CFL times the minimum partial, or the
// fixed step
__global__ void __launch_bounds__(256) k_tri_dt(const double* __restrict__ part, int npart,
                                                TriCtrl* ctrl, double cfl, double dt_fixed,
                                                double* dt_out, int step) {
  double m = INFINITY;
  for (int q = (int)threadIdx.x; q < npart; q += 256) m = fmin(m, part[q]);
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * m;
    ctrl->dt = dt;
    if (dt_out) dt_out[step] = dt;
  }
}

// One thread per slot t of the owned-edge list (each edge once, edge-major,
// so that no lane idles on an edge its cell does not own; slots past the
// list's end return). Output [kind][var][edge][cell] at the owner's slot, xy
// frame, Gauss-averaged: stage 1 F, dF/dt, W(dt/2) + dt^2/8 phi W_tt,
// W(dt) + dt^2/6 phi W_tt; stage 2 kinds 1 (dF/dt) and 2 (phi W_tt). Every
// point takes the full solution: the two sides of a triangle edge come from
// two cells' own reconstructions, so their pressures differ and tau > 0
// almost everywhere (a tau = 0 pass with a queue of the rest measured 21 %
// slower).
template <int STAGE>
__global__ void __launch_bounds__(256) k_tri_edges(int n, const double* __restrict__ ops,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ rec,
                                                   const double* __restrict__ sec,
                                                   double* __restrict__ ebuf, TriCtrl* ctrl,
                                                   geno::KParams k) {
  const int t = (int)(blockIdx.x * 256 + threadIdx.x);
  if (t >= 2 * n) return;
  const size_t sn = (size_t)n;
  const int code = (int)tab_at(ops, E_OWN + t / n, t % n, sn);
  if (code < 0) return;
  const int c = code / 3, e = code - 3 * (code / 3);
  const int g0 = E_GE + 6 * e;
  const double nx = tab_at(ops, g0, c, sn), ny = tab_at(ops, g0 + 1, c, sn);
  const double tx = -ny, ty = nx;
  const int m = (int)tab_at(ops, g0 + 3, c, sn), f = (int)tab_at(ops, g0 + 4, c, sn);
  const double hs[2] = {tab_at(ops, E_H, c, sn), tab_at(ops, E_H, m, sn)};
  const int cells[2] = {c, m};
  const double dt = ctrl->dt;
  double acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[q][v] = 0.0;
  unsigned int nguard = 0;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    double S[2][4], Dn[2][4], Dt[2][4], Snn[2][4], Snt[2][4], Stt[2][4];
    bool ok[2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int cell = cells[sd];
      const int pt = sd == 0 ? 2 * e + g : 2 * f + (1 - g);
      const double ih = 1.0 / hs[sd], ih2 = ih * ih;
      double gx[4], gy[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        S[sd][v] = rec[((size_t)(pt * 3 + 0) * 4 + v) * sn + cell];
        gx[v] = rec[((size_t)(pt * 3 + 1) * 4 + v) * sn + cell] * ih;
        gy[v] = rec[((size_t)(pt * 3 + 2) * 4 + v) * sn + cell] * ih;
        const double xx = sec[((size_t)(pt * 3 + 0) * 4 + v) * sn + cell] * ih2;
        const double xy = sec[((size_t)(pt * 3 + 1) * 4 + v) * sn + cell] * ih2;
        const double yy = sec[((size_t)(pt * 3 + 2) * 4 + v) * sn + cell] * ih2;
        Snn[sd][v] = xx * nx * nx + 2.0 * xy * nx * ny + yy * ny * ny;
        Snt[sd][v] = xx * nx * tx + xy * (nx * ty + ny * tx) + yy * ny * ty;
        Stt[sd][v] = xx * tx * tx + 2.0 * xy * tx * ty + yy * ty * ty;
      }
      ok[sd] = geno::admissible<4, double>(S[sd], k.gamma);
      if (!ok[sd]) {
        ++nguard;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          S[sd][v] = W[(size_t)v * sn + cell];
          gx[v] = gy[v] = 0.0;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Dn[sd][v] = gx[v] * nx + gy[v] * ny;
        Dt[sd][v] = gx[v] * tx + gy[v] * ty;
      }
      to_frame(S[sd], nx, ny);
      to_frame(Dn[sd], nx, ny);
      to_frame(Dt[sd], nx, ny);
      to_frame(Snn[sd], nx, ny);
      to_frame(Snt[sd], nx, ny);
      to_frame(Stt[sd], nx, ny);
    }
    double mnn[4], mnt[4], mtt[4];
    const bool both = ok[0] && ok[1];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      mnn[v] = both ? 0.5 * (Snn[0][v] + Snn[1][v]) : 0.0;
      mnt[v] = both ? 0.5 * (Snt[0][v] + Snt[1][v]) : 0.0;
      mtt[v] = both ? 0.5 * (Stt[0][v] + Stt[1][v]) : 0.0;
    }
    gks::PointOut<4, double> po;
    gks::point_flux<4, true, double>(S[0], S[1], Dn[0], Dn[1], Dt[0], Dt[1], mnn, mnt, mtt, dt, k,
                                     STAGE == 1, po);
    double q0[4], q1[4], q2[4], q3[4];
    const double c8 = dt * dt / 8.0, c6 = dt * dt / 6.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (STAGE == 1) {
        q0[v] = po.F[v];
        q2[v] = po.Wh[v] + c8 * po.Wtt[v];
        q3[v] = po.Wf[v] + c6 * po.Wtt[v];
      } else {
        q0[v] = q3[v] = 0.0;
        q2[v] = po.Wtt[v];
      }
      q1[v] = po.Ft[v];
    }
    from_frame(q0, nx, ny);
    from_frame(q1, nx, ny);
    from_frame(q2, nx, ny);
    from_frame(q3, nx, ny);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc[0][v] += 0.5 * q0[v];
      acc[1][v] += 0.5 * q1[v];
      acc[2][v] += 0.5 * q2[v];
      acc[3][v] += 0.5 * q3[v];
    }
  }
  if (nguard) atomicAdd(&ctrl->guard, (unsigned long long)nguard);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (STAGE == 2 && (q == 0 || q == 3)) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) ebuf[((size_t)(q * 4 + v) * 3 + e) * sn + c] = acc[q][v];
  }
}

// One thread per cell: Eq. (1) and the Gauss-theorem gradients over the three
// edges (an edge the cell does not own: the owner's F with a minus sign; the
// interface values as they are, with the cell's own outward normal), then the
// two-stage combination. Stage 2 also records non-physical cells and the CFL
// partials of the new state.
template <int STAGE>
__global__ void __launch_bounds__(256) k_tri_update(int n, const double* __restrict__ ops,
                                                    const double* __restrict__ Win,
                                                    double* __restrict__ Wout,
                                                    double* __restrict__ dWout,
                                                    double* __restrict__ R,
                                                    double* __restrict__ RG,
                                                    const double* __restrict__ ebuf,
                                                    TriCtrl* ctrl, double* __restrict__ part,
                                                    double gamma) {
  const int c = (int)(blockIdx.x * 256 + threadIdx.x);
  const size_t sn = (size_t)n;
  double tmin = INFINITY;
  if (c < n) {
    const double dt = ctrl->dt;
    double L[4] = {0, 0, 0, 0}, Lt[4] = {0, 0, 0, 0};
    double Ga[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, Gb[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int g0 = E_GE + 6 * e;
      const double nx = tab_at(ops, g0, c, sn), ny = tab_at(ops, g0 + 1, c, sn);
      const double len = tab_at(ops, g0 + 2, c, sn);
      const bool own = tab_at(ops, g0 + 5, c, sn) != 0.0;
      const int sc = own ? c : (int)tab_at(ops, g0 + 3, c, sn);
      const int se = own ? e : (int)tab_at(ops, g0 + 4, c, sn);
      const double sg = own ? 1.0 : -1.0;
      auto E = [&](int q, int v) { return ebuf[((size_t)(q * 4 + v) * 3 + se) * sn + sc]; };
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (STAGE == 1) L[v] -= sg * len * E(0, v);
        Lt[v] -= sg * len * E(1, v);
        const double wa = len * E(2, v);
        Ga[0][v] += wa * nx;
        Ga[1][v] += wa * ny;
        if (STAGE == 1) {
          const double wb = len * E(3, v);
          Gb[0][v] += wb * nx;
          Gb[1][v] += wb * ny;
        }
      }
    }
    const double ia = 1.0 / tab_at(ops, E_G, c, sn);
    double w[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t o = (size_t)v * sn + c;
      if (STAGE == 1) {
        const double l = L[v] * ia, lt = Lt[v] * ia, w0 = Win[o];
        Wout[o] = w0 + 0.5 * dt * l + dt * dt / 8.0 * lt;
        R[o] = w0 + dt * l + dt * dt / 6.0 * lt;
        dWout[o] = Ga[0][v] * ia;
        dWout[(size_t)(4 + v) * sn + c] = Ga[1][v] * ia;
        RG[o] = Gb[0][v] * ia;
        RG[(size_t)(4 + v) * sn + c] = Gb[1][v] * ia;
      } else {
        const double c3 = dt * dt / 3.0;
        w[v] = R[o] + c3 * (Lt[v] * ia);
        Wout[o] = w[v];
        dWout[o] = RG[o] + c3 * (Ga[0][v] * ia);
        dWout[(size_t)(4 + v) * sn + c] = RG[(size_t)(4 + v) * sn + c] + c3 * (Ga[1][v] * ia);
      }
    }
    if (STAGE == 2) {
      bool bad = false;
#pragma unroll
      for (int v = 0; v < 4; ++v) bad |= !isfinite(w[v]);
      bad |= !(w[0] > 0.0) || !(w[0] * w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) > 0.0);
      if (bad) atomicAdd(&ctrl->nonfinite, 1ull);
      tmin = tri_tmin(w, tab_at(ops, E_G + 1, c, sn), gamma);
    }
  }
  if (STAGE == 2) tri_block_min(tmin, part);
}
// workspace of geno_tri_step, in doubles: control block, CFL partials,
// reconstruction (values and gradients, second derivatives), edge results,
// stage state W*, grad W*, R and RG
struct TriWs {
  size_t ctrl, part, rec, sec, ebuf, wst, dwst, r, rg, total;
};
TriWs tri_ws(size_t n) {
  TriWs L{};
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t o = off;
    off += (doubles + 31) & ~(size_t)31;   // 256-byte aligned parts
    return o;
  };
  L.ctrl = take(4);
  L.part = take(n / 256 + 1);
  L.rec = take(72 * n);
  L.sec = take(72 * n);
  L.ebuf = take(48 * n);
  L.wst = take(4 * n);
  L.dwst = take(8 * n);
  L.r = take(4 * n);
  L.rg = take(8 * n);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

size_t geno_tri_table_doubles(void) { return (size_t)E_N; }

int geno_tri_build(int ncell, const double* xv, const int* nbr, const double* shift, double* ops) {
  if (ncell < 1 || !xv || !nbr || !shift || !ops) return fail(GENO_EINVAL, "bad mesh arguments");
  const size_t n = (size_t)ncell;
  for (size_t c = 0; c < n; ++c)
    for (int e = 0; e < 3; ++e)
      if (nbr[3 * c + e] < 0 || nbr[3 * c + e] >= ncell)
        return fail(GENO_EINVAL, "cell %zu: neighbour %d out of range", c, nbr[3 * c + e]);
  auto vert = [&](size_t c, int v, int d) { return xv[(c * 3 + v) * 2 + d]; };
  auto area_of = [&](size_t c) {
    return 0.5 * ((vert(c, 1, 0) - vert(c, 0, 0)) * (vert(c, 2, 1) - vert(c, 0, 1)) -
                  (vert(c, 2, 0) - vert(c, 0, 0)) * (vert(c, 1, 1) - vert(c, 0, 1)));
  };
  for (size_t c = 0; c < n; ++c) {
    const double area = area_of(c);
    if (!(area > 0.0)) return fail(GENO_EINVAL, "cell %zu is degenerate or clockwise", c);
    const double h = std::sqrt(area);
    const double xc = (vert(c, 0, 0) + vert(c, 1, 0) + vert(c, 2, 0)) / 3.0;
    const double yc = (vert(c, 0, 1) + vert(c, 1, 1) + vert(c, 2, 1)) / 3.0;
    // stencil: edge neighbours, then their neighbours other than c itself
    int cell[9];
    double tr[9][2];
    int ns = 3;
    for (int e = 0; e < 3; ++e) {
      cell[e] = nbr[3 * c + e];
      tr[e][0] = shift[(c * 3 + e) * 2];
      tr[e][1] = shift[(c * 3 + e) * 2 + 1];
    }
    for (int e = 0; e < 3; ++e) {
      const size_t d = (size_t)cell[e];
      for (int f = 0; f < 3; ++f) {
        const int q = nbr[3 * d + f];
        const double sx = tr[e][0] + shift[(d * 3 + f) * 2], sy = tr[e][1] + shift[(d * 3 + f) * 2 + 1];
        if ((size_t)q == c && sx == 0.0 && sy == 0.0) continue;
        if (ns == 9) return fail(GENO_EINVAL, "cell %zu: more than six second-level cells", c);
        cell[ns] = q;
        tr[ns][0] = sx;
        tr[ns][1] = sy;
        ++ns;
      }
    }
    if (ns != 9) return fail(GENO_EINVAL, "cell %zu: %d second-level cells, not six", c, ns - 3);
    // scaled triangle of a stencil cell (translated), about x_c
    auto scaled = [&](size_t d, double sx, double sy, double (&t)[3][2]) {
      for (int v = 0; v < 3; ++v) {
        t[v][0] = (vert(d, v, 0) + sx - xc) / h;
        t[v][1] = (vert(d, v, 1) + sy - yc) / h;
      }
    };
    double own[3][2];
    scaled(c, 0.0, 0.0, own);
    double mean[NA], mx[NA], my[NA];
    tri_avgs(own, mean, mx, my);
    double A[ND][NA];
    // h-scaled gradient rows: own cell (entries 9, 10), edge neighbour k (11 + 2k, 12 + 2k)
    for (int q = 0; q < NA; ++q) {
      A[9][q] = mx[q];
      A[10][q] = my[q];
    }
    for (int s = 0; s < 9; ++s) {
      double t[3][2], ms[NA], sx[NA], sy[NA];
      scaled((size_t)cell[s], tr[s][0], tr[s][1], t);
      tri_avgs(t, ms, sx, sy);
      for (int q = 0; q < NA; ++q) {
        A[s][q] = ms[q] - mean[q];
        if (s < 3) {
          A[11 + 2 * s][q] = sx[q];
          A[12 + 2 * s][q] = sy[q];
        }
      }
    }
    double P[NA][ND];
    if (!pinv(A, P)) return fail(GENO_EINVAL, "cell %zu: rank-deficient least-squares stencil", c);
    auto put = [&](int e, double x) { ops[tab_index(e, c, n)] = x; };
    for (int s = 0; s < 9; ++s) put(E_IDX + s, (double)cell[s]);
    put(E_H, h);
    for (int i = 0; i < ND; ++i) {
      for (int q = 0; q < NA; ++q) put(E_M + i * NAP + q, P[q][i]);
      put(E_M + i * NAP + NA, 0.0);
    }
    // linear candidate k: rows (centroid offset), (1, 0), (0, 1) of the
    // edge neighbour; its least-squares inverse in closed form
    for (int kk = 0; kk < 3; ++kk) {
      double t[3][2];
      scaled((size_t)cell[kk], tr[kk][0], tr[kk][1], t);
      const double cx = (t[0][0] + t[1][0] + t[2][0]) / 3.0, cy = (t[0][1] + t[1][1] + t[2][1]) / 3.0;
      const double det = 1.0 + cx * cx + cy * cy;
      const double inv[2][2] = {{(cy * cy + 1.0) / det, -cx * cy / det}, {-cx * cy / det, (cx * cx + 1.0) / det}};
      const double At[2][3] = {{cx, 1.0, 0.0}, {cy, 0.0, 1.0}};
      for (int r = 0; r < 2; ++r)
        for (int col = 0; col < 3; ++col)
          put(E_L + (kk * 2 + r) * 3 + col, inv[r][0] * At[0][col] + inv[r][1] * At[1][col]);
    }
    for (int v = 0; v < 3; ++v) {
      put(E_V + 2 * v, own[v][0]);
      put(E_V + 2 * v + 1, own[v][1]);
    }
    // flux and update geometry
    double perim = 0.0;
    for (int e = 0; e < 3; ++e) {
      const int w = (e + 1) % 3;
      const double dx = vert(c, w, 0) - vert(c, e, 0), dy = vert(c, w, 1) - vert(c, e, 1);
      const double len = std::sqrt(dx * dx + dy * dy);
      perim += len;
      const size_t m = (size_t)nbr[3 * c + e];
      int f = -1;
      for (int q = 0; q < 3; ++q) {
        const double sx = shift[(c * 3 + e) * 2] + shift[(m * 3 + q) * 2];
        const double sy = shift[(c * 3 + e) * 2 + 1] + shift[(m * 3 + q) * 2 + 1];
        if ((size_t)nbr[3 * m + q] == c && std::fabs(sx) <= 1e-12 && std::fabs(sy) <= 1e-12) f = q;
      }
      if (f < 0) return fail(GENO_EINVAL, "cell %zu, edge %d: the neighbour does not point back", c, e);
      const bool owner = c < m || (c == m && e < f);
      put(E_GE + 6 * e + 0, dy / len);
      put(E_GE + 6 * e + 1, -dx / len);
      put(E_GE + 6 * e + 2, len);
      put(E_GE + 6 * e + 3, (double)m);
      put(E_GE + 6 * e + 4, (double)f);
      put(E_GE + 6 * e + 5, owner ? 1.0 : 0.0);
    }
    put(E_G, area);
    put(E_G + 1, 4.0 * area / perim);

  }
  // the list of owned edges (edge-major, then by cell)
  size_t k = 0;
  for (int e = 0; e < 3; ++e)
    for (size_t c = 0; c < n; ++c)
      if (ops[tab_index(E_GE + 6 * e + 5, c, n)] != 0.0) {
        if (k >= 2 * n) return fail(GENO_EINVAL, "more owned edges than the list holds");
        ops[tab_index(E_OWN + (int)(k / n), k % n, n)] = (double)(3 * c + (size_t)e);
        ++k;
      }
  for (; k < 2 * n; ++k) ops[tab_index(E_OWN + (int)(k / n), k % n, n)] = -1.0;
  return GENO_OK;
}

int geno_tri_reconstruct(int ncell, int nv, const void* ops, const double* W, const double* dW,
                         double* out, double* chi, double* sec, void* stream) {
  if (ncell < 1 || nv < 1 || nv > GENO_TRI_MAXV) return fail(GENO_EINVAL, "bad ncell or nv");
  if (!ops || !W || !dW || !out) return fail(GENO_EINVAL, "null pointer");
  TriK k;
  k.C = 20.0;
  k.inv_tanhC = 1.0 / std::tanh(20.0);
  k.eps = 1e-15;
  k.d[0] = k.d[1] = k.d[2] = 1.0;
  const dim3 grid((unsigned)((ncell + 63) / 64)), block(64 * nv);
  hipStream_t s = (hipStream_t)stream;
  const double* T = (const double*)ops;
  switch (nv) {
    case 1: hipLaunchKernelGGL(k_tri<1>, grid, block, 0, s, ncell, T, W, dW, out, chi, sec, k); break;
    case 2: hipLaunchKernelGGL(k_tri<2>, grid, block, 0, s, ncell, T, W, dW, out, chi, sec, k); break;
    case 3: hipLaunchKernelGGL(k_tri<3>, grid, block, 0, s, ncell, T, W, dW, out, chi, sec, k); break;
    default: hipLaunchKernelGGL(k_tri<4>, grid, block, 0, s, ncell, T, W, dW, out, chi, sec, k); break;
  }
  HIP_TRY(hipGetLastError());
  return GENO_OK;
}

size_t geno_tri_workspace_bytes(int ncell) {
  if (ncell < 1) return 0;
  return tri_ws((size_t)ncell).total * sizeof(double);
}

int geno_tri_step(int ncell, const void* ops, double* W, double* dW, void* ws, int nsteps,
                  const geno_params* p, double* dt_out, geno_stats* stats, void* stream) {
  if (ncell < 1) return fail(GENO_EINVAL, "ncell must be >= 1");
  if (!ops || !W || !dW || !ws || !p) return fail(GENO_EINVAL, "null pointer");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  if (p->version != GENO_ABI_VERSION)
    return fail(GENO_EVERSION, "params version %d != %d", p->version, GENO_ABI_VERSION);
  if (p->precision != GENO_F64) return fail(GENO_EINVAL, "the triangle step runs in float64 only");
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->dt_fixed >= 0.0) || !(p->tau_c1 >= 0.0) ||
      !(p->tau_c2 >= 0.0))
    return fail(GENO_EINVAL, "bad method parameters");
  const size_t n = (size_t)ncell;
  const TriWs L = tri_ws(n);
  double* base = (double*)ws;
  TriCtrl* ctrl = reinterpret_cast<TriCtrl*>(base + L.ctrl);
  double* part = base + L.part;
  double* rec = base + L.rec;
  double* sec = base + L.sec;
  double* ebuf = base + L.ebuf;
  double* wst = base + L.wst;
  double* dwst = base + L.dwst;
  double* R = base + L.r;
  double* RG = base + L.rg;
  geno::KParams k{};
  k.gamma = p->gamma;
  k.K = (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0);
  k.tc1 = p->tau_c1;
  k.tc2 = p->tau_c2;
  k.cfl = p->cfl;
  k.dt_fixed = p->dt_fixed;
  TriK tk;
  tk.C = 20.0;
  tk.inv_tanhC = 1.0 / std::tanh(20.0);
  tk.eps = 1e-15;
  tk.d[0] = tk.d[1] = tk.d[2] = 1.0;
  hipStream_t s = (hipStream_t)stream;
  const double* T = (const double*)ops;
  const unsigned nb = (unsigned)((n + 255) / 256), npart = nb;
  const unsigned nrec = (unsigned)((n + 63) / 64), nedge = (unsigned)((2 * n + 255) / 256);
  hipLaunchKernelGGL(k_tri_init, dim3(nb), dim3(256), 0, s, ncell, T, W, part, ctrl, p->gamma);
  for (int step = 0; step < nsteps; ++step) {
    hipLaunchKernelGGL(k_tri_dt, dim3(1), dim3(256), 0, s, part, (int)npart, ctrl, p->cfl,
                       p->dt_fixed, dt_out, step);
    hipLaunchKernelGGL(k_tri<4>, dim3(nrec), dim3(256), 0, s, ncell, T, W, dW, rec,
                       (double*)nullptr, sec, tk);
    hipLaunchKernelGGL(k_tri_edges<1>, dim3(nedge), dim3(256), 0, s, ncell, T, W, rec, sec, ebuf,
                       ctrl, k);
    hipLaunchKernelGGL(k_tri_update<1>, dim3(nb), dim3(256), 0, s, ncell, T, W, wst, dwst, R, RG,
                       ebuf, ctrl, part, p->gamma);
    hipLaunchKernelGGL(k_tri<4>, dim3(nrec), dim3(256), 0, s, ncell, T, wst, dwst, rec,
                       (double*)nullptr, sec, tk);
    hipLaunchKernelGGL(k_tri_edges<2>, dim3(nedge), dim3(256), 0, s, ncell, T, wst, rec, sec,
                       ebuf, ctrl, k);
    hipLaunchKernelGGL(k_tri_update<2>, dim3(nb), dim3(256), 0, s, ncell, T, wst, W, dW, R, RG,
                       ebuf, ctrl, part, p->gamma);
  }
  HIP_TRY(hipGetLastError());
  if (stats) {
    TriCtrl h;
    HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->guard = (long long)h.guard;
    stats->nonfinite = (long long)h.nonfinite;
    stats->last_dt = nsteps > 0 ? h.dt : 0.0;
    if (h.nonfinite)
      return fail(GENO_ENONPHYS, "%llu non-physical cells (non-finite, rho <= 0 or p <= 0)",
                  h.nonfinite);
  }
  return GENO_OK;
}

// per cell and variable, as k_tri executes them: data entries 17, the
// operator product 2 * 153, IS^tau 11, the means and IS~^H over the six
// quadrature points 6 * 92 (point 10, monomials 7, means 18, first
// derivatives 26, second derivatives 20, squares and sum 11), IS^H 1,
// linear candidates 3 * (2 * 5 + 3), IS^L 4, alpha 13, chi 2 (tanh counted
// 1), weights 3 * 4 + 2 + 1, blended gradient 3 * 4, and per Gauss point
// (6): point 6, monomials 7, derivatives 9, cubic 9 * 2 + 2 * 2 * 9, linear
// blend 3 * 4, output 3 * 3
double geno_tri_op_cost(void) {
  const double per_point = 6 + 7 + 9 + (9 * 2 + 2 * 2 * 9) + 3 * 4 + 3 * 3;
  return 17 + 2 * 153 + 11 + 6 * 92 + 1 + 3 * (2 * 5 + 3) + 4 + 13 + 2 + (3 * 4 + 2 + 1) + 3 * 4 +
         6 * per_point;
}

}  // extern "C"
