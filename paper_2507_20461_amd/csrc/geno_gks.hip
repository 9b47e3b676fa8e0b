// HIP kernels and C ABI of the compact gas-kinetic scheme with GENO
// reconstruction for gfx950 (declarations and conventions: geno_gks.h).
//
// One S2O4 stage on a 2-D grid is seven launches on the caller's stream:
//   ghost_x, ghost_y   ghost layers of the stage state (periodic/transmissive)
//   normal<x>          GENO along x on every x-face of rows -1..ny -> face-row buffer
//   faces<x>           tangential step, positivity guard and the gas-kinetic
//                      flux at both Gauss points of every x-face -> F, dF/dt, W(dt/2)
//   normal<y>, faces<y>  the same for y-faces
//   update<stage>      Eq. (1) and the S2O4 stage, gradients by Eq. (2), and
//                      (stage 2) the CFL minimum for the next step
// The time step lives on the device (two ping-pong slots holding the bit
// pattern of min(dx/(|U|+c), dy/(|V|+c))), so a run of steps never waits
// for the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "geno_device.hpp"
#include "geno_gks.h"
#include "gks_device.hpp"

namespace {

constexpr int NG = 2;
constexpr int BLOCK = 256;

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(GENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Optional per-kernel timing: events recorded around every launch of
// gks_step while enabled (measurement support; not thread-safe).
// ---------------------------------------------------------------------------
struct Timing {
  hipEvent_t* ev = nullptr;
  int* kind = nullptr;
  int cap = 0, used = 0;
};
Timing g_tim;

const char* const KNAMES[GENO_NKERNELS] = {"ghost_x", "ghost_y", "normal_x", "normal_y", "faces_x",
                                           "faces_y", "update_1", "update_2", "dt_init", "faces_1d"};

inline void tim_begin(int kind, hipStream_t s) {
  if (g_tim.used < g_tim.cap) {
    g_tim.kind[g_tim.used] = kind;
    hipEventRecord(g_tim.ev[2 * g_tim.used], s);
  }
}
inline void tim_end(hipStream_t s) {
  if (g_tim.used < g_tim.cap) {
    hipEventRecord(g_tim.ev[2 * g_tim.used + 1], s);
    ++g_tim.used;
  }
}

// Geometry passed to the kernels by value.
struct Geo {
  int nx, ny, pitch, rows, yoff, nv;
  int bc[4];
  double dx, dy;
};

__device__ __forceinline__ size_t at(const Geo& g, int f, int j, int i) {
  return ((size_t)f * g.rows + (j + g.yoff)) * g.pitch + (i + NG);
}

// control block at the start of the workspace
struct Ctrl {
  unsigned long long tmin[2];   // CFL minimum per step slot (bit pattern of a positive double)
  unsigned long long guard;     // positivity fall-backs
  unsigned long long nonfinite; // non-finite cells after a stage-2 update
};

__device__ __forceinline__ double dt_of(const Ctrl* c, int slot, double cfl, double dt_fixed) {
  return c ? cfl * __longlong_as_double((long long)c->tmin[slot]) : dt_fixed;
}

template <int NV>
__device__ __forceinline__ bool admissible(const double* W, double gamma) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (!isfinite(W[v])) return false;
  if (!(W[0] > 0.0)) return false;
  double ke = W[1] * W[1];
  if constexpr (NV == 4) ke += W[2] * W[2];
  const double p = (gamma - 1.0) * (W[NV - 1] - 0.5 * ke / W[0]);
  return p > 0.0;
}

// ---------------------------------------------------------------------------
// Ghost cells. Periodic: copy of the periodic image (values and gradients).
// Transmissive: nearest interior cell, gradient normal to the boundary = 0.
// x-ghosts of the interior rows first, then y-ghosts of every column.
// ---------------------------------------------------------------------------
__global__ void k_ghost_x(Geo g, double* __restrict__ W, double* __restrict__ dW, int ndim,
                          Ctrl* ctrl, int step_slot, double cfl, double* dt_out, int step) {
  const int nf = g.nv * (1 + ndim);
  const int total = g.ny * 4 * nf;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (ctrl && t == 0) {
    // start of a step: record dt and clear the other slot for the next minimum
    if (dt_out) dt_out[step] = cfl * __longlong_as_double((long long)ctrl->tmin[step_slot]);
    ctrl->tmin[step_slot ^ 1] = 0x7ff0000000000000ull;   // +inf
  }
  if (t >= total) return;
  const int f = t % nf;
  const int q = (t / nf) % 4;
  const int j = t / (nf * 4);
  const int i = (q == 0) ? -2 : (q == 1) ? -1 : (q == 2) ? g.nx : g.nx + 1;
  const bool lo = q < 2;
  const bool per = g.bc[lo ? 0 : 1] == GENO_BC_PERIODIC;
  const int src = per ? (lo ? i + g.nx : i - g.nx) : (lo ? 0 : g.nx - 1);
  if (f < g.nv) {
    W[at(g, f, j, i)] = W[at(g, f, j, src)];
  } else {
    const int fd = f - g.nv;
    const bool normal = (fd / g.nv) == 0;
    dW[at(g, fd, j, i)] = (!per && normal) ? 0.0 : dW[at(g, fd, j, src)];
  }
}

__global__ void k_ghost_y(Geo g, double* __restrict__ W, double* __restrict__ dW) {
  const int nf = g.nv * 3;
  const int ncol = g.nx + 4;
  const int total = ncol * 4 * nf;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int f = t % nf;
  const int q = (t / nf) % 4;
  const int i = t / (nf * 4) - 2;
  const int j = (q == 0) ? -2 : (q == 1) ? -1 : (q == 2) ? g.ny : g.ny + 1;
  const bool lo = q < 2;
  const bool per = g.bc[lo ? 2 : 3] == GENO_BC_PERIODIC;
  const int src = per ? (lo ? j + g.ny : j - g.ny) : (lo ? 0 : g.ny - 1);
  if (f < g.nv) {
    W[at(g, f, j, i)] = W[at(g, f, src, i)];
  } else {
    const int fd = f - g.nv;
    const bool normal = (fd / g.nv) == 1;
    dW[at(g, fd, j, i)] = (!per && normal) ? 0.0 : dW[at(g, fd, src, i)];
  }
}

// ---------------------------------------------------------------------------
// Normal GENO on face-rows (2-D). DIR 0: rows a = 0..ny+1 (j = a-1), faces
// b = 0..nx (between cells b-1 and b). DIR 1: faces a = 0..ny (between rows
// a-1 and a), columns b = 0..nx+1 (i = b-1).
// fr: [side][quant(value, h d/dn)][var][a][b]; chi: [side][var][a][b].
// ---------------------------------------------------------------------------
template <int DIR>
__global__ void __launch_bounds__(BLOCK) k_normal2d(Geo g, geno::KParams k,
                                                    const double* __restrict__ W,
                                                    const double* __restrict__ dW,
                                                    double* __restrict__ fr,
                                                    double* __restrict__ chi) {
  const int n1 = DIR == 0 ? g.nx + 1 : g.nx + 2;
  const int n0 = DIR == 0 ? g.ny + 2 : g.ny + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * n1) return;
  const int a = t / n1, b = t % n1;
  const size_t plane = (size_t)n0 * n1;
  const size_t o = (size_t)a * n1 + b;
  const double h = DIR == 0 ? g.dx : g.dy;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t id;
      if (DIR == 0) id = at(g, v, a - 1, b - 2 + m);
      else id = at(g, v, a - 2 + m, b - 1);
      Q[m] = W[id];
      G[m] = h * dW[id + (size_t)(DIR * 4) * g.rows * g.pitch];
    }
    double vl, dl, xl, vr, dr, xr;
    geno::geno_face(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, vl, dl, xl, vr, dr, xr);
    fr[(size_t)(0 * 4 + v) * plane + o] = vl;
    fr[(size_t)(1 * 4 + v) * plane + o] = dl;
    fr[(size_t)(2 * 4 + v) * plane + o] = vr;
    fr[(size_t)(3 * 4 + v) * plane + o] = dr;
    if (chi) {
      chi[(size_t)(0 * 4 + v) * plane + o] = xl;
      chi[(size_t)(1 * 4 + v) * plane + o] = xr;
    }
  }
}

// ---------------------------------------------------------------------------
// Faces (2-D): tangential step, positivity guard, then either the point
// states (MODE 0, geno_reconstruct) or the Gauss-averaged flux (MODE 1).
// DIR 0: a = row t (0..ny-1), b = face (0..nx); DIR 1: a = face (0..ny),
// b = column t (0..nx-1).
// ---------------------------------------------------------------------------
template <int DIR, int MODE>
__global__ void __launch_bounds__(BLOCK) k_faces2d(Geo g, geno::KParams k,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ fr,
                                                   double* __restrict__ out, Ctrl* ctrl,
                                                   int slot, double dt_fixed, int want_F) {
  const int n1 = DIR == 0 ? g.nx + 1 : g.nx;
  const int n0 = DIR == 0 ? g.ny : g.ny + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * n1) return;
  const int a = t / n1, b = t % n1;
  // face-row buffer geometry
  const int r1 = DIR == 0 ? g.nx + 1 : g.nx + 2;
  const int r0 = DIR == 0 ? g.ny + 2 : g.ny + 1;
  const size_t rplane = (size_t)r0 * r1;
  // rows t-1, t, t+1 of this face in the face-row buffer
  size_t rm, rc, rp;
  if (DIR == 0) {
    rm = (size_t)a * r1 + b;
    rc = rm + r1;
    rp = rc + r1;
  } else {
    rm = (size_t)a * r1 + b;
    rc = rm + 1;
    rp = rc + 1;
  }
  // S[side][gauss][var], Dn[side][var], Dt[side][gauss][var] (h-scaled)
  double S[2][2][4], Dn[2][4], Dt[2][2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* p = fr + (size_t)((2 * s + 0) * 4 + v) * rplane;
      geno::tangential(p[rm], p[rc], p[rp], k, S[s][0][v], S[s][1][v], Dt[s][0][v], Dt[s][1][v]);
      Dn[s][v] = fr[(size_t)((2 * s + 1) * 4 + v) * rplane + rc];
    }
  }
  // positivity guard per side and point: fall back to the own cell average
  const double gamma = k.gamma;
  int nguard = 0;
  double Dnp[2][2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool ok = admissible<4>(S[s][q], gamma);
#pragma unroll
      for (int v = 0; v < 4; ++v) Dnp[s][q][v] = ok ? Dn[s][v] : 0.0;
      if (!ok) {
        ++nguard;
        int ci, cj;
        if (DIR == 0) { ci = b - 1 + s; cj = a; }
        else { ci = b; cj = a - 1 + s; }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          S[s][q][v] = W[at(g, v, cj, ci)];
          Dt[s][q][v] = 0.0;
        }
      }
    }
  }
  if (nguard && ctrl) atomicAdd(&ctrl->guard, (unsigned long long)nguard);
  const size_t plane = (size_t)n0 * n1;
  const size_t o = (size_t)a * n1 + b;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t base = (size_t)(((s * 2 + q) * 3) * 4);
          out[(base + 0 * 4 + v) * plane + o] = S[s][q][v];
          out[(base + 1 * 4 + v) * plane + o] = Dnp[s][q][v];
          out[(base + 2 * 4 + v) * plane + o] = Dt[s][q][v];
        }
  } else {
    const double dt = dt_of(ctrl, slot, k.cfl, dt_fixed);
    const double hn = DIR == 0 ? g.dx : g.dy, ht = DIR == 0 ? g.dy : g.dx;
    const double ihn = 1.0 / hn, iht = 1.0 / ht;
    // face frame: normal momentum first
    constexpr int p1 = DIR == 0 ? 1 : 2, p2 = DIR == 0 ? 2 : 1;
    double F[4] = {0, 0, 0, 0}, Ft[4] = {0, 0, 0, 0}, Wi[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double Wl[4], Wr[4], nl[4], nr[4], tl[4], tr[4];
      const int perm[4] = {0, p1, p2, 3};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Wl[v] = S[0][q][perm[v]];
        Wr[v] = S[1][q][perm[v]];
        nl[v] = Dnp[0][q][perm[v]] * ihn;
        nr[v] = Dnp[1][q][perm[v]] * ihn;
        tl[v] = Dt[0][q][perm[v]] * iht;
        tr[v] = Dt[1][q][perm[v]] * iht;
      }
      gks::point_flux<4>(Wl, Wr, nl, nr, tl, tr, dt, k, 0.5, want_F != 0, F, Ft, Wi);
    }
    const double Fo[4] = {F[0], DIR == 0 ? F[1] : F[2], DIR == 0 ? F[2] : F[1], F[3]};
    const double Fto[4] = {Ft[0], DIR == 0 ? Ft[1] : Ft[2], DIR == 0 ? Ft[2] : Ft[1], Ft[3]};
    const double Wio[4] = {Wi[0], DIR == 0 ? Wi[1] : Wi[2], DIR == 0 ? Wi[2] : Wi[1], Wi[3]};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (want_F) out[(size_t)(0 * 4 + v) * plane + o] = Fo[v];
      out[(size_t)(1 * 4 + v) * plane + o] = Fto[v];
      out[(size_t)(2 * 4 + v) * plane + o] = Wio[v];
    }
  }
}

// ---------------------------------------------------------------------------
// 1-D faces: normal GENO of the three variables at face f (cells f-2..f+1),
// guard, then states (MODE 0) or flux (MODE 1). out as the 2-D layouts with
// one Gauss point: states [side][quant(2)][var][f], flux [kind][var][f].
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(BLOCK) k_faces1d(Geo g, geno::KParams k,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ dW,
                                                   double* __restrict__ out,
                                                   double* __restrict__ chi, Ctrl* ctrl,
                                                   int slot, double dt_fixed, int want_F) {
  const int nfc = g.nx + 1;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  double S[2][3], Dn[2][3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const size_t id = at(g, v, 0, f - 2 + m);
      Q[m] = W[id];
      G[m] = g.dx * dW[id];
    }
    double xl, xr;
    geno::geno_face(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, S[0][v], Dn[0][v], xl,
                    S[1][v], Dn[1][v], xr);
    if (chi) {
      chi[(size_t)(0 * 3 + v) * nfc + f] = xl;
      chi[(size_t)(1 * 3 + v) * nfc + f] = xr;
    }
  }
  int nguard = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!admissible<3>(S[s], k.gamma)) {
      ++nguard;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        S[s][v] = W[at(g, v, 0, f - 1 + s)];
        Dn[s][v] = 0.0;
      }
    }
  }
  if (nguard && ctrl) atomicAdd(&ctrl->guard, (unsigned long long)nguard);
  if constexpr (MODE == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        out[(size_t)((s * 2 + 0) * 3 + v) * nfc + f] = S[s][v];
        out[(size_t)((s * 2 + 1) * 3 + v) * nfc + f] = Dn[s][v];
      }
  } else {
    const double dt = dt_of(ctrl, slot, k.cfl, dt_fixed);
    const double ih = 1.0 / g.dx;
    double nl[3], nr[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      nl[v] = Dn[0][v] * ih;
      nr[v] = Dn[1][v] * ih;
    }
    double F[3] = {0, 0, 0}, Ft[3] = {0, 0, 0}, Wi[3] = {0, 0, 0};
    gks::point_flux<3>(S[0], S[1], nl, nr, nullptr, nullptr, dt, k, 1.0, want_F != 0, F, Ft, Wi);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (want_F) out[(size_t)(0 * 3 + v) * nfc + f] = F[v];
      out[(size_t)(1 * 3 + v) * nfc + f] = Ft[v];
      out[(size_t)(2 * 3 + v) * nfc + f] = Wi[v];
    }
  }
}

// gks_flux on caller-given point states (layout of geno_reconstruct).
template <int NV>
__global__ void __launch_bounds__(BLOCK) k_flux_points(int nfaces, int ngauss, int dir,
                                                       geno::KParams k, double hn, double ht,
                                                       double dt, const double* __restrict__ st,
                                                       double* __restrict__ F,
                                                       double* __restrict__ Ft,
                                                       double* __restrict__ Wi) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nfaces) return;
  constexpr int Q = NV == 4 ? 3 : 2;
  const double w = 1.0 / ngauss;
  const int perm[4] = {0, dir == 0 ? 1 : 2, dir == 0 ? 2 : 1, 3};
  double Fa[NV], Fta[NV], Wia[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Fa[v] = Fta[v] = Wia[v] = 0.0;
  for (int q = 0; q < ngauss; ++q) {
    double Ws[2][NV], ns[2][NV], ts[2][NV];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int pv = NV == 4 ? perm[v] : v;
        const size_t base = (size_t)((s * ngauss + q) * Q) * NV;
        Ws[s][v] = st[(base + 0 * NV + pv) * nfaces + o];
        ns[s][v] = st[(base + 1 * NV + pv) * nfaces + o] / hn;
        ts[s][v] = NV == 4 ? st[(base + 2 * NV + pv) * nfaces + o] / ht : 0.0;
      }
    gks::point_flux<NV>(Ws[0], Ws[1], ns[0], ns[1], ts[0], ts[1], dt, k, w, true, Fa, Fta, Wia);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int pv = NV == 4 ? perm[v] : v;
    if (F) F[(size_t)pv * nfaces + o] = Fa[v];
    if (Ft) Ft[(size_t)pv * nfaces + o] = Fta[v];
    if (Wi) Wi[(size_t)pv * nfaces + o] = Wia[v];
  }
}

// ---------------------------------------------------------------------------
// Cell update. STAGE 1: W* = W + dt/2 L + dt^2/8 Lt, R = W + dt L + dt^2/6 Lt,
// grad* from W_int (Eq. (2)). STAGE 2: W = R + dt^2/3 Lt*, grad from the
// stage-2 W_int, and the CFL minimum of the new state into the next slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void atomic_min_pos(unsigned long long* p, double x) {
  atomicMin(p, (unsigned long long)__double_as_longlong(x));
}

template <int NDIM, int STAGE>
__global__ void __launch_bounds__(BLOCK) k_update(Geo g, geno::KParams k,
                                                  const double* __restrict__ Win,
                                                  double* __restrict__ Wout,
                                                  double* __restrict__ dWout,
                                                  double* __restrict__ R,
                                                  const double* __restrict__ fx,
                                                  const double* __restrict__ fy, Ctrl* ctrl,
                                                  int slot) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.nx * g.ny;
  const double dt = dt_of(ctrl, slot, k.cfl, 0.0);
  double tloc = INFINITY;
  bool bad = false;
  if (t < n) {
    const int j = t / g.nx, i = t % g.nx;
    const size_t px = (size_t)(g.nx + 1) * g.ny;
    const size_t py = (size_t)g.nx * (g.ny + 1);
    const size_t ox = (size_t)j * (g.nx + 1) + i;
    const size_t oy = (size_t)j * g.nx + i;
    double Wn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double l = -(fx[(0 * NV + v) * px + ox + 1] - fx[(0 * NV + v) * px + ox]) / g.dx;
      double lt = -(fx[(1 * NV + v) * px + ox + 1] - fx[(1 * NV + v) * px + ox]) / g.dx;
      const double gx = (fx[(2 * NV + v) * px + ox + 1] - fx[(2 * NV + v) * px + ox]) / g.dx;
      double gy = 0.0;
      if constexpr (NDIM == 2) {
        l += -(fy[(0 * NV + v) * py + oy + g.nx] - fy[(0 * NV + v) * py + oy]) / g.dy;
        lt += -(fy[(1 * NV + v) * py + oy + g.nx] - fy[(1 * NV + v) * py + oy]) / g.dy;
        gy = (fy[(2 * NV + v) * py + oy + g.nx] - fy[(2 * NV + v) * py + oy]) / g.dy;
      }
      const size_t c = at(g, v, j, i);
      if constexpr (STAGE == 1) {
        const double w = Win[c];
        Wout[c] = w + 0.5 * dt * l + dt * dt / 8.0 * lt;
        R[c] = w + dt * l + dt * dt / 6.0 * lt;
      } else {
        Wn[v] = R[c] + dt * dt / 3.0 * lt;
        Wout[c] = Wn[v];
      }
      dWout[at(g, v, j, i)] = gx;
      if constexpr (NDIM == 2) dWout[at(g, NV + v, j, i)] = gy;
    }
    if constexpr (STAGE == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) bad |= !isfinite(Wn[v]);
      const double rho = Wn[0], U = Wn[1] / rho;
      const double V = NV == 4 ? Wn[2] / rho : 0.0;
      const double p = (k.gamma - 1.0) * (Wn[NV - 1] - 0.5 * rho * (U * U + V * V));
      const double c = sqrt(k.gamma * p / rho);
      tloc = g.dx / (fabs(U) + c);
      if constexpr (NDIM == 2) tloc = fmin(tloc, g.dy / (fabs(V) + c));
      if (!(tloc > 0.0)) tloc = 0.0;   // NaN state: zero step, flagged below
    }
  }
  if constexpr (STAGE == 2) {
    // wavefront minimum, then one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tloc = fmin(tloc, __shfl_xor(tloc, off, 64));
    const unsigned long long nb = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && ctrl) {
      if (tloc < INFINITY) atomic_min_pos(&ctrl->tmin[slot ^ 1], tloc);
      if (nb) atomicAdd(&ctrl->nonfinite, (unsigned long long)__popcll(nb));
    }
  }
}

// CFL minimum of the initial state into slot 0 (one workgroup).
template <int NDIM>
__global__ void __launch_bounds__(1024) k_dt_init(Geo g, geno::KParams k,
                                                  const double* __restrict__ W, Ctrl* ctrl) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  __shared__ double red[16];
  double tloc = INFINITY;
  const int n = g.nx * g.ny;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int j = t / g.nx, i = t % g.nx;
    const double rho = W[at(g, 0, j, i)];
    const double U = W[at(g, 1, j, i)] / rho;
    const double V = NV == 4 ? W[at(g, 2, j, i)] / rho : 0.0;
    const double p = (k.gamma - 1.0) * (W[at(g, NV - 1, j, i)] - 0.5 * rho * (U * U + V * V));
    const double c = sqrt(k.gamma * p / rho);
    double tt = g.dx / (fabs(U) + c);
    if constexpr (NDIM == 2) tt = fmin(tt, g.dy / (fabs(V) + c));
    if (!(tt > 0.0)) tt = 0.0;
    tloc = fmin(tloc, tt);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tloc = fmin(tloc, __shfl_xor(tloc, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tloc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmin(m, red[w]);
    ctrl->tmin[0] = (unsigned long long)__double_as_longlong(m);
    ctrl->tmin[1] = 0x7ff0000000000000ull;
    ctrl->guard = 0;
    ctrl->nonfinite = 0;
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
struct Layout {
  size_t ctrl, wst, dwst, r, fr[2], fl[2], total;
  size_t nstate;   // doubles per field plane
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_of(const geno_grid* g) {
  Layout L{};
  const int nv = g->ndim == 2 ? 4 : 3;
  L.nstate = (size_t)g->rows * g->pitch;
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + sizeof(Ctrl));
  L.wst = off;
  off = align256(off + L.nstate * nv * sizeof(double));
  L.dwst = off;
  off = align256(off + L.nstate * nv * g->ndim * sizeof(double));
  L.r = off;
  off = align256(off + L.nstate * nv * sizeof(double));
  if (g->ndim == 2) {
    L.fr[0] = off;
    off = align256(off + (size_t)16 * (g->ny + 2) * (g->nx + 1) * sizeof(double));
    L.fr[1] = off;
    off = align256(off + (size_t)16 * (g->ny + 1) * (g->nx + 2) * sizeof(double));
    L.fl[0] = off;
    off = align256(off + (size_t)12 * g->ny * (g->nx + 1) * sizeof(double));
    L.fl[1] = off;
    off = align256(off + (size_t)12 * (g->ny + 1) * g->nx * sizeof(double));
  } else {
    L.fr[0] = L.fr[1] = 0;
    L.fl[0] = off;
    off = align256(off + (size_t)9 * (g->nx + 1) * sizeof(double));
    L.fl[1] = 0;
  }
  L.total = off;
  return L;
}

int check_params(const geno_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  if (p->version != GENO_ABI_VERSION)
    return fail(GENO_EVERSION, "params version %d != %d", p->version, GENO_ABI_VERSION);
  if (p->precision != GENO_F64) return fail(GENO_EINVAL, "unsupported precision %d", p->precision);
  if (p->r != 2.0 || p->rL != 2.0) return fail(GENO_EINVAL, "only r = rL = 2 are implemented");
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->C > 0.0) || !(p->cfl > 0.0))
    return fail(GENO_EINVAL, "gamma > 1, eps > 0, C > 0 and cfl > 0 are required");
  if (!(p->d[0] > 0.0 && p->d[1] > 0.0 && p->d[2] > 0.0))
    return fail(GENO_EINVAL, "linear weights d must be positive");
  if (!(p->tau_c1 >= 0.0) || !(p->tau_c2 >= 0.0))
    return fail(GENO_EINVAL, "tau coefficients must be >= 0");
  for (int i = 0; i < 4; ++i)
    if (p->bc[i] != GENO_BC_PERIODIC && p->bc[i] != GENO_BC_TRANSMISSIVE)
      return fail(GENO_EINVAL, "bad boundary code %d", p->bc[i]);
  if ((p->bc[0] == GENO_BC_PERIODIC) != (p->bc[1] == GENO_BC_PERIODIC) ||
      (p->bc[2] == GENO_BC_PERIODIC) != (p->bc[3] == GENO_BC_PERIODIC))
    return fail(GENO_EINVAL, "periodic boundaries must be set on both sides of an axis");
  return GENO_OK;
}

int check_grid(const geno_grid* g) {
  if (!g) return fail(GENO_EINVAL, "null grid");
  int rc = check_params(&g->params);
  if (rc) return rc;
  if (g->ndim != 1 && g->ndim != 2) return fail(GENO_EINVAL, "ndim must be 1 or 2");
  if (g->nx < 1 || g->ny < 1 || (g->ndim == 1 && g->ny != 1))
    return fail(GENO_EINVAL, "bad grid size");
  if (g->pitch < g->nx + 2 * NG || g->rows != (g->ndim == 2 ? g->ny + 2 * NG : 1))
    return fail(GENO_EINVAL, "grid pitch/rows inconsistent (use geno_grid_init)");
  // periodic images must exist: 2 ghost layers need at least 2 cells
  if ((g->params.bc[0] == GENO_BC_PERIODIC && g->nx < NG) ||
      (g->ndim == 2 && g->params.bc[2] == GENO_BC_PERIODIC && g->ny < NG))
    return fail(GENO_EINVAL, "periodic axis needs at least %d cells", NG);
  if ((size_t)(g->nx + 4) * (g->ny + 4) * 16 > (size_t)0x7fffffff)
    return fail(GENO_EINVAL, "grid too large for 32-bit thread indexing");
  if (!(g->dx > 0.0) || !(g->dy > 0.0)) return fail(GENO_EINVAL, "bad cell size");
  return GENO_OK;
}

geno::KParams kparams(const geno_grid* g) {
  geno::KParams k;
  const geno_params& p = g->params;
  k.C = p.C;
  k.tanhC = std::tanh(p.C);
  k.eps = p.eps;
  k.d1 = p.d[0];
  k.d2 = p.d[1];
  k.d3 = p.d[2];
  k.gamma = p.gamma;
  k.K = g->ndim == 1 ? (3.0 - p.gamma) / (p.gamma - 1.0) : (4.0 - 2.0 * p.gamma) / (p.gamma - 1.0);
  k.tc1 = p.tau_c1;
  k.tc2 = p.tau_c2;
  k.cfl = p.cfl;
  return k;
}

Geo geo_of(const geno_grid* g) {
  Geo o;
  o.nx = g->nx;
  o.ny = g->ny;
  o.pitch = g->pitch;
  o.rows = g->rows;
  o.yoff = g->ndim == 2 ? NG : 0;
  o.nv = g->ndim == 2 ? 4 : 3;
  for (int i = 0; i < 4; ++i) o.bc[i] = g->params.bc[i];
  o.dx = g->dx;
  o.dy = g->dy;
  return o;
}

inline unsigned nblocks(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// ghost fill of one state (W, dW)
int launch_ghosts(const geno_grid* g, const Geo& geo, double* W, double* dW, hipStream_t s,
                  Ctrl* ctrl, int slot, double cfl, double* dt_out, int step) {
  const int nv = geo.nv;
  const size_t nx_items = (size_t)g->ny * 4 * nv * (1 + g->ndim);
  tim_begin(GENO_K_GHOST_X, s);
  hipLaunchKernelGGL(k_ghost_x, dim3(nblocks(nx_items)), dim3(BLOCK), 0, s, geo, W, dW, g->ndim,
                     ctrl, slot, cfl, dt_out, step);
  tim_end(s);
  if (g->ndim == 2) {
    const size_t ny_items = (size_t)(g->nx + 4) * 4 * 12;
    tim_begin(GENO_K_GHOST_Y, s);
    hipLaunchKernelGGL(k_ghost_y, dim3(nblocks(ny_items)), dim3(BLOCK), 0, s, geo, W, dW);
    tim_end(s);
  }
  HIP_TRY(hipGetLastError());
  return GENO_OK;
}

// one stage of gks_step: faces and update
int launch_stage(const geno_grid* g, const Geo& geo, const geno::KParams& k, char* ws,
                 const Layout& L, double* Win, double* dWin, int stage, int slot, double* dt_out,
                 int step, double* Wfinal, double* dWfinal, hipStream_t s) {
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  double* Wst = reinterpret_cast<double*>(ws + L.wst);
  double* dWst = reinterpret_cast<double*>(ws + L.dwst);
  double* R = reinterpret_cast<double*>(ws + L.r);
  double* fl0 = reinterpret_cast<double*>(ws + L.fl[0]);
  double* fl1 = g->ndim == 2 ? reinterpret_cast<double*>(ws + L.fl[1]) : nullptr;
  int rc = launch_ghosts(g, geo, Win, dWin, s, stage == 1 ? ctrl : nullptr, slot, k.cfl,
                         dt_out, step);
  if (rc) return rc;
  const int want_F = stage == 1;
  if (g->ndim == 2) {
    double* fr0 = reinterpret_cast<double*>(ws + L.fr[0]);
    double* fr1 = reinterpret_cast<double*>(ws + L.fr[1]);
    tim_begin(GENO_K_NORMAL_X, s);
    hipLaunchKernelGGL(k_normal2d<0>, dim3(nblocks((size_t)(g->ny + 2) * (g->nx + 1))),
                       dim3(BLOCK), 0, s, geo, k, Win, dWin, fr0, nullptr);
    tim_end(s);
    tim_begin(GENO_K_FACES_X, s);
    hipLaunchKernelGGL((k_faces2d<0, 1>), dim3(nblocks((size_t)g->ny * (g->nx + 1))), dim3(BLOCK),
                       0, s, geo, k, Win, fr0, fl0, ctrl, slot, 0.0, want_F);
    tim_end(s);
    tim_begin(GENO_K_NORMAL_Y, s);
    hipLaunchKernelGGL(k_normal2d<1>, dim3(nblocks((size_t)(g->ny + 1) * (g->nx + 2))),
                       dim3(BLOCK), 0, s, geo, k, Win, dWin, fr1, nullptr);
    tim_end(s);
    tim_begin(GENO_K_FACES_Y, s);
    hipLaunchKernelGGL((k_faces2d<1, 1>), dim3(nblocks((size_t)(g->ny + 1) * g->nx)), dim3(BLOCK),
                       0, s, geo, k, Win, fr1, fl1, ctrl, slot, 0.0, want_F);
    tim_end(s);
  } else {
    tim_begin(GENO_K_FACES_1D, s);
    hipLaunchKernelGGL(k_faces1d<1>, dim3(nblocks((size_t)g->nx + 1)), dim3(BLOCK), 0, s, geo, k,
                       Win, dWin, fl0, nullptr, ctrl, slot, 0.0, want_F);
    tim_end(s);
  }
  const size_t ncell = (size_t)g->nx * g->ny;
  tim_begin(stage == 1 ? GENO_K_UPDATE_1 : GENO_K_UPDATE_2, s);
  if (g->ndim == 2) {
    if (stage == 1)
      hipLaunchKernelGGL((k_update<2, 1>), dim3(nblocks(ncell)), dim3(BLOCK), 0, s, geo, k, Win,
                         Wst, dWst, R, fl0, fl1, ctrl, slot);
    else
      hipLaunchKernelGGL((k_update<2, 2>), dim3(nblocks(ncell)), dim3(BLOCK), 0, s, geo, k, Win,
                         Wfinal, dWfinal, R, fl0, fl1, ctrl, slot);
  } else {
    if (stage == 1)
      hipLaunchKernelGGL((k_update<1, 1>), dim3(nblocks(ncell)), dim3(BLOCK), 0, s, geo, k, Win,
                         Wst, dWst, R, fl0, fl1, ctrl, slot);
    else
      hipLaunchKernelGGL((k_update<1, 2>), dim3(nblocks(ncell)), dim3(BLOCK), 0, s, geo, k, Win,
                         Wfinal, dWfinal, R, fl0, fl1, ctrl, slot);
  }
  tim_end(s);
  HIP_TRY(hipGetLastError());
  return GENO_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int geno_abi_version(void) { return GENO_ABI_VERSION; }

int geno_timing_enable(int max_launches) {
  for (int i = 0; i < 2 * g_tim.cap; ++i) hipEventDestroy(g_tim.ev[i]);
  free(g_tim.ev);
  free(g_tim.kind);
  g_tim = Timing{};
  if (max_launches <= 0) return GENO_OK;
  g_tim.ev = (hipEvent_t*)calloc((size_t)2 * max_launches, sizeof(hipEvent_t));
  g_tim.kind = (int*)calloc((size_t)max_launches, sizeof(int));
  if (!g_tim.ev || !g_tim.kind) return fail(GENO_EINVAL, "out of host memory");
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipError_t e = hipEventCreate(&g_tim.ev[i]);
    if (e != hipSuccess) {
      g_tim.cap = i / 2;
      return fail(GENO_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  g_tim.cap = max_launches;
  return GENO_OK;
}

int geno_timing_read(int nkinds, double* ms_total, long long* launches) {
  if (!ms_total || !launches || nkinds < 1) return fail(GENO_EINVAL, "null argument");
  for (int k = 0; k < nkinds; ++k) {
    ms_total[k] = 0.0;
    launches[k] = 0;
  }
  for (int i = 0; i < g_tim.used; ++i) {
    HIP_TRY(hipEventSynchronize(g_tim.ev[2 * i + 1]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, g_tim.ev[2 * i], g_tim.ev[2 * i + 1]));
    const int k = g_tim.kind[i];
    if (k < nkinds) {
      ms_total[k] += ms;
      launches[k] += 1;
    }
  }
  g_tim.used = 0;
  return GENO_OK;
}

const char* geno_kernel_name(int kind) {
  return (kind >= 0 && kind < GENO_NKERNELS) ? KNAMES[kind] : "";
}

const char* geno_last_error(void) { return g_err; }

int geno_params_default(geno_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  memset(p, 0, sizeof *p);
  p->version = GENO_ABI_VERSION;
  p->precision = GENO_F64;
  p->gamma = 1.4;
  p->C = 20.0;
  p->eps = 1e-15;
  p->r = 2.0;
  p->rL = 2.0;
  p->d[0] = 1.0;
  p->d[1] = 8.0;
  p->d[2] = 1.0;
  p->tau_c1 = 0.0;
  p->tau_c2 = 1.0;
  p->cfl = 0.5;
  for (int i = 0; i < 4; ++i) p->bc[i] = GENO_BC_TRANSMISSIVE;
  return GENO_OK;
}

int geno_grid_init(geno_grid* g, int ndim, int nx, int ny, double x0, double x1, double y0,
                   double y1, const geno_params* p) {
  if (!g || !p) return fail(GENO_EINVAL, "null argument");
  int rc = check_params(p);
  if (rc) return rc;
  if (ndim != 1 && ndim != 2) return fail(GENO_EINVAL, "ndim must be 1 or 2");
  if (nx < 1 || (ndim == 2 && ny < 1)) return fail(GENO_EINVAL, "bad grid size");
  if (!(x1 > x0) || (ndim == 2 && !(y1 > y0))) return fail(GENO_EINVAL, "empty interval");
  memset(g, 0, sizeof *g);
  g->ndim = ndim;
  g->nx = nx;
  g->ny = ndim == 2 ? ny : 1;
  g->pitch = ((nx + 2 * NG + 15) / 16) * 16;
  g->rows = ndim == 2 ? ny + 2 * NG : 1;
  g->x0 = x0;
  g->x1 = x1;
  g->y0 = ndim == 2 ? y0 : 0.0;
  g->y1 = ndim == 2 ? y1 : 1.0;
  g->dx = (x1 - x0) / nx;
  g->dy = ndim == 2 ? (y1 - y0) / ny : 1.0;
  g->params = *p;
  return check_grid(g);
}

size_t geno_state_elems(const geno_grid* g, int nfields) {
  if (!g || nfields < 1) return 0;
  return (size_t)nfields * g->rows * g->pitch;
}

size_t gks_workspace_bytes(const geno_grid* g) {
  if (!g || check_grid(g)) return 0;
  return layout_of(g).total;
}

int geno_reconstruct(const geno_grid* g, void* W, void* dW, int dir, void* face_state, void* chi,
                     void* ws, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !dW || !face_state || !ws) return fail(GENO_EINVAL, "null pointer");
  if (dir != 0 && !(g->ndim == 2 && dir == 1)) return fail(GENO_EINVAL, "bad direction %d", dir);
  hipStream_t s = (hipStream_t)stream;
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  char* w = (char*)ws;
  double* Wd = (double*)W;
  double* dWd = (double*)dW;
  rc = launch_ghosts(g, geo, Wd, dWd, s, nullptr, 0, 0.0, nullptr, 0);
  if (rc) return rc;
  if (g->ndim == 1) {
    hipLaunchKernelGGL(k_faces1d<0>, dim3(nblocks((size_t)g->nx + 1)), dim3(BLOCK), 0, s, geo, k,
                       Wd, dWd, (double*)face_state, (double*)chi, nullptr, 0, 0.0, 0);
  } else {
    double* fr = (double*)(w + L.fr[dir]);
    if (dir == 0) {
      hipLaunchKernelGGL(k_normal2d<0>, dim3(nblocks((size_t)(g->ny + 2) * (g->nx + 1))),
                         dim3(BLOCK), 0, s, geo, k, Wd, dWd, fr, (double*)chi);
      hipLaunchKernelGGL((k_faces2d<0, 0>), dim3(nblocks((size_t)g->ny * (g->nx + 1))),
                         dim3(BLOCK), 0, s, geo, k, Wd, fr, (double*)face_state, nullptr, 0, 0.0,
                         0);
    } else {
      hipLaunchKernelGGL(k_normal2d<1>, dim3(nblocks((size_t)(g->ny + 1) * (g->nx + 2))),
                         dim3(BLOCK), 0, s, geo, k, Wd, dWd, fr, (double*)chi);
      hipLaunchKernelGGL((k_faces2d<1, 0>), dim3(nblocks((size_t)(g->ny + 1) * g->nx)),
                         dim3(BLOCK), 0, s, geo, k, Wd, fr, (double*)face_state, nullptr, 0, 0.0,
                         0);
    }
  }
  HIP_TRY(hipGetLastError());
  return GENO_OK;
}

int gks_flux(const geno_grid* g, const void* face_state, double dt, int dir, void* F, void* Ft,
             void* Wint, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!face_state) return fail(GENO_EINVAL, "null face_state");
  if (!(dt > 0.0)) return fail(GENO_EINVAL, "dt must be positive");
  if (dir != 0 && !(g->ndim == 2 && dir == 1)) return fail(GENO_EINVAL, "bad direction %d", dir);
  hipStream_t s = (hipStream_t)stream;
  const geno::KParams k = kparams(g);
  if (g->ndim == 1) {
    const int nf = g->nx + 1;
    hipLaunchKernelGGL(k_flux_points<3>, dim3(nblocks(nf)), dim3(BLOCK), 0, s, nf, 1, 0, k, g->dx,
                       g->dy, dt, (const double*)face_state, (double*)F, (double*)Ft,
                       (double*)Wint);
  } else {
    const int nf = dir == 0 ? g->ny * (g->nx + 1) : (g->ny + 1) * g->nx;
    const double hn = dir == 0 ? g->dx : g->dy, ht = dir == 0 ? g->dy : g->dx;
    hipLaunchKernelGGL(k_flux_points<4>, dim3(nblocks(nf)), dim3(BLOCK), 0, s, nf, 2, dir, k, hn,
                       ht, dt, (const double*)face_state, (double*)F, (double*)Ft,
                       (double*)Wint);
  }
  HIP_TRY(hipGetLastError());
  return GENO_OK;
}

int gks_step(const geno_grid* g, void* W, void* dW, void* ws, int nsteps, double* dt_out,
             geno_stats* stats, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !dW || !ws) return fail(GENO_EINVAL, "null pointer");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  char* w = (char*)ws;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(w + L.ctrl);
  double* Wd = (double*)W;
  double* dWd = (double*)dW;
  double* Wst = reinterpret_cast<double*>(w + L.wst);
  double* dWst = reinterpret_cast<double*>(w + L.dwst);
  tim_begin(GENO_K_DT_INIT, s);
  if (g->ndim == 2)
    hipLaunchKernelGGL(k_dt_init<2>, dim3(1), dim3(1024), 0, s, geo, k, Wd, ctrl);
  else
    hipLaunchKernelGGL(k_dt_init<1>, dim3(1), dim3(1024), 0, s, geo, k, Wd, ctrl);
  tim_end(s);
  HIP_TRY(hipGetLastError());
  for (int n = 0; n < nsteps; ++n) {
    const int slot = n & 1;
    rc = launch_stage(g, geo, k, w, L, Wd, dWd, 1, slot, dt_out, n, nullptr, nullptr, s);
    if (rc) return rc;
    rc = launch_stage(g, geo, k, w, L, Wst, dWst, 2, slot, nullptr, n, Wd, dWd, s);
    if (rc) return rc;
  }
  if (stats) {
    Ctrl h;
    HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->guard = (long long)h.guard;
    stats->nonfinite = (long long)h.nonfinite;
    const int last = nsteps > 0 ? (nsteps - 1) & 1 : 0;
    double tm;
    memcpy(&tm, &h.tmin[last], sizeof tm);
    stats->last_dt = nsteps > 0 ? k.cfl * tm : 0.0;
    if (h.nonfinite) return fail(GENO_ENONPHYS, "%llu non-finite cells", h.nonfinite);
  }
  return GENO_OK;
}

}  // extern "C"
