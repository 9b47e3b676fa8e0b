// HIP kernels and C ABI of the compact gas-kinetic scheme with GENO
// reconstruction for gfx950 (declarations and conventions: geno_gks.h).
//
// One S2O4 stage on a 2-D grid, per direction d in {x, y}:
//   normal<d>   GENO along d on every face-row the tangential step reads
//               -> face-row buffer (value and h*d/dn per side and variable)
//   faces<d>    two lanes per face, one per Gauss point: tangential step,
//               positivity guard and the gas-kinetic flux for tau = 0; faces
//               with tau > 0 at either point go to a queue
// then slow: the queued faces of both directions with the full BGK solution
// (tau > 0), and update<stage>: Eq. (1) with the S2O4 stage, the gradients by Eq. (2),
// the ghost cells of the new state (every interior cell writes its ghost
// images) and, in stage 2, per-block CFL minima for the next step, reduced
// by the next step's first kernel. The time step therefore never leaves the
// device and a run of steps never waits for the host.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "geno6_device.hpp"
#include "geno_device.hpp"
#include "geno_gks.h"
#include "gks_device.hpp"
#include "mlp_device.hpp"

// error message of the last failed call on this thread (geno_last_error),
// shared with the other source files of the library
namespace geno_err {
thread_local char g_err[512] = "";
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}
}  // namespace geno_err

namespace {

constexpr int NG = 2;
constexpr int BLOCK = 256;          // work-group size of the single-grid launches
constexpr int MAXWAVES = 16;        // waves of the largest work-group (1024 lanes)
constexpr int SLOW_BLOCKS = 1024;   // fixed grid of the queue kernels (grid-stride)

using geno_err::fail;

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(GENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Optional per-kernel timing: start/stop events bound to the dispatch of each
// launch of gks_step while enabled (measurement support; not thread-safe).
// ---------------------------------------------------------------------------
struct Timing {
  hipEvent_t* ev = nullptr;
  int* kind = nullptr;
  int cap = 0, used = 0;
};
Timing g_tim;
int g_tim_suspend = 0;   // set while a launch sequence is captured into a graph

const char* const KNAMES[GENO_NKERNELS] = {"init",     "normal_x", "normal_y", "faces_x",
                                           "faces_y",  "slow",     "update_1", "update_2",
                                           "faces_1d", "gate",     "normal_xy",
                                           "fused_x",  "fused_y"};

// Every launch goes through here: a kernel of kind >= 0 is timed while
// timing is enabled (events bound to the dispatch itself).
template <typename... KArgs, typename... Args>
hipError_t launch_bs(int kind, void (*kern)(KArgs...), unsigned grid, unsigned bs, hipStream_t s,
                     Args&&... args) {
  std::tuple<KArgs...> tup = validateArgsCountType(kern, std::tuple<Args...>{args...});
  void* argv[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
  pArgs<0>(tup, argv);
  if (kind >= 0 && !g_tim_suspend && g_tim.used < g_tim.cap) {
    const int u = g_tim.used++;
    g_tim.kind[u] = kind;
    return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(bs), argv, 0,
                              s, g_tim.ev[2 * u], g_tim.ev[2 * u + 1], 0);
  }
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(bs), argv, 0, s);
}

template <typename... KArgs, typename... Args>
hipError_t launch(int kind, void (*kern)(KArgs...), unsigned grid, hipStream_t s, Args&&... args) {
  return launch_bs(kind, kern, grid, BLOCK, s, std::forward<Args>(args)...);
}

// Work counting: per-block sums of the work classes, [kind][class][cap]
// slots, one slot per work-group of a launch (no atomics). p == nullptr when
// counting is off.
struct Cnt {
  unsigned long long* p;
  int cap;
};
struct CountBuf {
  unsigned long long* p = nullptr;
  int cap = 0;
  int on = 0;
  int dev = -1;
};
CountBuf g_cnt;

__device__ void block_count(const Cnt& c, int kind, const unsigned int (&v)[GENO_NCLASS]) {
  __shared__ unsigned int red[MAXWAVES][GENO_NCLASS];
  const int nw = (int)(blockDim.x >> 6);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < GENO_NCLASS; ++q) {
    unsigned int x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[w][q] = x;
  }
  __syncthreads();
  if (threadIdx.x < GENO_NCLASS) {
    unsigned long long x = 0;
#pragma unroll
    for (int i = 0; i < nw; ++i) x += red[i][threadIdx.x];
    if (x) c.p[((size_t)kind * GENO_NCLASS + threadIdx.x) * c.cap + blockIdx.x] += x;
  }
}

// Work-group index remapped so that each of the 8 XCDs (which receive the
// work-groups of a launch round-robin and each have their own L2) processes
// one contiguous slab of the index space: neighbouring rows, which share
// stencil data, then meet in the same L2.
__device__ __forceinline__ int xcd_block() {
  constexpr int NXCD = 8;
  const int nb = (int)gridDim.x, p = (int)blockIdx.x;
  const int per = nb / NXCD, rem = nb % NXCD, x = p % NXCD;
  return x * per + min(x, rem) + p / NXCD;
}

// Geometry passed to the kernels by value.
struct Geo {
  int nx, ny, pitch, rows, yoff, nv;
  int bc[4];
  double dx, dy;
};

__host__ __device__ __forceinline__ size_t at(const Geo& g, int f, int j, int i) {
  return ((size_t)f * g.rows + (j + g.yoff)) * g.pitch + (i + NG);
}

// Row pitch of the 2-D x-face flux buffer: the nx + 1 faces of a row padded
// to a multiple of 8, so that the 8-face pieces of a row that the fused
// x-face tiles write start on 64-byte boundaries (a piece across two
// 64-byte segments was written as two).
__host__ __device__ __forceinline__ int xface_pitch(int nx) { return (nx + 8) & ~7; }

// Control block at the start of the workspace.
struct Ctrl {
  double dt;                        // time step of the current step
  unsigned long long guard;         // positivity fall-backs
  unsigned long long nonfinite;     // non-physical cells (non-finite, rho <= 0 or p <= 0) after a stage-2 update
  unsigned int qcount[2];           // queued tau > 0 faces per direction
};

__device__ __forceinline__ double dt_of(const Ctrl* c) { return c->dt; }

// ---------------------------------------------------------------------------
// Ghost cells. Periodic: copy of the periodic image (values and gradients).
// Transmissive: nearest interior cell, gradient normal to that boundary = 0.
// Reflecting wall: mirror image (ghost -1 of cell 0, -2 of cell 1): the
// normal momentum changes sign; a derivative normal to the wall changes sign
// unless its field is the normal momentum, a tangential one changes sign with
// its field. A corner takes both rules (the same as filling x-ghosts of the
// interior rows and then y-ghosts of every column). Every interior cell
// writes the ghost cells whose source it is.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ghost_src(int gi, int n, int bc_lo, int bc_hi) {
  // fixed ends: no interior cell is the source (the caller owns those ghosts)
  if ((gi < 0 && bc_lo == GENO_BC_FIXED) || (gi >= n && bc_hi == GENO_BC_FIXED)) return -1;
  if (gi < 0) {
    if (bc_lo == GENO_BC_PERIODIC) return gi + n;
    return bc_lo == GENO_BC_REFLECTING ? -gi - 1 : 0;
  }
  if (bc_hi == GENO_BC_PERIODIC) return gi - n;
  return bc_hi == GENO_BC_REFLECTING ? 2 * n - 1 - gi : n - 1;
}

// The boundary rule of one side applied to a copied state: axis 0 (x) or 1
// (y); w, dx, dy: values and the x and y derivatives (dy unused in 1-D).
template <int NV, typename T>
__device__ __forceinline__ void ghost_rule(int bc, int axis, double* w, T* dx, T* dy) {
  if (bc == GENO_BC_TRANSMISSIVE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (axis == 0) dx[v] = T(0);
      else dy[v] = T(0);
    }
  } else if (bc == GENO_BC_REFLECTING) {
    const int m = 1 + axis;   // normal momentum
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const bool odd = v == m;
      if (odd) w[v] = -w[v];
      // normal derivative: sign of the field times -1; tangential: the field's sign
      if (axis == 0) {
        if (!odd) dx[v] = -dx[v];
        if constexpr (NV == 4) if (odd) dy[v] = -dy[v];
      } else {
        if (!odd) dy[v] = -dy[v];
        if (odd) dx[v] = -dx[v];
      }
    }
  }
}

template <int NDIM, typename T>
__device__ __forceinline__ void scatter_ghosts(const Geo& g, double* __restrict__ W,
                                               T* __restrict__ dW, int j, int i, const double* w,
                                               const T* dw) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  // ghost columns / rows whose source is this cell, as bit masks
  const int cx[4] = {-2, -1, g.nx, g.nx + 1};
  const int cy[4] = {-2, -1, g.ny, g.ny + 1};
  unsigned mx = 0, my = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (ghost_src(cx[q], g.nx, g.bc[0], g.bc[1]) == i) mx |= 1u << q;
    if (NDIM == 2 && ghost_src(cy[q], g.ny, g.bc[2], g.bc[3]) == j) my |= 1u << q;
  }
  if (!mx && !my) return;
  // index 4 stands for the cell's own row / column
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    if (a < 4 && !((my >> a) & 1u)) continue;
    const int jj = a == 4 ? j : cy[a];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      if ((b < 4 && !((mx >> b) & 1u)) || (a == 4 && b == 4)) continue;
      const int ii = b == 4 ? i : cx[b];
      double wg[NV];
      T gx[NV], gy[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        wg[v] = w[v];
        gx[v] = dw[v];
        gy[v] = NDIM == 2 ? dw[NV + v] : T(0);
      }
      if (b < 4) ghost_rule<NV, T>(g.bc[b < 2 ? 0 : 1], 0, wg, gx, gy);
      if (a < 4) ghost_rule<NV, T>(g.bc[a < 2 ? 2 : 3], 1, wg, gx, gy);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        W[at(g, v, jj, ii)] = wg[v];
        dW[at(g, v, jj, ii)] = gx[v];
        if constexpr (NDIM == 2) dW[at(g, NV + v, jj, ii)] = gy[v];
      }
    }
  }
}

// a x + b y with both products rounded before the sum (no fused multiply-add),
// so swapping the pairs (x and y directions of a transposed grid) gives the
// same bits
__device__ __forceinline__ double dot2(double a, double x, double b, double y) {
#pragma clang fp contract(off)
  return a * x + b * y;
}

// CFL bound of one cell: min(dx/(|U|+c), dy/(|V|+c)).
template <int NDIM>
__device__ __forceinline__ double cell_tmin(const Geo& g, const double* w, double gamma) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  const double rho = w[0], ir = 1.0 / rho, U = w[1] * ir;
  const double V = NV == 4 ? w[2] * ir : 0.0;
  const double p = (gamma - 1.0) * (w[NV - 1] - 0.5 * rho * dot2(U, U, V, V));
  const double c = sqrt(gamma * p * ir);
  // min(dx / (|U| + c), dy / (|V| + c)) over the common numerator dx dy
  double t;
  if constexpr (NDIM == 2) t = (g.dx * g.dy) / fmax((fabs(U) + c) * g.dy, (fabs(V) + c) * g.dx);
  else t = g.dx / (fabs(U) + c);
  return (t > 0.0) ? t : 0.0;   // a NaN state gives a zero step (flagged by the caller)
}

// block minimum of t into part[slot]
__device__ __forceinline__ void block_min(double t, double* part, int slot) {
  __shared__ double red[MAXWAVES];
  const int nw = (int)(blockDim.x >> 6);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t = fmin(t, __shfl_xor(t, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
#pragma unroll
    for (int w = 1; w < nw; ++w) m = fmin(m, red[w]);
    part[slot] = m;
  }
}

// dt of the step into ctrl->dt (one block): cfl times the minimum of the
// npart partials, or dt_fixed if positive; records dt
__device__ __forceinline__ void reduce_dt(const double* part, int npart, Ctrl* ctrl, double cfl,
                                          double dt_fixed, double* dt_out, int step) {
  __shared__ double red[MAXWAVES];
  const int nw = (int)(blockDim.x >> 6);
  double m = INFINITY;
  for (int q = threadIdx.x; q < npart; q += blockDim.x) m = fmin(m, part[q]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = red[0];
    for (int w = 1; w < nw; ++w) m = fmin(m, red[w]);
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * m;
    ctrl->dt = dt;
    if (dt_out) dt_out[step] = dt;
  }
}

// Start of gks_step: ghost cells of the initial state, per-block CFL minima,
// cleared counters.
// (lb: the work-group's index within this grid's launch range; the kernel
// bodies below all take one.)
template <int NDIM, typename T>
__device__ __forceinline__ void init_body(const Geo& g, double gamma, double* __restrict__ W,
                                          T* __restrict__ dW, double* __restrict__ part,
                                          Ctrl* ctrl, int lb) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  const int t = lb * (int)blockDim.x + (int)threadIdx.x;
  if (lb == 0) {
    unsigned long long* z = &ctrl->guard;
    const int nz = (int)((sizeof(Ctrl) - offsetof(Ctrl, guard)) / sizeof(unsigned long long));
    for (int q = threadIdx.x; q < nz; q += blockDim.x) z[q] = 0;
  }
  double tl = INFINITY;
  if (t < g.nx * g.ny) {
    const int j = t / g.nx, i = t % g.nx;
    double w[NV];
    T dw[NV * NDIM];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = W[at(g, v, j, i)];
#pragma unroll
    for (int v = 0; v < NV * NDIM; ++v) dw[v] = dW[at(g, v, j, i)];
    scatter_ghosts<NDIM, T>(g, W, dW, j, i, w, dw);
    tl = cell_tmin<NDIM>(g, w, gamma);
  }
  block_min(tl, part, lb);
}

template <int NDIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_init(Geo g, double gamma, double* __restrict__ W,
                                                T* __restrict__ dW, double* __restrict__ part,
                                                Ctrl* ctrl) {
  init_body<NDIM, T>(g, gamma, W, dW, part, ctrl, (int)blockIdx.x);
}

// Normal GENO of one face-row entry o = a * n1 + b (indexing as normal_body)
// on characteristic variables: the stencil's four cells, values and
// h-scaled normal derivatives, in the normal frame (rho, rho un, rho ut,
// rho E), projected on the left eigenvectors at the Roe average of the two
// cells at the face (m = 1, 2), reconstructed field by field and mapped back
// with the right ones. A face whose average has no real sound speed keeps
// the conservative variables. Returns the sides on the low-order branch.
template <int DIR, typename T>
__device__ __forceinline__ unsigned int normal_char(const Geo& g, const geno::KParams& k,
                                                    const double* __restrict__ W,
                                                    const T* __restrict__ dW,
                                                    T* __restrict__ fr,
                                                    double* __restrict__ chi, int o, int n1,
                                                    int plane) {
  const int a = o / n1, b = o - a * n1;
  const double h = DIR == 0 ? g.dx : g.dy;
  // state variable of each normal-frame slot
  constexpr int VM[4] = {0, DIR == 0 ? 1 : 2, DIR == 0 ? 2 : 1, 3};
  double Qv[4][4], Gv[4][4];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t id;
      if (DIR == 0) id = at(g, VM[f], a - 1, b - 2 + m);
      else id = at(g, VM[f], a - 2 + m, b - 1);
      Qv[f][m] = W[id];
      Gv[f][m] = h * (double)dW[id + (size_t)(DIR * 4) * g.rows * g.pitch];
    }
  const double Wa[4] = {Qv[0][1], Qv[1][1], Qv[2][1], Qv[3][1]};
  const double Wb[4] = {Qv[0][2], Qv[1][2], Qv[2][2], Qv[3][2]};
  geno::Eig2 e;
  const bool ch = geno::roe_eigen2(Wa, Wb, k.gamma, e);
  unsigned int nlow = 0;
  double wv[2][4], wd[2][4], w2[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (ch) {
        Q[m] = e.L[c][0] * Qv[0][m] + e.L[c][1] * Qv[1][m] + e.L[c][2] * Qv[2][m] +
               e.L[c][3] * Qv[3][m];
        G[m] = e.L[c][0] * Gv[0][m] + e.L[c][1] * Gv[1][m] + e.L[c][2] * Gv[2][m] +
               e.L[c][3] * Gv[3][m];
      } else {
        Q[m] = Qv[c][m];
        G[m] = Gv[c][m];
      }
    }
    T vl, dl, vr, dr, h2;
    double xl, xr;
    nlow += geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, vl, dl,
                                       xl, vr, dr, xr, h2);
    wv[0][c] = (double)vl;
    wd[0][c] = (double)dl;
    wv[1][c] = (double)vr;
    wd[1][c] = (double)dr;
    w2[c] = (double)h2;
    if (chi) {
      // characteristic field c, or the state variable of slot c
      const int cv = ch ? c : VM[c];
      chi[(size_t)(0 * 4 + cv) * plane + o] = xl;
      chi[(size_t)(1 * 4 + cv) * plane + o] = xr;
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double Sv[4], Dv[4];
    if (ch) {
      geno::from_characteristic2(e, wv[s], Sv);
      geno::from_characteristic2(e, wd[s], Dv);
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        Sv[f] = wv[s][f];
        Dv[f] = wd[s][f];
      }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      __builtin_nontemporal_store(T(Sv[f]), &fr[(size_t)((2 * s + 0) * 4 + VM[f]) * plane + o]);
      __builtin_nontemporal_store(T(Dv[f]), &fr[(size_t)((2 * s + 1) * 4 + VM[f]) * plane + o]);
    }
  }
  // the mean of the two sides' h^2 * second derivatives, mapped back like
  // the states (the map is linear and common to both sides)
  double S2[4];
  if (ch) {
    geno::from_characteristic2(e, w2, S2);
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) S2[f] = w2[f];
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) __builtin_nontemporal_store(T(S2[f]), &fr[(size_t)(16 + VM[f]) * plane + o]);
  return nlow;
}

// ---------------------------------------------------------------------------
// Normal GENO on face-rows (2-D), one thread per (variable, face-row entry).
// DIR 0: rows a = 0..ny+1 (j = a-1), faces b = 0..nx (between cells b-1 and
// b). DIR 1: faces a = 0..ny (between rows a-1 and a), columns b = 0..nx+1
// (i = b-1). Thread index (v, a, b) with b fastest, so that a wave reads and
// writes 64 consecutive entries of one plane.
// fr: [side][quant(value, h d/dn)][var][a][b] (16 planes), then the mean
// over the two sides of h^2 d^2/dn^2, [var][a][b] (4 planes); chi:
// [side][var][a][b].
// With part (first kernel of a step), block 0 also reduces the CFL partial
// minima of the previous kernel into ctrl->tmin and records dt.
// ---------------------------------------------------------------------------
// gate: the learned gate's flags of the interior cells for this direction
// ([ny][nx], 1 = chi of the cell's sides is 1), or nullptr.
// CHAR: characteristic variables, one thread per face-row entry (all four
// variables of its stencil are needed for the projection); chi then holds
// the characteristic fields (un - c, un, shear, un + c).
template <int DIR, typename T, bool CHAR = false>
__device__ __forceinline__ void normal_body(const Geo& g, const geno::KParams& k,
                                            const double* __restrict__ W,
                                            const T* __restrict__ dW, T* __restrict__ fr,
                                            double* __restrict__ chi, Ctrl* ctrl,
                                            const double* __restrict__ part, int npart,
                                            double* dt_out, int step, const Cnt& cnt, int lb,
                                            const unsigned char* __restrict__ gate = nullptr) {
  if (part && lb == 0) reduce_dt(part, npart, ctrl, k.cfl, k.dt_fixed, dt_out, step);
  if (ctrl && lb == 0 && threadIdx.x == 0) ctrl->qcount[DIR] = 0;
  const int n1 = DIR == 0 ? g.nx + 1 : g.nx + 2;
  const int n0 = DIR == 0 ? g.ny + 2 : g.ny + 1;
  const int plane = n0 * n1;
  const int t = lb * (int)blockDim.x + (int)threadIdx.x;
  unsigned int nlow = 0, ngated = 0;
  const int nent = CHAR ? plane : 4 * plane;
  if constexpr (CHAR) {
    if (t < plane) nlow = normal_char<DIR, T>(g, k, W, dW, fr, chi, t, n1, plane);
  } else if (t < nent) {
    const int v = t / plane, o = t - v * plane;
    const int a = o / n1, b = o - a * n1;
    const double h = DIR == 0 ? g.dx : g.dy;
    bool skipL = false, skipR = false;
    if (gate) {
      // cells of the two sides: DIR 0 (row a-1; columns b-1, b), DIR 1 (rows a-1, a; column b-1)
      const int jl = DIR == 0 ? a - 1 : a - 1, il = DIR == 0 ? b - 1 : b - 1;
      const int jr = DIR == 0 ? a - 1 : a, ir = DIR == 0 ? b : b - 1;
      if (jl >= 0 && jl < g.ny && il >= 0 && il < g.nx) skipL = gate[jl * g.nx + il] != 0;
      if (jr >= 0 && jr < g.ny && ir >= 0 && ir < g.nx) skipR = gate[jr * g.nx + ir] != 0;
      ngated = (skipL ? 1u : 0u) + (skipR ? 1u : 0u);
    }
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t id;
      if (DIR == 0) id = at(g, v, a - 1, b - 2 + m);
      else id = at(g, v, a - 2 + m, b - 1);
      Q[m] = W[id];
      G[m] = h * (double)dW[id + (size_t)(DIR * 4) * g.rows * g.pitch];
    }
    T vl, dl, vr, dr, h2;
    double xl, xr;
    nlow = geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, vl, dl,
                                      xl, vr, dr, xr, h2, skipL, skipR);
    // face-row and face buffers are written once and read by the next
    // launch: streamed past the caches (non-temporal stores)
    __builtin_nontemporal_store(vl, &fr[(size_t)(0 * 4 + v) * plane + o]);
    __builtin_nontemporal_store(dl, &fr[(size_t)(1 * 4 + v) * plane + o]);
    __builtin_nontemporal_store(vr, &fr[(size_t)(2 * 4 + v) * plane + o]);
    __builtin_nontemporal_store(dr, &fr[(size_t)(3 * 4 + v) * plane + o]);
    __builtin_nontemporal_store(h2, &fr[(size_t)(16 + v) * plane + o]);
    if (chi) {
      chi[(size_t)(0 * 4 + v) * plane + o] = xl;
      chi[(size_t)(1 * 4 + v) * plane + o] = xr;
    }
  }
  if (cnt.p) {
    unsigned int wc[GENO_NCLASS] = {};
    wc[GENO_W_UNITS] = t < nent ? (CHAR ? 4u : 1u) : 0u;
    wc[GENO_W_LOW] = nlow;
    wc[GENO_W_GATED] = ngated;
    block_count(cnt, DIR == 0 ? GENO_K_NORMAL_X : GENO_K_NORMAL_Y, wc);
  }
}

template <int DIR, typename T, bool CHAR>
__global__ void __launch_bounds__(BLOCK) k_normal2d(Geo g, geno::KParams k,
                                                    const double* __restrict__ W,
                                                    const T* __restrict__ dW,
                                                    T* __restrict__ fr,
                                                    double* __restrict__ chi, Ctrl* ctrl,
                                                    const double* __restrict__ part, int npart,
                                                    double* dt_out, int step, Cnt cnt,
                                                    const unsigned char* __restrict__ gate) {
  normal_body<DIR, T, CHAR>(g, k, W, dW, fr, chi, ctrl, part, npart, dt_out, step, cnt,
                            xcd_block(), gate);
}

// The paper's comparison of the nonlinear weights at every face-side of a
// direction, from the same stencils as the normal step: chi of GENO (its
// path function), of WENO-Z and of TENO (geno_device.hpp). One thread per
// (variable, face-row entry) as in normal_body; 1-D uses the x-direction
// indexing on its single row. out: [method][side][var][a][b], method 0 GENO,
// 1 WENO-Z, 2 TENO.
template <int DIR, typename T>
__global__ void __launch_bounds__(BLOCK) k_linearity(Geo g, geno::KParams k, int ndim,
                                                     const double* __restrict__ W,
                                                     const T* __restrict__ dW,
                                                     double* __restrict__ out, double ct) {
  const int nv = ndim == 2 ? 4 : 3;
  const int n1 = DIR == 0 ? g.nx + 1 : g.nx + 2;
  const int n0 = ndim == 1 ? 1 : (DIR == 0 ? g.ny + 2 : g.ny + 1);
  const int plane = n0 * n1;
  const int t = xcd_block() * (int)blockDim.x + (int)threadIdx.x;
  if (t >= nv * plane) return;
  const int v = t / plane, o = t - v * plane;
  const int a = o / n1, b = o - a * n1;
  const double h = DIR == 0 ? g.dx : g.dy;
  double Q[4], G[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    size_t id;
    if (DIR == 0) id = at(g, v, ndim == 1 ? 0 : a - 1, b - 2 + m);
    else id = at(g, v, a - 2 + m, b - 1);
    Q[m] = W[id];
    G[m] = h * (double)dW[id + (size_t)(DIR * nv) * g.rows * g.pitch];
  }
  const size_t mplane = (size_t)2 * nv * plane;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    // the right state is the left-state formula on the data mirrored about the face
    const geno::SideQuads<double> sq =
        side == 0 ? geno::side_quads<double>(Q[0], Q[1], Q[2], Q[3], G[0])
                  : geno::side_quads<double>(Q[3], Q[2], Q[1], Q[0], -G[3]);
    const double ISH = fmax(sq.IS1, fmax(sq.IS2, sq.IS3));
    const double ISL = fmin(sq.IS1, fmin(sq.IS2, sq.IS3));
    const double IStau = fabs(0.5 * (sq.IS2 + sq.IS3) - sq.IS1);
    const size_t e = ((size_t)side * nv + v) * plane + o;
    out[0 * mplane + e] = geno::path_chi<double>(IStau, ISH, ISL, k.eps, k);
    out[1 * mplane + e] = geno::wenoz_chi<double>(sq.IS1, sq.IS2, sq.IS3, k);
    out[2 * mplane + e] = geno::teno_chi<double>(sq.IS1, sq.IS2, sq.IS3, ct, k);
  }
}

// ---------------------------------------------------------------------------
// Faces (2-D), two lanes per face: lane q owns Gauss point q and computes the
// tangential step of side q for both points; the halves are exchanged with
// the partner lane. DIR 0: face (a = row t, b = face 0..nx); DIR 1: face
// (a = face 0..ny, b = column t).
// MODE 0: write the point states (geno_reconstruct).
// MODE 1: flux for tau = 0; faces with tau > 0 at either point are queued.
// MODE 2: flux of the queued faces with the full solution (grid-stride).
// Second derivatives of a point (time stepping of the gradients): h_n^2 d_nn
// is the normal step's mean of row t; per side h_t^2 d_tt = chi_t D2 and
// h_n h_t d_nt = chi_t (psi_{t+1} - psi_{t-1})/2 from the tangential step of
// the value (chi_t, D2) and the h-scaled normal derivatives psi of the three
// rows; the point takes the mean of the two sides, and zero if a side is
// guarded.
// Flux outputs, Gauss-averaged, [kind][var][face]: stage 1 (want_F) F, dF/dt,
// W(dt/2) + dt^2/8 W_tt and W(dt) + dt^2/6 W_tt (the interface values at the
// stage time and the first part of those at the end of the step); stage 2
// dF/dt in kind 1 and W_tt in kind 2.
// ---------------------------------------------------------------------------
// Value of the partner lane (lane ^ 1) by a DPP quad permutation [1, 0, 3, 2]
// (a VALU move, no trip through LDS). Both lanes of a pair are always active
// together.
__device__ __forceinline__ int pair_swap(int x) {
  return __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(pair_swap(__float_as_int(x)));
}
__device__ __forceinline__ double pair_swap(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned int lo = (unsigned int)pair_swap((int)(unsigned int)(u & 0xffffffffull));
  const unsigned int hi = (unsigned int)pair_swap((int)(unsigned int)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int DIR>
struct FaceGeo {
  int n0, n1, r0, r1;
  __device__ explicit FaceGeo(const Geo& g) {
    n1 = DIR == 0 ? g.nx + 1 : g.nx;
    n0 = DIR == 0 ? g.ny : g.ny + 1;
    r1 = DIR == 0 ? g.nx + 1 : g.nx + 2;
    r0 = DIR == 0 ? g.ny + 2 : g.ny + 1;
  }
};

// What the tangential step of one face side reads, through an accessor:
// v(i, f), d(i, f) the side's value and h-scaled normal derivative of
// variable f on the face rows t-1, t, t+1 (i = 0, 1, 2), h2(f) the normal
// step's two-side mean of h^2 d^2/dn^2 on row t. Each element is read where
// it is used.
// From the face-row buffer (layout of normal_body).
template <typename T>
struct RowsMem {
  const T* fr;
  size_t plane, r[3];
  int q;
  __device__ T v(int i, int f) const { return fr[(size_t)((2 * q + 0) * 4 + f) * plane + r[i]]; }
  __device__ T d(int i, int f) const { return fr[(size_t)((2 * q + 1) * 4 + f) * plane + r[i]]; }
  __device__ T h2(int f) const { return fr[(size_t)(16 + f) * plane + r[1]]; }
};
// The same values loaded all at once (one round trip to memory instead of
// one per variable), for the queue kernel: with one wave per SIMD nothing
// else hides the latency of its loads.
template <typename T>
struct RowsReg {
  T vv[3][4], dd[3][4], hh[4];
  __device__ explicit RowsReg(const RowsMem<T>& m) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        vv[i][f] = m.v(i, f);
        dd[i][f] = m.d(i, f);
      }
#pragma unroll
    for (int f = 0; f < 4; ++f) hh[f] = m.h2(f);
  }
  __device__ T v(int i, int f) const { return vv[i][f]; }
  __device__ T d(int i, int f) const { return dd[i][f]; }
  __device__ T h2(int f) const { return hh[f]; }
};
// From LDS: element (i, quantity, f) at p[o[i] + (quantity * 4 + f) * st],
// h2(f) at p[oh + f * st].
template <typename T>
struct RowsLds {
  const T* p;
  int o[3], oh, st;
  __device__ T v(int i, int f) const { return p[o[i] + f * st]; }
  __device__ T d(int i, int f) const { return p[o[i] + (4 + f) * st]; }
  __device__ T h2(int f) const { return p[oh + f * st]; }
};

// Face-row offsets of face (a, b): rows t-1, t, t+1 of its side data.
template <int DIR>
struct FaceRows {
  size_t plane, rm, rc, rp;
  __device__ FaceRows(const FaceGeo<DIR>& fg, int a, int b) {
    plane = (size_t)fg.r0 * fg.r1;
    rm = (size_t)a * fg.r1 + b;
    rc = DIR == 0 ? rm + fg.r1 : rm + 1;
    rp = DIR == 0 ? rc + fg.r1 : rc + 1;
  }
};

// The face step of lane q of a pair from its side's rows sr. Returns true
// (MODE 1) when the face is valid and was queued for the full solution.
// NTS: flux outputs written with non-temporal stores (streamed past the
// caches to the update that reads them).
template <int DIR, int MODE, typename T, typename Rows, bool NTS = true>
__device__ __forceinline__ bool face_core(const Geo& g, const geno::KParams& k,
                                          const double* __restrict__ W, T* __restrict__ out,
                                          Ctrl* ctrl, int want_F, unsigned int (&wc)[GENO_NCLASS],
                                          int face, bool valid, unsigned int* __restrict__ queue,
                                          const Rows& sr) {
  const FaceGeo<DIR> fg(g);
  const int q = threadIdx.x & 1;
  const int nfaces = fg.n0 * fg.n1;
  const int fc = valid ? face : nfaces - 1;
  const int a = fc / fg.n1, b = fc % fg.n1;
  // tangential step of side q for both points, and the side's second
  // tangential and cross derivatives
  T own_v[4], own_t[4], snd_v[4], snd_t[4], dn[4], s_tt[4], s_nt[4];
  unsigned int nlow = 0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T v0, v1, t0, t1, cht, d2;
    nlow += geno::tangential<T, double>(sr.v(0, v), sr.v(1, v), sr.v(2, v), k, v0, v1, t0, t1,
                                        cht, d2);
    own_v[v] = q ? v1 : v0;
    own_t[v] = q ? t1 : t0;
    snd_v[v] = q ? v0 : v1;
    snd_t[v] = q ? t0 : t1;
    dn[v] = sr.d(1, v);
    s_tt[v] = cht * d2;
    s_nt[v] = cht * (T(0.5) * (sr.d(2, v) - sr.d(0, v)));
  }
  // states of both sides at this lane's point
  T S[2][4], Dn[2][4], Dt[2][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T rv = pair_swap(snd_v[v]);
    const T rt = pair_swap(snd_t[v]);
    const T rd = pair_swap(dn[v]);
    S[0][v] = q ? rv : own_v[v];
    S[1][v] = q ? own_v[v] : rv;
    Dt[0][v] = q ? rt : own_t[v];
    Dt[1][v] = q ? own_t[v] : rt;
    Dn[0][v] = q ? rd : dn[v];
    Dn[1][v] = q ? dn[v] : rd;
    // the mean of the two sides (the same sum in both lanes)
    s_tt[v] = T(0.5) * (s_tt[v] + pair_swap(s_tt[v]));
    s_nt[v] = T(0.5) * (s_nt[v] + pair_swap(s_nt[v]));
  }
  // positivity guard per side: fall back to the own cell average
  unsigned int nguard = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!geno::admissible<4, T>(S[s], k.gamma)) {
      ++nguard;
      const int ci = DIR == 0 ? b - 1 + s : b;
      const int cj = DIR == 0 ? a : a - 1 + s;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        S[s][v] = T(W[at(g, v, cj, ci)]);
        Dn[s][v] = T(0);
        Dt[s][v] = T(0);
      }
    }
  }
  T s_nn[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    s_nn[v] = nguard ? T(0) : sr.h2(v);
    if (nguard) s_tt[v] = s_nt[v] = T(0);
  }
  if (!valid) nguard = nlow = 0;
  // face_state (MODE 0) and the y-face buffer are compact; the x-face flux
  // buffer has padded rows
  const bool padded = MODE != 0 && DIR == 0;
  const size_t plane = padded ? (size_t)fg.n0 * xface_pitch(g.nx) : (size_t)nfaces;
  const size_t o = padded ? (size_t)a * xface_pitch(g.nx) + b : (size_t)fc;
  bool queued = false;
  if constexpr (MODE == 0) {
    if (valid) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t base = (size_t)(((s * 2 + q) * 3) * 4);
          out[(base + 0 * 4 + v) * plane + o] = S[s][v];
          out[(base + 1 * 4 + v) * plane + o] = Dn[s][v];
          out[(base + 2 * 4 + v) * plane + o] = Dt[s][v];
        }
      // second derivatives of this lane's point, after the 48 state planes
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const size_t base = (size_t)48 + (size_t)(q * 3) * 4;
        out[(base + 0 * 4 + v) * plane + o] = s_nn[v];
        out[(base + 1 * 4 + v) * plane + o] = s_nt[v];
        out[(base + 2 * 4 + v) * plane + o] = s_tt[v];
      }
    }
  } else {
    const double dt = dt_of(ctrl);
    const double hn = DIR == 0 ? g.dx : g.dy, ht = DIR == 0 ? g.dy : g.dx;
    const T ihn = T(1.0 / hn), iht = T(1.0 / ht);
    const T inn = T(1.0 / (hn * hn)), int_ = T(1.0 / (hn * ht)), itt = T(1.0 / (ht * ht));
    constexpr int p1 = DIR == 0 ? 1 : 2, p2 = DIR == 0 ? 2 : 1;
    constexpr int perm[4] = {0, p1, p2, 3};
    T Wl[4], Wr[4], nl[4], nr[4], tl[4], tr[4], xnn[4], xnt[4], xtt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wl[v] = S[0][perm[v]];
      Wr[v] = S[1][perm[v]];
      nl[v] = Dn[0][perm[v]] * ihn;
      nr[v] = Dn[1][perm[v]] * ihn;
      tl[v] = Dt[0][perm[v]] * iht;
      tr[v] = Dt[1][perm[v]] * iht;
      xnn[v] = s_nn[perm[v]] * inn;
      xnt[v] = s_nt[perm[v]] * int_;
      xtt[v] = s_tt[perm[v]] * itt;
    }
    gks::PointOut<4, T> po;
    int pk;   // point kind; MODE 1: PT_SLOW not evaluated; MODE 2: evaluated
    if constexpr (MODE == 1)
      pk = gks::point_flux<4, false, T>(Wl, Wr, nl, nr, tl, tr, xnn, xnt, xtt, dt, k, want_F != 0,
                                        po);
    else
      pk = gks::point_flux<4, true, T>(Wl, Wr, nl, nr, tl, tr, xnn, xnt, xtt, dt, k, want_F != 0,
                                       po);
    const bool slow = pk == gks::PT_SLOW;
    bool pair_slow = false;
    if constexpr (MODE == 1) {
      // every lane takes part in the exchange (no short-circuit around it:
      // a lane that skips a cross-lane read leaves its partner reading an
      // inactive lane)
      const int partner_slow = pair_swap(slow ? 1 : 0);
      pair_slow = slow || partner_slow != 0;
      // queue the faces that need the full solution (one atomic per wave)
      const bool enq = valid && q == 0 && pair_slow;
      const unsigned long long m = __ballot(enq);
      unsigned int base = 0;
      if ((threadIdx.x & 63) == 0 && m)
        base = atomicAdd(&ctrl->qcount[DIR], (unsigned int)__popcll(m));
      base = __shfl(base, 0, 64);
      if (enq) {
        const unsigned int rank = (unsigned int)__popcll(m & ((1ull << (threadIdx.x & 63)) - 1));
        queue[base + rank] = (unsigned int)face;
      }
      queued = valid && pair_slow;
    }
    if (nguard && (MODE == 2 || !pair_slow)) atomicAdd(&ctrl->guard, (unsigned long long)nguard);
    // this point's share of the Gauss average (weights 1/2) of the stage's
    // four outputs: stage 1 F, dF/dt, W(dt/2) + dt^2/8 W_tt, W(dt) + dt^2/6
    // W_tt; stage 2 -, dF/dt, W_tt, -. Results of a PT_SLOW point in MODE 1
    // are not formed (the face is written by MODE 2).
    T So[16];
    const T c8 = T(dt * dt / 8.0), c6 = T(dt * dt / 6.0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (slow && MODE == 1) {
        So[v] = So[4 + v] = So[8 + v] = So[12 + v] = T(0);
      } else if (want_F) {
        So[v] = T(0.5) * po.F[v];
        So[4 + v] = T(0.5) * po.Ft[v];
        So[8 + v] = T(0.5) * (po.Wh[v] + c8 * po.Wtt[v]);
        So[12 + v] = T(0.5) * (po.Wf[v] + c6 * po.Wtt[v]);
      } else {
        So[v] = So[12 + v] = T(0);
        So[4 + v] = T(0.5) * po.Ft[v];
        So[8 + v] = T(0.5) * po.Wtt[v];
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) So[e] = So[e] + pair_swap(So[e]);
    if (valid && !pair_slow) {
      // back to the (x, y) frame; lane 0 writes kinds 0, 1 and lane 1 kinds
      // 2, 3 (stage 2: lane 0 dF/dt, lane 1 W_tt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pv = perm[v];
        auto put = [&](int kind, T x) {
          T* dst = &out[(size_t)(kind * 4 + pv) * plane + o];
          if constexpr (NTS) __builtin_nontemporal_store(x, dst);
          else *dst = x;
        };
        if (q == 0) {
          if (want_F) put(0, So[v]);
          put(1, So[4 + v]);
        } else {
          put(2, So[8 + v]);
          if (want_F) put(3, So[12 + v]);
        }
      }
    }
    // work classes of this lane (a pair queued for the full solution is
    // counted where it is evaluated)
    const bool ev = valid && !pair_slow;
    wc[GENO_W_UNITS] += (ev && q == 0) ? 1u : 0u;
    wc[GENO_W_EQUAL] += (ev && pk == gks::PT_EQUAL) ? 1u : 0u;
    wc[GENO_W_FAST] += (ev && pk == gks::PT_FAST) ? 1u : 0u;
    wc[GENO_W_SLOW] += (ev && slow) ? 1u : 0u;
    wc[GENO_W_LOW] += ev ? nlow : 0u;
    wc[GENO_W_GUARD] += ev ? nguard : 0u;
  }
  return queued;
}

// A queued face's rows into the face-row buffer fr (layout of normal_body),
// where the queue kernel reads them; neighbouring queued faces write equal
// values to the entries they share. Called after face_core so that the rows
// are read again from LDS here, not held in registers through the flux.
template <int DIR, typename T, typename Rows>
__device__ __forceinline__ void spill_rows(const Geo& g, int face, const Rows& sr,
                                           T* __restrict__ fr) {
  const FaceGeo<DIR> fg(g);
  const int q = threadIdx.x & 1;
  const FaceRows<DIR> fw(fg, face / fg.n1, face % fg.n1);
  const size_t rr[3] = {fw.rm, fw.rc, fw.rp};
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      fr[(size_t)((2 * q + 0) * 4 + v) * fw.plane + rr[i]] = sr.v(i, v);
      fr[(size_t)((2 * q + 1) * 4 + v) * fw.plane + rr[i]] = sr.d(i, v);
    }
  if (q == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) fr[(size_t)(16 + v) * fw.plane + fw.rc] = sr.h2(v);
}

// The face step of lane q with its side's rows read from the face-row
// buffer fr.
template <int DIR, int MODE, typename T>
__device__ __forceinline__ void face_pair(const Geo& g, const geno::KParams& k,
                                          const double* __restrict__ W,
                                          const T* __restrict__ fr, T* __restrict__ out,
                                          Ctrl* ctrl, int want_F, unsigned int (&wc)[GENO_NCLASS],
                                          int face, bool valid, unsigned int* __restrict__ queue) {
  const FaceGeo<DIR> fg(g);
  const int q = threadIdx.x & 1;
  const int nfaces = fg.n0 * fg.n1;
  const int fc = valid ? face : nfaces - 1;
  const FaceRows<DIR> fw(fg, fc / fg.n1, fc % fg.n1);
  const RowsMem<T> sr{fr, fw.plane, {fw.rm, fw.rc, fw.rp}, q};
  if constexpr (MODE == 2) {
    face_core<DIR, MODE, T>(g, k, W, out, ctrl, want_F, wc, face, valid, queue, RowsReg<T>(sr));
  } else {
    face_core<DIR, MODE, T>(g, k, W, out, ctrl, want_F, wc, face, valid, queue, sr);
  }
}

template <int DIR, int MODE, typename T>
__device__ __forceinline__ void faces_body(const Geo& g, const geno::KParams& k,
                                           const double* __restrict__ W,
                                           const T* __restrict__ fr, T* __restrict__ out,
                                           Ctrl* ctrl, int want_F, const Cnt& cnt,
                                           unsigned int* __restrict__ queue, int lb) {
  const FaceGeo<DIR> fg(g);
  const int nfaces = fg.n0 * fg.n1;
  const int t = lb * (int)blockDim.x + (int)threadIdx.x;
  const int face = t >> 1;
  unsigned int wc[GENO_NCLASS] = {};
  face_pair<DIR, MODE, T>(g, k, W, fr, out, ctrl, want_F, wc, face, face < nfaces, queue);
  if (MODE == 1 && cnt.p) block_count(cnt, DIR == 0 ? GENO_K_FACES_X : GENO_K_FACES_Y, wc);
}

// WF: stage 1 (F and the interface values wanted) or stage 2 (dF/dt and
// W_tt only), a template parameter so that each stage's kernel carries only
// its own outputs' arithmetic and registers
template <int DIR, int MODE, typename T, bool WF>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WF ? 1 : 4))) k_faces2d(Geo g, geno::KParams k,
                                                   const double* __restrict__ W,
                                                   const T* __restrict__ fr,
                                                   T* __restrict__ out, Ctrl* ctrl, Cnt cnt,
                                                   unsigned int* __restrict__ queue) {
  faces_body<DIR, MODE, T>(g, k, W, fr, out, ctrl, WF ? 1 : 0, cnt, queue, xcd_block());
}

// The normal step of both directions in one launch: work-groups [0, nbx)
// take the x-direction entries, the rest the y-direction ones (a uniform
// branch per work-group; with the XCD remapping, XCDs 0-3 take x and 4-7
// y). Twice the waves of one direction per launch, and one launch ramp
// less per stage. (The face step stays one launch per direction: over both,
// each XCD's L2 would hold twice the face-row rows it reuses.)
template <typename T, bool CHAR>
__global__ void __launch_bounds__(BLOCK) k_normal2d_xy(Geo g, geno::KParams k,
                                                       const double* __restrict__ W,
                                                       const T* __restrict__ dW,
                                                       T* __restrict__ frx, T* __restrict__ fry,
                                                       Ctrl* ctrl,
                                                       const double* __restrict__ part, int npart,
                                                       double* dt_out, int step, Cnt cnt,
                                                       const unsigned char* __restrict__ gx,
                                                       const unsigned char* __restrict__ gy,
                                                       int nbx) {
  const int b = xcd_block();
  if (b < nbx)
    normal_body<0, T, CHAR>(g, k, W, dW, frx, nullptr, ctrl, part, npart, dt_out, step, cnt, b,
                            gx);
  else
    normal_body<1, T, CHAR>(g, k, W, dW, fry, nullptr, ctrl, nullptr, 0, nullptr, 0, cnt,
                            b - nbx, gy);
}


// The faces of both directions queued by k_faces2d<DIR, 1> (tau > 0 at one
// of their Gauss points), with the full solution: lane pairs as there,
// grid-stride over the pairs; pairs [0, nqx) are x-faces, the rest y-faces.
// Both lanes of a pair always take the same branch and trip count, so each
// cross-lane read finds its partner active.
// (lb, nb: this work-group's index among the nb work-groups serving the grid)
template <typename T>
__device__ __forceinline__ void slow_body(const Geo& g, const geno::KParams& k,
                                          const double* __restrict__ W,
                                          const T* __restrict__ frx, const T* __restrict__ fry,
                                          T* __restrict__ outx, T* __restrict__ outy, Ctrl* ctrl,
                                          int want_F, const Cnt& cnt,
                                          const unsigned int* __restrict__ qx,
                                          const unsigned int* __restrict__ qy, int lb, int nb) {
  const unsigned int nqx = ctrl->qcount[0];
  const unsigned int nq = nqx + ctrl->qcount[1];
  const unsigned int stride = (unsigned int)nb * blockDim.x / 2;
  unsigned int wc[GENO_NCLASS] = {};
  for (unsigned int e = ((unsigned int)lb * blockDim.x + threadIdx.x) >> 1; e < nq; e += stride) {
    if (e < nqx)
      face_pair<0, 2, T>(g, k, W, frx, outx, ctrl, want_F, wc, (int)qx[e], true, nullptr);
    else
      face_pair<1, 2, T>(g, k, W, fry, outy, ctrl, want_F, wc, (int)qy[e - nqx], true, nullptr);
  }
  if (cnt.p) block_count(cnt, GENO_K_SLOW, wc);
}

template <typename T, bool WF>
__global__ void __launch_bounds__(BLOCK) k_slow2d(Geo g, geno::KParams k,
                                                  const double* __restrict__ W,
                                                  const T* __restrict__ frx,
                                                  const T* __restrict__ fry,
                                                  T* __restrict__ outx, T* __restrict__ outy,
                                                  Ctrl* ctrl, Cnt cnt,
                                                  const unsigned int* __restrict__ qx,
                                                  const unsigned int* __restrict__ qy) {
  slow_body<T>(g, k, W, frx, fry, outx, outy, ctrl, WF ? 1 : 0, cnt, qx, qy, (int)blockIdx.x,
               (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// Face step with the normal step on chip (2-D gks_step, conservative
// variables): the face-row values a face needs are computed by the kernel
// that uses them, so the face-row buffer makes no round trip through HBM.
// The arithmetic is that of normal_body and face_pair, so the results are
// bitwise those of the two-launch path.
// ---------------------------------------------------------------------------
// Normal GENO of face-row entry (a, b) (indexing of normal_body) by a lane
// pair: lane q reconstructs variables 2q and 2q+1 (both sides), then the two
// lanes exchange halves so that lane q holds side q of all four variables
// (v, d: value and h-scaled normal derivative) and the two-side mean h2.
template <int DIR, typename T>
__device__ __forceinline__ void normal_pair(const Geo& g, const geno::KParams& k,
                                            const double* __restrict__ W,
                                            const T* __restrict__ dW, int a, int b, int q,
                                            T (&v)[4], T (&d)[4], T (&h2)[4],
                                            bool skipL = false, bool skipR = false) {
  const double h = DIR == 0 ? g.dx : g.dy;
  T sv[2][2], sd[2][2], sh[2];   // [variable 2q + i][side]
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int var = 2 * q + i;
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t id;
      if (DIR == 0) id = at(g, var, a - 1, b - 2 + m);
      else id = at(g, var, a - 2 + m, b - 1);
      Q[m] = W[id];
      G[m] = h * (double)dW[id + (size_t)(DIR * 4) * g.rows * g.pitch];
    }
    T vl, dl, vr, dr, hh;
    double xl, xr;
    geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, vl, dl, xl, vr,
                               dr, xr, hh, skipL, skipR);
    sv[i][0] = vl;
    sd[i][0] = dl;
    sv[i][1] = vr;
    sd[i][1] = dr;
    sh[i] = hh;
  }
  // keep side q of the own variables, send side 1 - q to the partner
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const T kv = q ? sv[i][1] : sv[i][0], kd = q ? sd[i][1] : sd[i][0];
    const T rv = pair_swap(q ? sv[i][0] : sv[i][1]);
    const T rd = pair_swap(q ? sd[i][0] : sd[i][1]);
    const T rh = pair_swap(sh[i]);
    v[i] = q ? rv : kv;
    d[i] = q ? rd : kd;
    h2[i] = q ? rh : sh[i];
    v[2 + i] = q ? kv : rv;
    d[2 + i] = q ? kd : rd;
    h2[2 + i] = q ? sh[i] : rh;
  }
}

// normal_pair with characteristic variables (the arithmetic of
// normal_char): both lanes load the four variables of the stencil and form
// the Roe eigenvectors at the face; lane q reconstructs the characteristic
// fields 2q and 2q+1 (both sides), the lanes swap halves, and lane q maps
// side q of all four fields, and the two-side mean h2, back to the state
// variables.
template <int DIR, typename T>
__device__ __forceinline__ void normal_pair_char(const Geo& g, const geno::KParams& k,
                                                 const double* __restrict__ W,
                                                 const T* __restrict__ dW, int a, int b, int q,
                                                 T (&v)[4], T (&d)[4], T (&h2)[4]) {
  const double h = DIR == 0 ? g.dx : g.dy;
  // state variable of each normal-frame slot
  constexpr int VM[4] = {0, DIR == 0 ? 1 : 2, DIR == 0 ? 2 : 1, 3};
  double Qv[4][4], Gv[4][4];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t id;
      if (DIR == 0) id = at(g, VM[f], a - 1, b - 2 + m);
      else id = at(g, VM[f], a - 2 + m, b - 1);
      Qv[f][m] = W[id];
      Gv[f][m] = h * (double)dW[id + (size_t)(DIR * 4) * g.rows * g.pitch];
    }
  const double Wa[4] = {Qv[0][1], Qv[1][1], Qv[2][1], Qv[3][1]};
  const double Wb[4] = {Qv[0][2], Qv[1][2], Qv[2][2], Qv[3][2]};
  geno::Eig2 e;
  const bool ch = geno::roe_eigen2(Wa, Wb, k.gamma, e);
  T sv[2][2], sd[2][2], sh[2];   // [field 2q + i][side]
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    // row 2q + i of the left eigenvectors, or slot 2q + i itself
    double L[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) L[f] = q ? e.L[2 + i][f] : e.L[i][f];
    double Q[4], G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (ch) {
        Q[m] = L[0] * Qv[0][m] + L[1] * Qv[1][m] + L[2] * Qv[2][m] + L[3] * Qv[3][m];
        G[m] = L[0] * Gv[0][m] + L[1] * Gv[1][m] + L[2] * Gv[2][m] + L[3] * Gv[3][m];
      } else {
        Q[m] = q ? Qv[2 + i][m] : Qv[i][m];
        G[m] = q ? Gv[2 + i][m] : Gv[i][m];
      }
    }
    T vl, dl, vr, dr, hh;
    double xl, xr;
    geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k, vl, dl, xl, vr,
                               dr, xr, hh);
    sv[i][0] = vl;
    sd[i][0] = dl;
    sv[i][1] = vr;
    sd[i][1] = dr;
    sh[i] = hh;
  }
  // side q of all four fields: the own ones kept, the partner's received
  double wq[4], dq[4], w2[4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const T kv = q ? sv[i][1] : sv[i][0], kd = q ? sd[i][1] : sd[i][0];
    const T rv = pair_swap(q ? sv[i][0] : sv[i][1]);
    const T rd = pair_swap(q ? sd[i][0] : sd[i][1]);
    const T rh = pair_swap(sh[i]);
    wq[i] = (double)(q ? rv : kv);
    dq[i] = (double)(q ? rd : kd);
    w2[i] = (double)(q ? rh : sh[i]);
    wq[2 + i] = (double)(q ? kv : rv);
    dq[2 + i] = (double)(q ? kd : rd);
    w2[2 + i] = (double)(q ? sh[i] : rh);
  }
  double Sv[4], Dv[4], S2[4];
  if (ch) {
    geno::from_characteristic2(e, wq, Sv);
    geno::from_characteristic2(e, dq, Dv);
    geno::from_characteristic2(e, w2, S2);
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      Sv[f] = wq[f];
      Dv[f] = dq[f];
      S2[f] = w2[f];
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    v[VM[f]] = T(Sv[f]);
    d[VM[f]] = T(Dv[f]);
    h2[VM[f]] = T(S2[f]);
  }
}

// the normal step inside the fused kernels: conservative variables,
// characteristic variables, or conservative variables with the learned
// gate's flags (a template parameter, so that each variant carries only its
// own arithmetic and shows under its own name in kernel traces)
enum { FUSED_PLAIN = 0, FUSED_CHAR = 1, FUSED_GATE = 2 };

// One work-group per tile of NT x NN face-row entries, NT along the
// tangential direction of the faces and NN across it (x-faces: NT rows by NN
// face columns; y-faces: NT columns of one face row, NN = 1). Every lane pair
// reconstructs one entry into LDS; after a barrier the pairs of the first
// NT - 2 tangential positions each evaluate the face whose three rows t,
// t+1, t+2 are in the tile. Neighbouring tiles overlap by two entries along
// the tangential direction (recomputed, 2/NT of the normal step). Entry e =
// t NN + u, u fastest, so that a wave's loads run along x. nbu: tiles across
// the tangential direction; a work-group takes tile (bt, bu) = (blk / nbu,
// blk % nbu).
template <int DIR, int NT, int NN>
struct FusedTile {
  static constexpr int NE = NT * NN;              // entries (lane pairs)
  static constexpr int BS = (2 * NE + 63) / 64 * 64;   // work-group size (whole waves)
  static constexpr int SS = 8 * NE + 1;           // LDS side stride (padded)
  static constexpr int LDS = 2 * SS + 4 * NE;     // elements of T
};
// (stage 2: at most 4 waves per SIMD for the y tile, 3 for the x tile, the
// faster of the two caps for each; 3 with characteristic variables, whose
// normal step needs more registers)
template <int DIR, typename T, bool WF, int VAR, int NT, int NN>
__device__ __forceinline__ void fused_body(const Geo& g, const geno::KParams& k,
                                           const double* __restrict__ W,
                                           const T* __restrict__ dW, T* __restrict__ fr,
                                           T* __restrict__ out, Ctrl* ctrl,
                                           unsigned int* __restrict__ queue, int nbu, int blk,
                                           const unsigned char* __restrict__ gate = nullptr) {
  using TL = FusedTile<DIR, NT, NN>;
  // [side][quantity (value, h d/dn)][variable][entry], the side stride padded
  // against bank conflicts between the two lanes of a pair; then h2
  // [variable][entry]
  __shared__ T lds[TL::LDS];
  const int bt = blk / nbu, bu = blk % nbu;
  const int q = threadIdx.x & 1, p = (int)(threadIdx.x >> 1);
  const int t = p / NN, u = p % NN;
  // entry (t, u) of the tile: face-row indices (a, b) of normal_body, and the
  // largest in-range ones
  int ea, eb, amax, bmax;
  if (DIR == 0) {
    ea = bt * (NT - 2) + t;   // face row of the entry (cell row ea - 1)
    eb = bu * NN + u;         // face column
    amax = g.ny + 1;
    bmax = g.nx;
  } else {
    ea = bu;                  // face row (NN = 1: one face row per tile)
    eb = bt * (NT - 2) + t;   // column of the entry (cell column eb - 1)
    amax = g.ny;
    bmax = g.nx + 1;
  }
  // (lanes past the tile's entries, in a last partial wave, only take part)
  const bool need = p < TL::NE && ea <= amax && eb <= bmax;
  if (__ballot(need)) {   // whole waves out of the grid skip the normal step
    T v[4], d[4], h2[4];
    const int a = min(ea, amax), b = min(eb, bmax);
    if constexpr (VAR == FUSED_CHAR) {
      normal_pair_char<DIR, T>(g, k, W, dW, a, b, q, v, d, h2);
    } else {
      // the learned gate's flags of the cells of the two sides (as in
      // normal_body): chi = 1 without the indicators where set
      bool skipL = false, skipR = false;
      if (VAR == FUSED_GATE) {
        const int jl = a - 1, il = b - 1;
        const int jr = DIR == 0 ? a - 1 : a, ir = DIR == 0 ? b : b - 1;
        if (jl >= 0 && jl < g.ny && il >= 0 && il < g.nx) skipL = gate[jl * g.nx + il] != 0;
        if (jr >= 0 && jr < g.ny && ir >= 0 && ir < g.nx) skipR = gate[jr * g.nx + ir] != 0;
      }
      normal_pair<DIR, T>(g, k, W, dW, a, b, q, v, d, h2, skipL, skipR);
    }
    if (p < TL::NE) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        lds[q * TL::SS + (0 * 4 + f) * TL::NE + p] = v[f];
        lds[q * TL::SS + (1 * 4 + f) * TL::NE + p] = d[f];
      }
    }
    if (q == 0 && p < TL::NE)
#pragma unroll
      for (int f = 0; f < 4; ++f) lds[2 * TL::SS + f * TL::NE + p] = h2[f];
  }
  __syncthreads();
  // the face of this pair: rows t, t+1, t+2 of its tangential line
  int fa, fb;
  bool valid;
  if (DIR == 0) {
    fa = ea;
    fb = eb;
    valid = t < NT - 2 && fa < g.ny && fb <= g.nx;
  } else {
    fa = ea;
    fb = eb;
    valid = t < NT - 2 && fb < g.nx;
  }
  if (!__ballot(valid)) return;   // no face in this wave (no barrier follows)
  const int pc = valid ? p : u;   // an invalid pair reads entries of row 0
  const RowsLds<T> sr{lds, {q * TL::SS + pc, q * TL::SS + pc + NN, q * TL::SS + pc + 2 * NN},
                      2 * TL::SS + pc + NN, TL::NE};
  const FaceGeo<DIR> fg(g);
  const int face = valid ? fa * fg.n1 + fb : 0;
  unsigned int wc[GENO_NCLASS] = {};
  // (the x tile writes 64-byte pieces of each face row: in the mixed form
  // plain stores, which the L2 merges, were faster; in FP64 and for the
  // y-faces non-temporal ones)
  constexpr bool NTS = sizeof(T) == 8 || DIR == 1;
  const bool queued = face_core<DIR, 1, T, RowsLds<T>, NTS>(g, k, W, out, ctrl, WF ? 1 : 0, wc,
                                                           face, valid, queue, sr);
  // the rows are read from LDS again for the spill
  asm volatile("" ::: "memory");
  if (queued) spill_rows<DIR, T>(g, face, sr, fr);
}

template <int DIR, typename T, bool WF, int VAR, int NT, int NN>
__global__ void __launch_bounds__((2 * NT * NN + 63) / 64 * 64)
__attribute__((amdgpu_waves_per_eu(WF ? 1 : (DIR == 0 || VAR == FUSED_CHAR ? 2 : 4))))
k_fused2d(Geo g, geno::KParams k, const double* __restrict__ W, const T* __restrict__ dW,
          T* __restrict__ fr, T* __restrict__ out, Ctrl* ctrl, unsigned int* __restrict__ queue,
          int nbu, const unsigned char* __restrict__ gate) {
  fused_body<DIR, T, WF, VAR, NT, NN>(g, k, W, dW, fr, out, ctrl, queue, nbu, xcd_block(), gate);
}
// tile shapes
// (measured at 2048^2: 16 x 8 beat 32 x 8, 32 x 4, 64 x 4, 64 x 8 and 128 x 2
// for the x-faces, 128 beat 64 and 256 for the y-faces)
constexpr int FX_NT = 16, FX_NN = 8;    // x-faces: 16 rows x 8 face columns, 256 lanes
constexpr int FY_NT = 128, FY_NN = 1;   // y-faces: 128 columns of one face row, 256 lanes
constexpr int FX_BS = FusedTile<0, FX_NT, FX_NN>::BS;
constexpr int FY_BS = FusedTile<1, FY_NT, FY_NN>::BS;
// work-groups of the fused launches of a grid, and their tiles across the
// tangential direction
int fused_nbu(const Geo& g, int dir) {
  return dir == 0 ? (g.nx + 1 + FX_NN - 1) / FX_NN : g.ny + 1;
}
unsigned fused_blocks(const Geo& g, int dir) {
  const size_t nt = dir == 0 ? (size_t)(g.ny + FX_NT - 3) / (FX_NT - 2)
                             : (size_t)(g.nx + FY_NT - 3) / (FY_NT - 2);
  return (unsigned)(nt * fused_nbu(g, dir));
}

// Before the face kernels of a stage: the step's dt from the CFL partial
// minima (stage 1) and empty face queues.
__global__ void __launch_bounds__(1024) k_stage_prep(const double* __restrict__ part, int npart,
                                                      Ctrl* ctrl, double cfl, double dt_fixed,
                                                      double* dt_out, int step) {
  if (part) reduce_dt(part, npart, ctrl, cfl, dt_fixed, dt_out, step);
  if (threadIdx.x < 2) ctrl->qcount[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// 1-D faces: normal GENO of the three variables at face f (cells f-2..f+1),
// guard, then states (MODE 0) or flux (MODE 1). out as the 2-D layouts with
// one Gauss point: states [side][quant(2)][var][f] followed by the mean
// h^2 d^2/dx^2 [var][f] (zero if a side is guarded), flux [kind][var][f]
// with the kinds of the 2-D face step. The 1-D step is reduced before this
// kernel (k_dt1d).
// ---------------------------------------------------------------------------
template <int MODE, typename T>
__global__ void __launch_bounds__(BLOCK) k_faces1d(Geo g, geno::KParams k,
                                                   const double* __restrict__ W,
                                                   const T* __restrict__ dW,
                                                   T* __restrict__ out,
                                                   double* __restrict__ chi, Ctrl* ctrl,
                                                   int want_F, Cnt cnt) {
  const int nfc = g.nx + 1;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned int nlow = 0, nguard = 0;
  int pk = -1;
  if (f < nfc) {
    T S[2][3], Dn[2][3], D2[3];
    // characteristic variables: the left eigenvectors at the Roe average of
    // cells f-1 and f (both stencil quantities projected), back with the
    // right ones; a face without a real sound speed stays conservative
    geno6::Eig<double> e;
    bool ch = false;
    if (k.charvars) {
      double Wa[3], Wb[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Wa[v] = W[at(g, v, 0, f - 1)];
        Wb[v] = W[at(g, v, 0, f)];
      }
      ch = geno6::roe_eigen<double>(Wa, Wb, k.gamma, e);
    }
    if (ch) {
      double Qv[3][4], Gv[3][4];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const size_t id = at(g, v, 0, f - 2 + m);
          Qv[v][m] = W[id];
          Gv[v][m] = g.dx * (double)dW[id];
        }
      double wv[2][3], wd[2][3], w2[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double Q[4], G[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          Q[m] = e.L[c][0] * Qv[0][m] + e.L[c][1] * Qv[1][m] + e.L[c][2] * Qv[2][m];
          G[m] = e.L[c][0] * Gv[0][m] + e.L[c][1] * Gv[1][m] + e.L[c][2] * Gv[2][m];
        }
        T s0, d0, s1, d1, h2;
        double xl, xr;
        nlow += geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k,
                                           s0, d0, xl, s1, d1, xr, h2);
        wv[0][c] = (double)s0;
        wd[0][c] = (double)d0;
        wv[1][c] = (double)s1;
        wd[1][c] = (double)d1;
        w2[c] = (double)h2;
        if (chi) {
          chi[(size_t)(0 * 3 + c) * nfc + f] = xl;
          chi[(size_t)(1 * 3 + c) * nfc + f] = xr;
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        double Sv[3], Dv[3];
        geno6::from_characteristic(e, wv[s], Sv);
        geno6::from_characteristic(e, wd[s], Dv);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          S[s][v] = T(Sv[v]);
          Dn[s][v] = T(Dv[v]);
        }
      }
      double S2[3];
      geno6::from_characteristic(e, w2, S2);
#pragma unroll
      for (int v = 0; v < 3; ++v) D2[v] = T(S2[v]);
    } else {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double Q[4], G[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const size_t id = at(g, v, 0, f - 2 + m);
          Q[m] = W[id];
          G[m] = g.dx * (double)dW[id];
        }
        double xl, xr;
        nlow += geno::geno_face<T, double>(Q[0], Q[1], Q[2], Q[3], G[0], G[1], G[2], G[3], k,
                                           S[0][v], Dn[0][v], xl, S[1][v], Dn[1][v], xr, D2[v]);
        if (chi) {
          chi[(size_t)(0 * 3 + v) * nfc + f] = xl;
          chi[(size_t)(1 * 3 + v) * nfc + f] = xr;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!geno::admissible<3, T>(S[s], k.gamma)) {
        ++nguard;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          S[s][v] = T(W[at(g, v, 0, f - 1 + s)]);
          Dn[s][v] = T(0);
        }
      }
    }
    if (nguard && ctrl) atomicAdd(&ctrl->guard, (unsigned long long)nguard);
    if (nguard)
#pragma unroll
      for (int v = 0; v < 3; ++v) D2[v] = T(0);
    if constexpr (MODE == 0) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          out[(size_t)((s * 2 + 0) * 3 + v) * nfc + f] = S[s][v];
          out[(size_t)((s * 2 + 1) * 3 + v) * nfc + f] = Dn[s][v];
        }
#pragma unroll
      for (int v = 0; v < 3; ++v) out[(size_t)(12 + v) * nfc + f] = D2[v];
    } else {
      const double dt = dt_of(ctrl);
      const T ih = T(1.0 / g.dx), ih2 = T(1.0 / (g.dx * g.dx));
      T nl[3], nr[3], xx[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        nl[v] = Dn[0][v] * ih;
        nr[v] = Dn[1][v] * ih;
        xx[v] = D2[v] * ih2;
      }
      gks::PointOut<3, T> po;
      pk = gks::point_flux<3, true, T>(S[0], S[1], nl, nr, nullptr, nullptr, xx, nullptr, nullptr,
                                       dt, k, want_F != 0, po);
      const T c8 = T(dt * dt / 8.0), c6 = T(dt * dt / 6.0);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        out[(size_t)(1 * 3 + v) * nfc + f] = po.Ft[v];
        if (want_F) {
          out[(size_t)(0 * 3 + v) * nfc + f] = po.F[v];
          out[(size_t)(2 * 3 + v) * nfc + f] = po.Wh[v] + c8 * po.Wtt[v];
          out[(size_t)(3 * 3 + v) * nfc + f] = po.Wf[v] + c6 * po.Wtt[v];
        } else {
          out[(size_t)(2 * 3 + v) * nfc + f] = po.Wtt[v];
        }
      }
    }
  }
  if (MODE == 1 && cnt.p) {
    unsigned int wc[GENO_NCLASS] = {};
    wc[GENO_W_UNITS] = f < nfc ? 1u : 0u;
    wc[GENO_W_LOW] = nlow;
    wc[GENO_W_EQUAL] = pk == gks::PT_EQUAL ? 1u : 0u;
    wc[GENO_W_FAST] = pk == gks::PT_FAST ? 1u : 0u;
    wc[GENO_W_SLOW] = pk == gks::PT_SLOW ? 1u : 0u;
    wc[GENO_W_GUARD] = nguard;
    block_count(cnt, GENO_K_FACES_1D, wc);
  }
}

// Conserved totals: one work-group of 1024 lanes per field. Each lane sums
// its cells (strided, in index order) with Neumaier's compensation; the
// (sum, correction) pairs are then combined in a fixed tree, first across
// the wave, then across the waves in order.
__device__ __forceinline__ void two_sum_acc(double& s, double& c, double x) {
  const double t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

__global__ void __launch_bounds__(1024) k_totals(Geo g, const double* __restrict__ W,
                                                 double area, double* __restrict__ totals) {
  __shared__ double rs[16], rc[16];
  const int f = (int)blockIdx.x;
  const int n = g.nx * g.ny;
  double s = 0.0, c = 0.0;
  for (int t = (int)threadIdx.x; t < n; t += (int)blockDim.x) {
    const int j = t / g.nx, i = t - j * g.nx;
    two_sum_acc(s, c, W[at(g, f, j, i)]);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double s2 = __shfl_xor(s, off, 64), c2 = __shfl_xor(c, off, 64);
    // lanes l and l ^ off combine in the order (lower lane, higher lane)
    const bool lo = ((int)threadIdx.x & off) == 0;
    double a = lo ? s : s2, b = lo ? s2 : s;
    double cc = lo ? c + c2 : c2 + c;
    two_sum_acc(a, cc, b);
    s = a;
    c = cc;
  }
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rs[w] = s;
    rc[w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)blockDim.x >> 6;
    double a = rs[0], cc = rc[0];
    for (int q = 1; q < nw; ++q) {
      cc += rc[q];
      two_sum_acc(a, cc, rs[q]);
    }
    totals[f] = (a + cc) * area;
  }
}

// 1-D: reduce the CFL partials of the previous kernel (single block).
__global__ void __launch_bounds__(BLOCK) k_dt1d(const double* __restrict__ part, int npart,
                                                Ctrl* ctrl, double cfl, double dt_fixed,
                                                double* dt_out, int step) {
  reduce_dt(part, npart, ctrl, cfl, dt_fixed, dt_out, step);
}

// gks_flux on caller-given point states (layout of geno_reconstruct: the
// point states, then the points' h-scaled second derivatives). Outputs the
// Gauss averages of F, dF/dt, and in Wi three blocks [W(dt/2), W(dt),
// W_tt][var][face].
template <int NV, typename T>
__global__ void __launch_bounds__(BLOCK) k_flux_points(int nfaces, int ngauss, int dir,
                                                       geno::KParams k, double hn, double ht,
                                                       double dt, const T* __restrict__ st,
                                                       T* __restrict__ F, T* __restrict__ Ft,
                                                       T* __restrict__ Wi) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nfaces) return;
  constexpr int Q = NV == 4 ? 3 : 2;
  constexpr int NQ2 = NV == 4 ? 3 : 1;   // second-derivative quantities per point
  const T w = T(1.0 / ngauss);
  const T ihn = T(1.0 / hn), iht = T(1.0 / ht);
  const T inn = T(1.0 / (hn * hn)), int_ = T(1.0 / (hn * ht)), itt = T(1.0 / (ht * ht));
  const int perm[4] = {0, dir == 0 ? 1 : 2, dir == 0 ? 2 : 1, 3};
  const size_t sec0 = (size_t)2 * ngauss * Q * NV;
  T A[5][NV];
#pragma unroll
  for (int e = 0; e < 5; ++e)
#pragma unroll
    for (int v = 0; v < NV; ++v) A[e][v] = T(0);
  for (int q = 0; q < ngauss; ++q) {
    T Ws[2][NV], ns[2][NV], ts[2][NV], xnn[NV], xnt[NV], xtt[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int pv = NV == 4 ? perm[v] : v;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const size_t base = (size_t)((s * ngauss + q) * Q) * NV;
        Ws[s][v] = st[(base + 0 * NV + pv) * nfaces + o];
        ns[s][v] = st[(base + 1 * NV + pv) * nfaces + o] * ihn;
        ts[s][v] = NV == 4 ? st[(base + 2 * NV + pv) * nfaces + o] * iht : T(0);
      }
      const size_t sb = sec0 + (size_t)(q * NQ2) * NV;
      xnn[v] = st[(sb + pv) * nfaces + o] * inn;
      xnt[v] = NV == 4 ? st[(sb + NV + pv) * nfaces + o] * int_ : T(0);
      xtt[v] = NV == 4 ? st[(sb + 2 * NV + pv) * nfaces + o] * itt : T(0);
    }
    gks::PointOut<NV, T> po;
    gks::point_flux<NV, true, T>(Ws[0], Ws[1], ns[0], ns[1], ts[0], ts[1], xnn, xnt, xtt, dt, k,
                                 true, po);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      A[0][v] = A[0][v] + w * po.F[v];
      A[1][v] = A[1][v] + w * po.Ft[v];
      A[2][v] = A[2][v] + w * po.Wh[v];
      A[3][v] = A[3][v] + w * po.Wf[v];
      A[4][v] = A[4][v] + w * po.Wtt[v];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int pv = NV == 4 ? perm[v] : v;
    if (F) F[(size_t)pv * nfaces + o] = A[0][v];
    if (Ft) Ft[(size_t)pv * nfaces + o] = A[1][v];
    if (Wi)
#pragma unroll
      for (int e = 0; e < 3; ++e) Wi[(size_t)(e * NV + pv) * nfaces + o] = A[2 + e][v];
  }
}

// ---------------------------------------------------------------------------
// Cell update (two-stage fourth-order method). STAGE 1: W* = W + dt/2 L +
// dt^2/8 Lt, R = W + dt L + dt^2/6 Lt; grad* by the Gauss theorem (Eq. (2))
// from the interface values at the stage time, W(dt/2) + dt^2/8 W_tt.
// STAGE 2: W = R + dt^2/3 Lt*, grad = the Gauss theorem on the stage-1
// interface values W(dt) + dt^2/6 W_tt (face kind 3, which the stage-2 face
// step leaves in place) plus dt^2/3 times the Gauss theorem on W_tt*, and
// the CFL minima of the new state per block. Both write the ghost cells of
// the state they produce.
// ---------------------------------------------------------------------------
template <int NDIM, int STAGE, typename T>
__device__ __forceinline__ void update_body(const Geo& g, const geno::KParams& k,
                                            const double* __restrict__ Win,
                                            double* __restrict__ Wout, T* __restrict__ dWout,
                                            double* __restrict__ R,
                                            const T* __restrict__ fx,
                                            const T* __restrict__ fy, Ctrl* ctrl,
                                            double* __restrict__ part, const Cnt& cnt, int lb) {
  constexpr int NV = NDIM == 2 ? 4 : 3;
  const int t = lb * (int)blockDim.x + (int)threadIdx.x;
  const int n = g.nx * g.ny;
  const double dt = dt_of(ctrl);
  double tloc = INFINITY;
  if (t < n) {
    const int j = t / g.nx, i = t % g.nx;
    const size_t xp = NDIM == 2 ? (size_t)xface_pitch(g.nx) : (size_t)(g.nx + 1);
    const size_t px = xp * g.ny;
    const size_t py = (size_t)g.nx * (g.ny + 1);
    const size_t ox = (size_t)j * xp + i;
    const size_t oy = (size_t)j * g.nx + i;
    // every value the cell's update reads, loaded before its arithmetic (more
    // loads in flight per wave: the update is bound by memory, not by
    // registers): the face planes of the stage's kinds on both sides of the
    // cell (stage 1 kinds 0-2, stage 2 kinds 1-3), then W (stage 1) or R;
    // flux differences and gradients in float64 whatever the storage type
    double xl[4 * NV], xr[4 * NV], yl[4 * NV], yu[4 * NV];
#pragma unroll
    for (int p = 0; p < 4 * NV; ++p) {
      const int kind = p / NV;
      xl[p] = xr[p] = yl[p] = yu[p] = 0.0;
      if (STAGE == 1 ? kind > 2 : kind < 1) continue;
      xl[p] = (double)fx[p * px + ox];
      xr[p] = (double)fx[p * px + ox + 1];
      if constexpr (NDIM == 2) {
        yl[p] = (double)fy[p * py + oy];
        yu[p] = (double)fy[p * py + oy + g.nx];
      }
    }
    double wr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wr[v] = STAGE == 1 ? Win[at(g, v, j, i)] : R[at(g, v, j, i)];
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
    const double c3 = dt * dt / 3.0;
    double w[NV];
    T dw[NV * NDIM];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double l, lt, gx, gy = 0.0;
      // Gauss theorem on kind 2: W(dt/2) + dt^2/8 W_tt (stage 1), W_tt* (stage 2)
      gx = (xr[2 * NV + v] - xl[2 * NV + v]) * idx;
      if constexpr (NDIM == 2) {
        l = -dot2(xr[0 * NV + v] - xl[0 * NV + v], idx, yu[0 * NV + v] - yl[0 * NV + v], idy);
        lt = -dot2(xr[1 * NV + v] - xl[1 * NV + v], idx, yu[1 * NV + v] - yl[1 * NV + v], idy);
        gy = (yu[2 * NV + v] - yl[2 * NV + v]) * idy;
      } else {
        l = -(xr[0 * NV + v] - xl[0 * NV + v]) * idx;
        lt = -(xr[1 * NV + v] - xl[1 * NV + v]) * idx;
      }
      const size_t c = at(g, v, j, i);
      if constexpr (STAGE == 1) {
        const double w0 = wr[v];
        w[v] = w0 + 0.5 * dt * l + dt * dt / 8.0 * lt;
        R[c] = w0 + dt * l + dt * dt / 6.0 * lt;
        dw[v] = T(gx);
        if constexpr (NDIM == 2) dw[NV + v] = T(gy);
      } else {
        (void)l;
        w[v] = wr[v] + c3 * lt;
        // kind 3 of stage 1: W(dt) + dt^2/6 W_tt
        const double gx1 = (xr[3 * NV + v] - xl[3 * NV + v]) * idx;
        dw[v] = T(gx1 + c3 * gx);
        if constexpr (NDIM == 2) {
          const double gy1 = (yu[3 * NV + v] - yl[3 * NV + v]) * idy;
          dw[NV + v] = T(gy1 + c3 * gy);
        }
      }
      Wout[c] = w[v];
    }
#pragma unroll
    for (int v = 0; v < NV * NDIM; ++v) dWout[at(g, v, j, i)] = dw[v];
    scatter_ghosts<NDIM, T>(g, Wout, dWout, j, i, w, dw);
    if constexpr (STAGE == 2) {
      // non-physical cell: a non-finite value, rho <= 0 or p <= 0
      bool bad = false;
#pragma unroll
      for (int v = 0; v < NV; ++v) bad |= !isfinite(w[v]);
      const double ke = NV == 4 ? dot2(w[1], w[1], w[2], w[2]) : w[1] * w[1];
      // p > 0 <=> rho rhoE - |m|^2 / 2 > 0 once rho > 0
      bad |= !(w[0] > 0.0) || !(w[0] * w[NV - 1] - 0.5 * ke > 0.0);
      if (bad) atomicAdd(&ctrl->nonfinite, 1ull);
      tloc = cell_tmin<NDIM>(g, w, k.gamma);
    }
  }
  if constexpr (STAGE == 2) block_min(tloc, part, lb);
  if (cnt.p) {
    unsigned int wc[GENO_NCLASS] = {};
    wc[GENO_W_UNITS] = t < n ? 1u : 0u;
    block_count(cnt, STAGE == 1 ? GENO_K_UPDATE_1 : GENO_K_UPDATE_2, wc);
  }
}

// (2-D FP64: two waves per SIMD, so that the compiler keeps every load of a
// cell in flight at once instead of trading them for occupancy; 2048^2:
// stage 1 300 -> 281 us, stage 2 269 -> 262 us. The float-gradient form
// measured slower so in stage 2 and keeps the default.)
template <int NDIM, int STAGE, typename T>
__global__ void __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(NDIM == 2 && sizeof(T) == 8 ? 2 : 1,
                                   NDIM == 2 && sizeof(T) == 8 ? 2 : 10)))
k_update(Geo g, geno::KParams k,
                                                  const double* __restrict__ Win,
                                                  double* __restrict__ Wout,
                                                  T* __restrict__ dWout,
                                                  double* __restrict__ R,
                                                  const T* __restrict__ fx,
                                                  const T* __restrict__ fy, Ctrl* ctrl,
                                                  double* __restrict__ part, Cnt cnt) {
  update_body<NDIM, STAGE, T>(g, k, Win, Wout, dWout, R, fx, fy, ctrl, part, cnt,
                              xcd_block());
}

// ---------------------------------------------------------------------------
// Learned gate. The loaded network lives in device globals as bfloat16
// fragments of the B operands of v_mfma_f32_16x16x32_bf16, in lane order:
// g_mlp_frag[layer * 8 + kb * 4 + nt][lane] holds B[k][n] for k = kb * 32 +
// 8 * (lane / 16) + e (e = 0..7), n = nt * 16 + lane % 16, with B = W1^T
// (inputs padded from 40 to 64 with zeros) or W2^T. One wave evaluates 16
// samples per tile: the A operand lane (r = lane % 16, g = lane / 16) holds
// X[r][kb * 32 + 8 g + e], and the accumulator lane holds rows 4 g + e of
// column lane % 16. The weights stay in registers across tiles; the
// transposes between layers go through LDS.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ bf16x8 g_mlp_frag[16][64];
__device__ float g_mlp_vec[3 * mlp::NH + 1];   // b1, b2, w3, b3

struct MlpRegs {
  bf16x8 w[16];
  float b1[4], b2[4], w3[4], b3;
};

__device__ __forceinline__ void mlp_regs(MlpRegs& R) {
  const int lane = threadIdx.x & 63, r = lane & 15;
#pragma unroll
  for (int f = 0; f < 16; ++f) R.w[f] = g_mlp_frag[f][lane];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    R.b1[nt] = g_mlp_vec[nt * 16 + r];
    R.b2[nt] = g_mlp_vec[mlp::NH + nt * 16 + r];
    R.w3[nt] = g_mlp_vec[2 * mlp::NH + nt * 16 + r];
  }
  R.b3 = g_mlp_vec[3 * mlp::NH];
}

// Network on the 16 samples of this wave's tile: xs, hs are the wave's LDS
// tiles [16][64] (xs filled by the caller, columns 40..63 zero). Every wave
// of the work-group calls this together (it synchronises the work-group).
// Returns the probabilities of samples 4 (lane / 16) + e in p[e].
__device__ __forceinline__ void mlp_tile(const MlpRegs& R, const __bf16* xs, __bf16* hs,
                                         float (&p)[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  bf16x8 a0 = *reinterpret_cast<const bf16x8*>(xs + r * 64 + 8 * g);
  bf16x8 a1 = *reinterpret_cast<const bf16x8*>(xs + r * 64 + 32 + 8 * g);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, R.w[nt], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, R.w[4 + nt], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) hs[(4 * g + e) * 64 + nt * 16 + r] = (__bf16)mlp::gelu_fast(acc[e] + R.b1[nt]);
  }
  __syncthreads();
  a0 = *reinterpret_cast<const bf16x8*>(hs + r * 64 + 8 * g);
  a1 = *reinterpret_cast<const bf16x8*>(hs + r * 64 + 32 + 8 * g);
  float zs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, R.w[8 + nt], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, R.w[12 + nt], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) zs[e] += mlp::gelu_fast(acc[e] + R.b2[nt]) * R.w3[nt];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float z = zs[e];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) z += __shfl_xor(z, off, 64);
    p[e] = mlp::sigmoid(z + R.b3);
  }
}

// The 10 features of variable v (face frame) of cell (j, i) along DIR.
template <int DIR, typename T>
__device__ __forceinline__ void gate_features(const Geo& g, const double* __restrict__ W,
                                              const T* __restrict__ dW, int j, int i, int v,
                                              float* f) {
  const int vv = DIR == 0 ? v : (v == 1 ? 2 : (v == 2 ? 1 : v));
  const double h = DIR == 0 ? g.dx : g.dy;
  const size_t gplane = (size_t)(DIR * 4) * g.rows * g.pitch;
  double q[5], d[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const size_t id = DIR == 0 ? at(g, vv, j, i - 2 + m) : at(g, vv, j - 2 + m, i);
    q[m] = W[id];
    d[m] = h * (double)dW[id + gplane];
  }
  double mx = q[0], mn = q[0];
#pragma unroll
  for (int m = 1; m < 5; ++m) {
    mx = fmax(mx, q[m]);
    mn = fmin(mn, q[m]);
  }
  const double inv = 1.0 / ((mx - mn) + 1e-12 * fabs(q[2]) + 1e-300);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    f[m] = (float)fmin(64.0, fmax(-64.0, (q[m] - q[2]) * inv));
    f[5 + m] = (float)fmin(64.0, fmax(-64.0, d[m] * inv));
  }
}

constexpr int GATE_TILES = 8;   // tiles of 16 cells per wave of a gate work-group

// Gate of every interior cell for DIR: flags (PROB = 0: out[c] = p >= thr)
// or probabilities (PROB = 1: outp[c] = p). Work-group = 4 waves; every wave
// runs GATE_TILES tiles (all waves the same count: mlp_tile synchronises).
template <int DIR, typename T, int PROB>
__global__ void __launch_bounds__(256) k_gate(Geo g, const double* __restrict__ W,
                                              const T* __restrict__ dW, float thr,
                                              unsigned char* __restrict__ out,
                                              float* __restrict__ outp) {
  __shared__ __align__(16) __bf16 xs[4][16 * 64];
  __shared__ __align__(16) __bf16 hs[4][16 * 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MlpRegs R;
  mlp_regs(R);
  const int ncell = g.nx * g.ny;
  const int s = lane >> 2, v = lane & 3;
  for (int it = 0; it < GATE_TILES; ++it) {
    const int tile = (blockIdx.x * GATE_TILES + it) * 4 + w;
    const int c = tile * 16 + s;
    float f[10];
    if (c < ncell) {
      gate_features<DIR, T>(g, W, dW, c / g.nx, c % g.nx, v, f);
    } else {
#pragma unroll
      for (int m = 0; m < 10; ++m) f[m] = 0.0f;
    }
#pragma unroll
    for (int m = 0; m < 10; ++m) xs[w][s * 64 + v * 10 + m] = (__bf16)f[m];
#pragma unroll
    for (int m = 0; m < 6; ++m) xs[w][s * 64 + 40 + v * 6 + m] = (__bf16)0.0f;
    __syncthreads();
    float p[4];
    mlp_tile(R, xs[w], hs[w], p);
    if ((lane & 15) == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c2 = tile * 16 + 4 * (lane >> 4) + e;
        if (c2 < ncell) {
          if (PROB) outp[c2] = p[e];
          else out[c2] = p[e] >= thr ? 1 : 0;
        }
      }
    }
    __syncthreads();
  }
}

// the network on given inputs X[n][40] (float), for tests of the inference
__global__ void __launch_bounds__(256) k_mlp_infer(const float* __restrict__ X, int n,
                                                   float* __restrict__ prob) {
  __shared__ __align__(16) __bf16 xs[4][16 * 64];
  __shared__ __align__(16) __bf16 hs[4][16 * 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MlpRegs R;
  mlp_regs(R);
  const int s = lane >> 2, v = lane & 3;
  const int tile = blockIdx.x * 4 + w;
  const int c = tile * 16 + s;
#pragma unroll
  for (int m = 0; m < 10; ++m)
    xs[w][s * 64 + v * 10 + m] = (__bf16)(c < n ? X[(size_t)c * mlp::NIN + v * 10 + m] : 0.0f);
#pragma unroll
  for (int m = 0; m < 6; ++m) xs[w][s * 64 + 40 + v * 6 + m] = (__bf16)0.0f;
  __syncthreads();
  float p[4];
  mlp_tile(R, xs[w], hs[w], p);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c2 = tile * 16 + 4 * (lane >> 4) + e;
      if (c2 < n) prob[c2] = p[e];
    }
  }
}

// Harvest: features (float) and the plain-GENO target (float64 indicators)
// of every interior cell for DIR.
template <int DIR, typename T>
__global__ void __launch_bounds__(BLOCK) k_harvest(Geo g, geno::KParams k,
                                                   const double* __restrict__ W,
                                                   const T* __restrict__ dW,
                                                   float* __restrict__ X, float* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.nx * g.ny) return;
  const int j = c / g.nx, i = c % g.nx;
  double tmin = 1.0;
#pragma unroll 1
  for (int v = 0; v < 4; ++v) {
    float f[10];
    gate_features<DIR, T>(g, W, dW, j, i, v, f);
#pragma unroll
    for (int m = 0; m < 10; ++m) X[(size_t)c * mlp::NIN + v * 10 + m] = f[m];
    if (y) {
      const int vv = DIR == 0 ? v : (v == 1 ? 2 : (v == 2 ? 1 : v));
      const double h = DIR == 0 ? g.dx : g.dy;
      const size_t gplane = (size_t)(DIR * 4) * g.rows * g.pitch;
      double q[5], d[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const size_t id = DIR == 0 ? at(g, vv, j, i - 2 + m) : at(g, vv, j - 2 + m, i);
        q[m] = W[id];
        d[m] = h * (double)dW[id + gplane];
      }
      double val, der, xl, xr;
      // left state of face j+1/2 (cells j-1..j+2) and right state of face j-1/2
      // (cells j-2..j+1 reflected about that face)
      double d2;
      geno::geno_side<double, double>(q[1], q[2], q[3], q[4], d[1], 0.0, 0.0, 0.0, k, val, der, d2,
                                      xl);
      geno::geno_side<double, double>(q[3], q[2], q[1], q[0], -d[3], 0.0, 0.0, 0.0, k, val, der, d2,
                                      xr);
      tmin = fmin(tmin, fmin(xl, xr));
    }
  }
  if (y) y[c] = (float)tmin;
}

// ---------------------------------------------------------------------------
// Batched launches: many independent 2-D grids advanced together. Each launch
// runs one kernel kind for every grid: the grids' work-group ranges are
// concatenated, and a work-group finds its grid by binary search over the
// range starts. The search takes the XCD slab index, so each XCD works on
// neighbouring ranges of one or a few grids. Work-group size BS is a template
// parameter chosen per kind by the caller (autotuned).
// ---------------------------------------------------------------------------
enum {
  BK_INIT = 0, BK_NORMAL_X, BK_FACES_X, BK_NORMAL_Y, BK_FACES_Y, BK_SLOW, BK_UPDATE,
  BK_FUSED_X, BK_FUSED_Y, BK_PREP,   // the fused stage: prep, fused x, fused y, slow, update
  BK_N
};

struct BEntry {
  Geo geo;
  double* W;
  void* dW;
  Ctrl* ctrl;
  double* part;
  unsigned int* queue[2];
  double* wst;
  double* r;
  void* dwst;
  void* fr[2];
  void* fl[2];
  int npart;     // update work-groups of this grid (CFL partials)
  int slow_nb;   // work-groups serving this grid in the tau > 0 launch
  int fnbu[2];   // fused launches: tiles across the tangential direction
};

// index of the grid whose range [start[g], start[g+1]) holds global work-group gb
__device__ __forceinline__ int find_grid(const int* __restrict__ start, int ngrids, int gb) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= gb) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int BS>
__global__ void __launch_bounds__(BS) kb_init(const BEntry* __restrict__ tab,
                                              const int* __restrict__ offs, int ngrids,
                                              double gamma) {
  const int* st = offs + BK_INIT * (ngrids + 1);
  const int gb = xcd_block();
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  init_body<2, T>(e.geo, gamma, e.W, (T*)e.dW, e.part, e.ctrl, gb - st[gi]);
}

template <int DIR, typename T, int BS, bool CHAR>
__global__ void __launch_bounds__(BS) kb_normal(const BEntry* __restrict__ tab,
                                                const int* __restrict__ offs, int ngrids,
                                                geno::KParams k, int stage, Cnt cnt) {
  const int* st = offs + (DIR == 0 ? BK_NORMAL_X : BK_NORMAL_Y) * (ngrids + 1);
  const int gb = xcd_block();
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  const double* W = stage == 1 ? e.W : e.wst;
  const T* dW = (const T*)(stage == 1 ? e.dW : e.dwst);
  const double* part = (DIR == 0 && stage == 1) ? e.part : nullptr;
  normal_body<DIR, T, CHAR>(e.geo, k, W, dW, (T*)e.fr[DIR], nullptr, e.ctrl, part, e.npart,
                            nullptr, 0, cnt, gb - st[gi]);
}

template <int DIR, typename T, int BS>
__global__ void __launch_bounds__(BS) kb_faces(const BEntry* __restrict__ tab,
                                               const int* __restrict__ offs, int ngrids,
                                               geno::KParams k, int stage, Cnt cnt) {
  const int* st = offs + (DIR == 0 ? BK_FACES_X : BK_FACES_Y) * (ngrids + 1);
  const int gb = xcd_block();
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  const double* W = stage == 1 ? e.W : e.wst;
  faces_body<DIR, 1, T>(e.geo, k, W, (const T*)e.fr[DIR], (T*)e.fl[DIR], e.ctrl, stage == 1, cnt,
                        e.queue[DIR], gb - st[gi]);
}

template <typename T, int BS>
__global__ void __launch_bounds__(BS) kb_slow(const BEntry* __restrict__ tab,
                                              const int* __restrict__ offs, int ngrids,
                                              geno::KParams k, int stage, Cnt cnt) {
  const int* st = offs + BK_SLOW * (ngrids + 1);
  const int gb = (int)blockIdx.x;
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  const double* W = stage == 1 ? e.W : e.wst;
  slow_body<T>(e.geo, k, W, (const T*)e.fr[0], (const T*)e.fr[1], (T*)e.fl[0], (T*)e.fl[1],
               e.ctrl, stage == 1, cnt, e.queue[0], e.queue[1], gb - st[gi], e.slow_nb);
}

template <int STAGE, typename T, int BS>
__global__ void __launch_bounds__(BS) kb_update(const BEntry* __restrict__ tab,
                                                const int* __restrict__ offs, int ngrids,
                                                geno::KParams k, Cnt cnt) {
  const int* st = offs + BK_UPDATE * (ngrids + 1);
  const int gb = xcd_block();
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  if (STAGE == 1)
    update_body<2, 1, T>(e.geo, k, e.W, e.wst, (T*)e.dwst, e.r, (const T*)e.fl[0],
                         (const T*)e.fl[1], e.ctrl, e.part, cnt, gb - st[gi]);
  else
    update_body<2, 2, T>(e.geo, k, e.wst, e.W, (T*)e.dW, e.r, (const T*)e.fl[0],
                         (const T*)e.fl[1], e.ctrl, e.part, cnt, gb - st[gi]);
}

// The fused face step of a batch (the normal step inside the face kernels):
// kb_prep, one work-group per grid, then kb_fused per direction.
template <typename T>
__global__ void __launch_bounds__(1024) kb_prep(const BEntry* __restrict__ tab, geno::KParams k,
                                                int stage) {
  const BEntry& e = tab[blockIdx.x];
  if (stage == 1) reduce_dt(e.part, e.npart, e.ctrl, k.cfl, k.dt_fixed, nullptr, 0);
  if (threadIdx.x < 2) e.ctrl->qcount[threadIdx.x] = 0;
}

template <int DIR, typename T, bool WF, int VAR>
__global__ void __launch_bounds__(DIR == 0 ? FX_BS : FY_BS)
__attribute__((amdgpu_waves_per_eu(WF ? 1 : (DIR == 0 || VAR == FUSED_CHAR ? 2 : 4))))
kb_fused(const BEntry* __restrict__ tab, const int* __restrict__ offs, int ngrids,
         geno::KParams k) {
  const int* st = offs + (DIR == 0 ? BK_FUSED_X : BK_FUSED_Y) * (ngrids + 1);
  const int gb = xcd_block();
  const int gi = find_grid(st, ngrids, gb);
  const BEntry& e = tab[gi];
  const double* W = WF ? e.W : e.wst;
  const T* dW = (const T*)(WF ? e.dW : e.dwst);
  if (DIR == 0)
    fused_body<0, T, WF, VAR, FX_NT, FX_NN>(e.geo, k, W, dW, (T*)e.fr[0], (T*)e.fl[0], e.ctrl,
                                             e.queue[0], e.fnbu[0], gb - st[gi]);
  else
    fused_body<1, T, WF, VAR, FY_NT, FY_NN>(e.geo, k, W, dW, (T*)e.fr[1], (T*)e.fl[1], e.ctrl,
                                             e.queue[1], e.fnbu[1], gb - st[gi]);
}

// ---------------------------------------------------------------------------
// Persistent batched step: one launch advances every grid of the batch by one
// step. The work items are the work-groups of the twelve phases of a step
// (stages 1 and 2, each: normal x, faces x, normal y, faces y, tau > 0
// faces, update), numbered phase-major (every grid's blocks of a phase, then
// the next phase). A work-group takes the next item from a device counter and
// waits until the grid's previous phase is complete (a per-grid, per-phase
// count of finished blocks, release/acquire at device scope), runs the block
// with the phase's body, and counts it finished. Items are taken in an order
// in which every dependency precedes its dependents, and a work-group that
// waits holds an item whose dependencies were taken earlier by running
// work-groups that never wait on later items, so the launch always drains;
// each wait is also bounded (spin_limit): past it the launch sets an error
// flag, counts the block finished without running it, and goes on, so every
// work-group reaches the end. The last work-group to finish clears the
// counters for the next launch.
// A work-group is one wave, so that a work-group holding an item is wholly
// resident (no barrier of a holder waits on waves not yet launched), and the
// launch has at most as many work-groups as the largest phase has items.
// Waiting polls with relaxed loads and a sleep between polls; one acquire
// fence follows the last poll (an acquiring poll would invalidate the
// caches at every poll of every waiting wave).
// ---------------------------------------------------------------------------
constexpr int PB = 64;                   // threads per persistent work-group (one wave)
constexpr int PSEG = 12;                 // phases per step
struct PSegs {
  int start[PSEG + 1];                   // first item of each phase
};
// sched: [0] next item, [1] finished work-groups, [2] error flag (cleared by
// the host-side start of a call, never by the kernel); done: [grid][phase]
__device__ __forceinline__ int pseg_kind(int seg) {
  constexpr int order[6] = {BK_NORMAL_X, BK_FACES_X, BK_NORMAL_Y, BK_FACES_Y, BK_SLOW, BK_UPDATE};
  return order[seg % 6];
}

__global__ void __launch_bounds__(PB) kb_sched_clear(unsigned int* __restrict__ sched,
                                                     unsigned int* __restrict__ done, int n) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t < 4) sched[t] = 0u;
  for (int i = t; i < n; i += (int)(gridDim.x * blockDim.x)) done[i] = 0u;
}

template <typename T, bool CHAR>
__global__ void __launch_bounds__(PB) __attribute__((amdgpu_waves_per_eu(4))) kb_persist(const BEntry* __restrict__ tab,
                                                 const int* __restrict__ offs, int ngrids,
                                                 geno::KParams k, PSegs segs,
                                                 unsigned int* __restrict__ sched,
                                                 unsigned int* __restrict__ done,
                                                 unsigned int spin_limit) {
  __shared__ int s_item, s_run, s_last;
  const int total = segs.start[PSEG];
  const Cnt cnt{nullptr, 0};
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&sched[0], 1u);
    __syncthreads();
    const int it = s_item;
    if (it >= total) break;
    int seg = 0;
    while (segs.start[seg + 1] <= it) ++seg;
    const int kind = pseg_kind(seg);
    const int stage = seg < 6 ? 1 : 2;
    const int* st = offs + kind * (ngrids + 1);
    const int gb = it - segs.start[seg];
    const int gi = find_grid(st, ngrids, gb);
    const int lb = gb - st[gi];
    if (threadIdx.x == 0) {
      int run = 1;
      if (seg > 0) {
        const int* pst = offs + pseg_kind(seg - 1) * (ngrids + 1);
        const unsigned int need = (unsigned int)(pst[gi + 1] - pst[gi]);
        unsigned int* d = &done[gi * PSEG + seg - 1];
        unsigned int n = 0;
        while (__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          ++n;
          // past the bound, or once any wait of this launch has failed
          if (n > spin_limit ||
              ((n & 255u) == 0u &&
               __hip_atomic_load(&sched[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            run = 0;
            atomicOr(&sched[2], 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_run = run;
    }
    __syncthreads();
    if (s_run) {
      const BEntry& e = tab[gi];
      const double* W = stage == 1 ? e.W : e.wst;
      const T* dW = (const T*)(stage == 1 ? e.dW : e.dwst);
      switch (kind) {
        case BK_NORMAL_X:
          normal_body<0, T, CHAR>(e.geo, k, W, dW, (T*)e.fr[0], nullptr, e.ctrl,
                                  stage == 1 ? e.part : nullptr, e.npart, nullptr, 0, cnt, lb);
          break;
        case BK_FACES_X:
          faces_body<0, 1, T>(e.geo, k, W, (const T*)e.fr[0], (T*)e.fl[0], e.ctrl, stage == 1,
                              cnt, e.queue[0], lb);
          break;
        case BK_NORMAL_Y:
          normal_body<1, T, CHAR>(e.geo, k, W, dW, (T*)e.fr[1], nullptr, e.ctrl, nullptr, 0,
                                  nullptr, 0, cnt, lb);
          break;
        case BK_FACES_Y:
          faces_body<1, 1, T>(e.geo, k, W, (const T*)e.fr[1], (T*)e.fl[1], e.ctrl, stage == 1,
                              cnt, e.queue[1], lb);
          break;
        case BK_SLOW:
          slow_body<T>(e.geo, k, W, (const T*)e.fr[0], (const T*)e.fr[1], (T*)e.fl[0],
                       (T*)e.fl[1], e.ctrl, stage == 1, cnt, e.queue[0], e.queue[1], lb,
                       e.slow_nb);
          break;
        default:
          if (stage == 1)
            update_body<2, 1, T>(e.geo, k, e.W, e.wst, (T*)e.dwst, e.r,
                                 (const T*)e.fl[0], (const T*)e.fl[1], e.ctrl, e.part, cnt, lb);
          else
            update_body<2, 2, T>(e.geo, k, e.wst, e.W, (T*)e.dW, e.r,
                                 (const T*)e.fl[0], (const T*)e.fl[1], e.ctrl, e.part, cnt, lb);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&done[gi * PSEG + seg], 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  // the last work-group to finish clears the counters for the next launch
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(&sched[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
             gridDim.x - 1u;
  __syncthreads();
  if (s_last) {
    for (int i = (int)threadIdx.x; i < ngrids * PSEG; i += PB) done[i] = 0u;
    if (threadIdx.x == 0) {
      sched[0] = 0u;
      sched[1] = 0u;
    }
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
struct Layout {
  size_t ctrl, part, queue[2], gate, wst, dwst, r, fr[2], fl[2], total;
  size_t nstate;   // elements per field plane
  int npart;
};

// bytes of one element of dW and of the face buffers
size_t elem_bytes(const geno_grid* g) {
  return g->params.precision == GENO_MIXED ? sizeof(float) : sizeof(double);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline unsigned nblocks(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

Layout layout_of(const geno_grid* g) {
  Layout L{};
  const int nv = g->ndim == 2 ? 4 : 3;
  const size_t es = elem_bytes(g);
  L.nstate = (size_t)g->rows * g->pitch;
  L.npart = (int)nblocks((size_t)g->nx * g->ny);
  size_t off = 0;
  L.ctrl = off;
  off = align256(off + sizeof(Ctrl));
  L.part = off;   // room for the partials of work-groups as small as 64 lanes
  off = align256(off + ((size_t)g->nx * g->ny / 64 + 1) * sizeof(double));
  if (g->ndim == 2) {
    L.queue[0] = off;
    off = align256(off + (size_t)g->ny * (g->nx + 1) * sizeof(unsigned int));
    L.queue[1] = off;
    off = align256(off + (size_t)(g->ny + 1) * g->nx * sizeof(unsigned int));
    L.gate = off;   // learned-gate flags, [dir][ny][nx]
    off = align256(off + 2 * (size_t)g->nx * g->ny);
  }
  L.wst = off;
  off = align256(off + L.nstate * nv * sizeof(double));
  L.dwst = off;
  off = align256(off + L.nstate * nv * g->ndim * es);
  L.r = off;
  off = align256(off + L.nstate * nv * sizeof(double));
  if (g->ndim == 2) {
    L.fr[0] = off;
    off = align256(off + (size_t)20 * (g->ny + 2) * (g->nx + 1) * es);
    L.fr[1] = off;
    off = align256(off + (size_t)20 * (g->ny + 1) * (g->nx + 2) * es);
    L.fl[0] = off;
    off = align256(off + (size_t)16 * g->ny * xface_pitch(g->nx) * es);
    L.fl[1] = off;
    off = align256(off + (size_t)16 * (g->ny + 1) * g->nx * es);
  } else {
    L.fl[0] = off;
    off = align256(off + (size_t)15 * (g->nx + 1) * es);
  }
  L.total = off;
  return L;
}

int check_params(const geno_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  if (p->version != GENO_ABI_VERSION)
    return fail(GENO_EVERSION, "params version %d != %d", p->version, GENO_ABI_VERSION);
  if (p->precision != GENO_F64 && p->precision != GENO_MIXED)
    return fail(GENO_EINVAL, "unsupported precision %d", p->precision);
  if (!(p->dt_fixed >= 0.0)) return fail(GENO_EINVAL, "dt_fixed must be >= 0");
  if (!(p->eps_ulps >= 0.0)) return fail(GENO_EINVAL, "eps_ulps must be >= 0");
  if (!(p->gate_delta >= 0.0 && p->gate_delta < 1.0))
    return fail(GENO_EINVAL, "gate_delta must be in [0, 1)");
  if (p->r != 2.0 || p->rL != 2.0) return fail(GENO_EINVAL, "only r = rL = 2 are implemented");
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->C > 0.0) || !(p->cfl > 0.0))
    return fail(GENO_EINVAL, "gamma > 1, eps > 0, C > 0 and cfl > 0 are required");
  if (!(p->d[0] > 0.0 && p->d[1] > 0.0 && p->d[2] > 0.0))
    return fail(GENO_EINVAL, "linear weights d must be positive");
  if (!(p->tau_c1 >= 0.0) || !(p->tau_c2 >= 0.0))
    return fail(GENO_EINVAL, "tau coefficients must be >= 0");
  for (int i = 0; i < 4; ++i)
    if (p->bc[i] != GENO_BC_PERIODIC && p->bc[i] != GENO_BC_TRANSMISSIVE &&
        p->bc[i] != GENO_BC_REFLECTING && p->bc[i] != GENO_BC_FIXED)
      return fail(GENO_EINVAL, "bad boundary code %d", p->bc[i]);
  if ((p->bc[0] == GENO_BC_PERIODIC) != (p->bc[1] == GENO_BC_PERIODIC) ||
      (p->bc[2] == GENO_BC_PERIODIC) != (p->bc[3] == GENO_BC_PERIODIC))
    return fail(GENO_EINVAL, "periodic boundaries must be set on both sides of an axis");
  if (p->variables != GENO_VARS_CONSERVATIVE && p->variables != GENO_VARS_CHARACTERISTIC)
    return fail(GENO_EINVAL, "bad variables code %d", p->variables);
  if (p->fuse < 0 || p->fuse > 2) return fail(GENO_EINVAL, "fuse must be 0, 1 or 2");
  return GENO_OK;
}

int check_grid(const geno_grid* g) {
  if (!g) return fail(GENO_EINVAL, "null grid");
  int rc = check_params(&g->params);
  if (rc) return rc;
  if (g->ndim != 1 && g->ndim != 2) return fail(GENO_EINVAL, "ndim must be 1 or 2");
  for (int i = 0; i < 4; ++i)
    if (g->ndim == 2 && g->params.bc[i] == GENO_BC_FIXED)
      return fail(GENO_EINVAL, "fixed-state ends are available in 1-D only");
  if (g->params.variables == GENO_VARS_CHARACTERISTIC && g->ndim == 2 &&
      g->params.gate_delta > 0.0)
    return fail(GENO_EINVAL, "the learned gate works on conservative variables only");
  if (g->nx < 1 || g->ny < 1 || (g->ndim == 1 && g->ny != 1))
    return fail(GENO_EINVAL, "bad grid size");
  if (g->pitch < g->nx + 2 * NG || g->rows != (g->ndim == 2 ? g->ny + 2 * NG : 1))
    return fail(GENO_EINVAL, "grid pitch/rows inconsistent (use geno_grid_init)");
  // periodic and mirror images must exist: 2 ghost layers need 2 cells
  const auto imaged = [&](int side) {
    return g->params.bc[side] == GENO_BC_PERIODIC || g->params.bc[side] == GENO_BC_REFLECTING;
  };
  if (((imaged(0) || imaged(1)) && g->nx < NG) ||
      (g->ndim == 2 && (imaged(2) || imaged(3)) && g->ny < NG))
    return fail(GENO_EINVAL, "periodic or reflecting axis needs at least %d cells", NG);
  // 32-bit thread indexing: two lanes per face and 20 face-row planes
  if ((size_t)(g->nx + 4) * (g->ny + 4) * 20 > (size_t)0x7fffffff)
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
  k.dt_fixed = p.dt_fixed;
  k.eps_ulps = p.eps_ulps;
  k.gate = (p.gate_delta > 0.0 && g->ndim == 2) ? 1 : 0;
  k.gate_thr = 1.0 - p.gate_delta;
  k.charvars = p.variables == GENO_VARS_CHARACTERISTIC ? 1 : 0;
  k.fuse = p.fuse;
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

template <typename T>
struct Bufs {
  Ctrl* ctrl;
  double* part;
  unsigned int* queue[2];
  unsigned char* gate;
  double *wst, *r;
  T *dwst, *fr[2], *fl[2];
};

template <typename T>
Bufs<T> bufs_of(char* ws, const Layout& L, int ndim) {
  Bufs<T> b{};
  b.ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  b.part = reinterpret_cast<double*>(ws + L.part);
  b.wst = reinterpret_cast<double*>(ws + L.wst);
  b.dwst = reinterpret_cast<T*>(ws + L.dwst);
  b.r = reinterpret_cast<double*>(ws + L.r);
  b.fl[0] = reinterpret_cast<T*>(ws + L.fl[0]);
  if (ndim == 2) {
    b.queue[0] = reinterpret_cast<unsigned int*>(ws + L.queue[0]);
    b.queue[1] = reinterpret_cast<unsigned int*>(ws + L.queue[1]);
    b.gate = reinterpret_cast<unsigned char*>(ws + L.gate);
    b.fr[0] = reinterpret_cast<T*>(ws + L.fr[0]);
    b.fr[1] = reinterpret_cast<T*>(ws + L.fr[1]);
    b.fl[1] = reinterpret_cast<T*>(ws + L.fl[1]);
  }
  return b;
}

template <typename T>
int launch_init(const geno_grid* g, const Geo& geo, double gamma, double* W, T* dW,
                const Bufs<T>& B, hipStream_t s) {
  const size_t n = (size_t)g->nx * g->ny;
  if (g->ndim == 2)
    HIP_TRY(launch(GENO_K_INIT, k_init<2, T>, nblocks(n), s, geo, gamma, W, dW, B.part, B.ctrl));
  else
    HIP_TRY(launch(GENO_K_INIT, k_init<1, T>, nblocks(n), s, geo, gamma, W, dW, B.part, B.ctrl));
  // 1-D fixed ends: the caller's ghost cells also serve the stage state
  // (NG cells of each of the three field rows)
  for (int side = 0; side < 2 && g->ndim == 1; ++side) {
    if (g->params.bc[side] != GENO_BC_FIXED) continue;
    const size_t col = side == 0 ? 0 : (size_t)g->nx + NG;
    HIP_TRY(hipMemcpy2DAsync(B.wst + col, g->pitch * sizeof(double), W + col,
                             g->pitch * sizeof(double), NG * sizeof(double), 3,
                             hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpy2DAsync(B.dwst + col, g->pitch * sizeof(T), dW + col, g->pitch * sizeof(T),
                             NG * sizeof(T), 3, hipMemcpyDeviceToDevice, s));
  }
  return GENO_OK;
}

// launch sizes of gks_step
size_t face_rows(const geno_grid* g, int dir) {
  return dir == 0 ? (size_t)(g->ny + 2) * (g->nx + 1) : (size_t)(g->ny + 1) * (g->nx + 2);
}
// threads of the normal step: one per (variable, face-row entry), or one
// per entry with characteristic variables
bool char2d(const geno_grid* g) {
  return g->ndim == 2 && g->params.variables == GENO_VARS_CHARACTERISTIC;
}
size_t normal_threads(const geno_grid* g, int dir) {
  return (char2d(g) ? 1 : 4) * face_rows(g, dir);
}
size_t faces_of(const geno_grid* g, int dir) {
  return dir == 0 ? (size_t)g->ny * (g->nx + 1) : (size_t)(g->ny + 1) * g->nx;
}
unsigned slow_blocks(const geno_grid* g) {
  return (unsigned)std::min<size_t>(SLOW_BLOCKS, nblocks(faces_of(g, 0) + faces_of(g, 1)));
}
// the largest grid of a counted launch (slots per kind and class)
int count_cap(const geno_grid* g) {
  size_t m = nblocks((size_t)g->nx * g->ny);
  if (g->ndim == 2) {
    for (int d = 0; d < 2; ++d) {
      m = std::max<size_t>(m, nblocks(4 * face_rows(g, d)));
      m = std::max<size_t>(m, nblocks(2 * faces_of(g, d)));
    }
    // the normal-step launch over both directions
    m = std::max<size_t>(m, nblocks(4 * face_rows(g, 0)) + nblocks(4 * face_rows(g, 1)));
    m = std::max<size_t>(m, slow_blocks(g));
  } else {
    m = std::max<size_t>(m, nblocks((size_t)g->nx + 1));
  }
  return (int)m;
}

// work-groups of a gate launch over nc cells
unsigned gate_blocks(size_t nc) {
  const size_t tiles = (nc + 15) / 16;
  return (unsigned)((tiles + 4 * GATE_TILES - 1) / (4 * GATE_TILES));
}

// Whether a 2-D stage takes the fused face kernels (tiles: the fused
// work-groups of both directions over every grid of the launch). Never with
// work counting (it counts in the separate normal-step launch). params.fuse
// 2: always; 0: never; 1 (automatic): when the launch has at least
// FUSE_MIN_TILES tiles, and not for characteristic variables in the mixed
// form. Measured crossovers: a 256^2 grid (1398 tiles) ran 11-13 % slower
// fused, 512^2 (4970 tiles) within 2 %, 1024^2 and larger 12-28 % faster;
// mixed-precision characteristic variables, where the fused kernels run at
// the characteristic normal step's register count (163-166 VGPRs against
// 73-81 for the float face kernels), ran slower at 2048^2 (3230 against 3435
// Mcell-updates/s per stage).
constexpr size_t FUSE_MIN_TILES = 4096;
template <typename T>
bool use_fused(const geno::KParams& k, const Cnt& cnt, size_t tiles) {
  if (cnt.p || k.fuse == 0) return false;
  if (k.fuse == 2) return true;
  return tiles >= FUSE_MIN_TILES && !(k.charvars && sizeof(T) == sizeof(float));
}

// the fused face launches of one stage (both directions)
template <typename T, bool WF, int VAR>
int launch_fused(const Geo& geo, const geno::KParams& k, const Bufs<T>& B, const double* Win,
                 const T* dWin, const unsigned char* gx, const unsigned char* gy,
                 hipStream_t s) {
  HIP_TRY(launch_bs(GENO_K_FUSED_X, k_fused2d<0, T, WF, VAR, FX_NT, FX_NN>, fused_blocks(geo, 0),
                    FX_BS, s, geo, k, Win, dWin, B.fr[0], B.fl[0], B.ctrl, B.queue[0],
                    fused_nbu(geo, 0), gx));
  HIP_TRY(launch_bs(GENO_K_FUSED_Y, k_fused2d<1, T, WF, VAR, FY_NT, FY_NN>, fused_blocks(geo, 1),
                    FY_BS, s, geo, k, Win, dWin, B.fr[1], B.fl[1], B.ctrl, B.queue[1],
                    fused_nbu(geo, 1), gy));
  return GENO_OK;
}

// one stage of gks_step: faces and update
template <typename T>
int launch_stage(const geno_grid* g, const Geo& geo, const geno::KParams& k, const Bufs<T>& B,
                 int npart, const double* Win, const T* dWin, int stage, double* dt_out, int step,
                 double* Wfinal, T* dWfinal, const Cnt& cnt, hipStream_t s) {
  const int want_F = stage == 1;
  const double* part = stage == 1 ? B.part : nullptr;   // dt of the step is reduced once
  if (g->ndim == 2) {
    const unsigned char* gx = nullptr;
    const unsigned char* gy = nullptr;
    if (k.gate) {
      // the gate is evaluated once per step, on the state at its start; the
      // second stage reuses those flags
      const size_t nc = (size_t)g->nx * g->ny;
      const unsigned nbg = gate_blocks(nc);
      if (stage == 1) {
        HIP_TRY(launch(GENO_K_GATE, k_gate<0, T, 0>, nbg, s, geo, Win, dWin, (float)k.gate_thr,
                       B.gate, (float*)nullptr));
        HIP_TRY(launch(GENO_K_GATE, k_gate<1, T, 0>, nbg, s, geo, Win, dWin, (float)k.gate_thr,
                       B.gate + nc, (float*)nullptr));
      }
      gx = B.gate;
      gy = B.gate + nc;
    }
    if (use_fused<T>(k, cnt, (size_t)fused_blocks(geo, 0) + fused_blocks(geo, 1))) {
      HIP_TRY(launch_bs(-1, k_stage_prep, 1, 1024, s, part, npart, B.ctrl, k.cfl, k.dt_fixed,
                        dt_out, step));
      int rc;
      if (want_F)
        rc = k.charvars ? launch_fused<T, true, FUSED_CHAR>(geo, k, B, Win, dWin, gx, gy, s)
             : k.gate   ? launch_fused<T, true, FUSED_GATE>(geo, k, B, Win, dWin, gx, gy, s)
                        : launch_fused<T, true, FUSED_PLAIN>(geo, k, B, Win, dWin, gx, gy, s);
      else
        rc = k.charvars ? launch_fused<T, false, FUSED_CHAR>(geo, k, B, Win, dWin, gx, gy, s)
             : k.gate   ? launch_fused<T, false, FUSED_GATE>(geo, k, B, Win, dWin, gx, gy, s)
                        : launch_fused<T, false, FUSED_PLAIN>(geo, k, B, Win, dWin, gx, gy, s);
      if (rc) return rc;
      if (want_F)
        HIP_TRY(launch(GENO_K_SLOW, k_slow2d<T, true>, slow_blocks(g), s, geo, k, Win, B.fr[0],
                       B.fr[1], B.fl[0], B.fl[1], B.ctrl, cnt, B.queue[0], B.queue[1]));
      else
        HIP_TRY(launch(GENO_K_SLOW, k_slow2d<T, false>, slow_blocks(g), s, geo, k, Win, B.fr[0],
                       B.fr[1], B.fl[0], B.fl[1], B.ctrl, cnt, B.queue[0], B.queue[1]));
    } else {
    const unsigned nnx = nblocks(normal_threads(g, 0)), nny = nblocks(normal_threads(g, 1));
    if (k.charvars)
      HIP_TRY(launch(GENO_K_NORMAL_XY, k_normal2d_xy<T, true>, nnx + nny, s, geo, k, Win, dWin,
                     B.fr[0], B.fr[1], B.ctrl, part, npart, dt_out, step, cnt, gx, gy, (int)nnx));
    else
      HIP_TRY(launch(GENO_K_NORMAL_XY, k_normal2d_xy<T, false>, nnx + nny, s, geo, k, Win, dWin,
                     B.fr[0], B.fr[1], B.ctrl, part, npart, dt_out, step, cnt, gx, gy, (int)nnx));
    if (want_F) {
      HIP_TRY(launch(GENO_K_FACES_X, k_faces2d<0, 1, T, true>, nblocks(2 * faces_of(g, 0)), s, geo,
                     k, Win, B.fr[0], B.fl[0], B.ctrl, cnt, B.queue[0]));
      HIP_TRY(launch(GENO_K_FACES_Y, k_faces2d<1, 1, T, true>, nblocks(2 * faces_of(g, 1)), s, geo,
                     k, Win, B.fr[1], B.fl[1], B.ctrl, cnt, B.queue[1]));
      HIP_TRY(launch(GENO_K_SLOW, k_slow2d<T, true>, slow_blocks(g), s, geo, k, Win, B.fr[0],
                     B.fr[1], B.fl[0], B.fl[1], B.ctrl, cnt, B.queue[0], B.queue[1]));
    } else {
      HIP_TRY(launch(GENO_K_FACES_X, k_faces2d<0, 1, T, false>, nblocks(2 * faces_of(g, 0)), s,
                     geo, k, Win, B.fr[0], B.fl[0], B.ctrl, cnt, B.queue[0]));
      HIP_TRY(launch(GENO_K_FACES_Y, k_faces2d<1, 1, T, false>, nblocks(2 * faces_of(g, 1)), s,
                     geo, k, Win, B.fr[1], B.fl[1], B.ctrl, cnt, B.queue[1]));
      HIP_TRY(launch(GENO_K_SLOW, k_slow2d<T, false>, slow_blocks(g), s, geo, k, Win, B.fr[0],
                     B.fr[1], B.fl[0], B.fl[1], B.ctrl, cnt, B.queue[0], B.queue[1]));
    }
    }
  } else {
    if (part)
      HIP_TRY(launch(-1, k_dt1d, 1, s, B.part, npart, B.ctrl, k.cfl, k.dt_fixed, dt_out, step));
    HIP_TRY(launch(GENO_K_FACES_1D, k_faces1d<1, T>, nblocks((size_t)g->nx + 1), s, geo, k, Win,
                   dWin, B.fl[0], (double*)nullptr, B.ctrl, want_F, cnt));
  }
  const unsigned nc = nblocks((size_t)g->nx * g->ny);
  const int kind = stage == 1 ? GENO_K_UPDATE_1 : GENO_K_UPDATE_2;
  const T* fy = g->ndim == 2 ? B.fl[1] : nullptr;
  if (g->ndim == 2) {
    if (stage == 1)
      HIP_TRY(launch(kind, k_update<2, 1, T>, nc, s, geo, k, Win, B.wst, B.dwst, B.r, B.fl[0], fy,
                     B.ctrl, B.part, cnt));
    else
      HIP_TRY(launch(kind, k_update<2, 2, T>, nc, s, geo, k, Win, Wfinal, dWfinal, B.r, B.fl[0],
                     fy, B.ctrl, B.part, cnt));
  } else {
    if (stage == 1)
      HIP_TRY(launch(kind, k_update<1, 1, T>, nc, s, geo, k, Win, B.wst, B.dwst, B.r, B.fl[0], fy,
                     B.ctrl, B.part, cnt));
    else
      HIP_TRY(launch(kind, k_update<1, 2, T>, nc, s, geo, k, Win, Wfinal, dWfinal, B.r, B.fl[0],
                     fy, B.ctrl, B.part, cnt));
  }
  return GENO_OK;
}

template <typename T>
int reconstruct_t(const geno_grid* g, double* W, T* dW, int dir, T* face_state, double* chi,
                  void* ws, hipStream_t s) {
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  const Bufs<T> B = bufs_of<T>((char*)ws, L, g->ndim);
  int rc = launch_init<T>(g, geo, k.gamma, W, dW, B, s);
  if (rc) return rc;
  const Cnt none{nullptr, 0};
  if (g->ndim == 1) {
    HIP_TRY(launch(-1, k_faces1d<0, T>, nblocks((size_t)g->nx + 1), s, geo, k, (const double*)W,
                   (const T*)dW, face_state, chi, (Ctrl*)nullptr, 0, none));
  } else if (dir == 0) {
    HIP_TRY(launch(-1, k.charvars ? k_normal2d<0, T, true> : k_normal2d<0, T, false>,
                   nblocks(normal_threads(g, 0)), s, geo, k, (const double*)W, (const T*)dW,
                   B.fr[0], chi, (Ctrl*)nullptr, (const double*)nullptr, 0, (double*)nullptr, 0,
                   none, (const unsigned char*)nullptr));
    HIP_TRY(launch(-1, k_faces2d<0, 0, T, true>, nblocks(2 * faces_of(g, 0)), s, geo, k,
                   (const double*)W, (const T*)B.fr[0], face_state, (Ctrl*)nullptr, none,
                   (unsigned int*)nullptr));
  } else {
    HIP_TRY(launch(-1, k.charvars ? k_normal2d<1, T, true> : k_normal2d<1, T, false>,
                   nblocks(normal_threads(g, 1)), s, geo, k, (const double*)W, (const T*)dW,
                   B.fr[1], chi, (Ctrl*)nullptr, (const double*)nullptr, 0, (double*)nullptr, 0,
                   none, (const unsigned char*)nullptr));
    HIP_TRY(launch(-1, k_faces2d<1, 0, T, true>, nblocks(2 * faces_of(g, 1)), s, geo, k,
                   (const double*)W, (const T*)B.fr[1], face_state, (Ctrl*)nullptr, none,
                   (unsigned int*)nullptr));
  }
  return GENO_OK;
}

template <typename T>
int flux_t(const geno_grid* g, const T* face_state, double dt, int dir, T* F, T* Ft, T* Wint,
           hipStream_t s) {
  const geno::KParams k = kparams(g);
  if (g->ndim == 1) {
    const int nf = g->nx + 1;
    HIP_TRY(launch(-1, k_flux_points<3, T>, nblocks(nf), s, nf, 1, 0, k, g->dx, g->dy, dt,
                   face_state, F, Ft, Wint));
  } else {
    const int nf = dir == 0 ? g->ny * (g->nx + 1) : (g->ny + 1) * g->nx;
    const double hn = dir == 0 ? g->dx : g->dy, ht = dir == 0 ? g->dy : g->dx;
    HIP_TRY(launch(-1, k_flux_points<4, T>, nblocks(nf), s, nf, 2, dir, k, hn, ht, dt, face_state,
                   F, Ft, Wint));
  }
  return GENO_OK;
}

template <typename T>
int step_t(const geno_grid* g, double* W, T* dW, void* ws, int nsteps, double* dt_out,
           const Cnt& cnt, hipStream_t s, Ctrl** ctrl_out) {
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  const Bufs<T> B = bufs_of<T>((char*)ws, L, g->ndim);
  *ctrl_out = B.ctrl;
  int rc = launch_init<T>(g, geo, k.gamma, W, dW, B, s);
  if (rc) return rc;
  for (int n = 0; n < nsteps; ++n) {
    rc = launch_stage<T>(g, geo, k, B, L.npart, W, dW, 1, dt_out, n, nullptr, nullptr, cnt, s);
    if (rc) return rc;
    rc = launch_stage<T>(g, geo, k, B, L.npart, B.wst, B.dwst, 2, nullptr, n, W, dW, cnt, s);
    if (rc) return rc;
  }
  return GENO_OK;
}

// ---------------------------------------------------------------------------
// batched host side
// ---------------------------------------------------------------------------
struct BatchPlan {
  int ngrids = 0;
  int bs[BK_N] = {};
  int nb[BK_N] = {};             // work-groups of each launch kind (all grids)
  std::vector<BEntry> tab;
  std::vector<int> offs;         // [kind][ngrids + 1] range starts
  std::vector<size_t> goff;      // workspace offset of each grid
  size_t tab_off = 0, offs_off = 0, sched_off = 0, total = 0;
  PSegs segs{};                  // persistent step: first item of each phase
};

bool bs_ok(int b) { return b == 128 || b == 256 || b == 512; }
unsigned nblocks_bs(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int tuning_of(const geno_tuning* t, geno_tuning* out) {
  geno_tuning d{GENO_ABI_VERSION, 256, 256, 256, 256, 2048};
  if (t) {
    if (t->version != GENO_ABI_VERSION)
      return fail(GENO_EVERSION, "tuning version %d != %d", t->version, GENO_ABI_VERSION);
    if (t->block_normal) d.block_normal = t->block_normal;
    if (t->block_faces) d.block_faces = t->block_faces;
    if (t->block_slow) d.block_slow = t->block_slow;
    if (t->block_update) d.block_update = t->block_update;
    if (t->slow_faces_per_block) d.slow_faces_per_block = t->slow_faces_per_block;
  }
  if (!bs_ok(d.block_normal) || !bs_ok(d.block_faces) || !bs_ok(d.block_slow) ||
      !bs_ok(d.block_update))
    return fail(GENO_EINVAL, "work-group sizes must be 128, 256 or 512");
  if (d.slow_faces_per_block < 1) return fail(GENO_EINVAL, "slow_faces_per_block must be >= 1");
  *out = d;
  return GENO_OK;
}

// the method parameters every grid of a batch shares (all but bc)
bool same_method(const geno_params& a, const geno_params& b) {
  return a.version == b.version && a.precision == b.precision && a.gamma == b.gamma &&
         a.C == b.C && a.eps == b.eps && a.r == b.r && a.rL == b.rL && a.d[0] == b.d[0] &&
         a.d[1] == b.d[1] && a.d[2] == b.d[2] && a.tau_c1 == b.tau_c1 &&
         a.tau_c2 == b.tau_c2 && a.cfl == b.cfl && a.dt_fixed == b.dt_fixed &&
         a.eps_ulps == b.eps_ulps && a.variables == b.variables && a.fuse == b.fuse;
}

// devices on which a network has been loaded (geno_mlp_load)
bool g_mlp_loaded[64] = {};

int check_gate(const geno_grid* g) {
  if (g->params.gate_delta > 0.0 && g->ndim == 2) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || !g_mlp_loaded[dev])
      return fail(GENO_EINVAL, "gate_delta > 0 but no network is loaded (geno_mlp_load)");
  }
  return GENO_OK;
}

// float to bfloat16 bits, rounding to nearest even
unsigned short f2bf(float f) {
  unsigned int u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

int check_batch(int ngrids, const geno_grid* grids) {
  if (ngrids < 1 || ngrids > GENO_BATCH_MAX)
    return fail(GENO_EINVAL, "ngrids must be in [1, %d]", GENO_BATCH_MAX);
  if (!grids) return fail(GENO_EINVAL, "null grids");
  for (int i = 0; i < ngrids; ++i) {
    int rc = check_grid(&grids[i]);
    if (rc) return rc;
    if (grids[i].ndim != 2) return fail(GENO_EINVAL, "batched grids must be 2-D (grid %d)", i);
    if (!same_method(grids[i].params, grids[0].params))
      return fail(GENO_EINVAL, "grid %d: method parameters differ from grid 0", i);
    if (grids[i].params.gate_delta > 0.0)
      return fail(GENO_EINVAL, "the learned gate is not available in batched steps");
  }
  return GENO_OK;
}

// Work-group ranges, table and workspace layout of a batch (no device access).
int plan_batch(int ngrids, const geno_grid* grids, const geno_tuning& t, BatchPlan* P) {
  P->ngrids = ngrids;
  P->bs[BK_INIT] = P->bs[BK_UPDATE] = t.block_update;
  P->bs[BK_NORMAL_X] = P->bs[BK_NORMAL_Y] = t.block_normal;
  P->bs[BK_FACES_X] = P->bs[BK_FACES_Y] = t.block_faces;
  P->bs[BK_SLOW] = t.block_slow;
  P->bs[BK_FUSED_X] = FX_BS;
  P->bs[BK_FUSED_Y] = FY_BS;
  P->bs[BK_PREP] = 1024;
  P->offs.assign((size_t)BK_N * (ngrids + 1), 0);
  P->tab.assign(ngrids, BEntry{});
  P->goff.assign(ngrids, 0);
  size_t off = 0;
  P->tab_off = off;
  off = align256(off + sizeof(BEntry) * ngrids);
  P->offs_off = off;
  off = align256(off + sizeof(int) * P->offs.size());
  P->sched_off = off;   // persistent step: 4 scheduler words, then [grid][phase] counts
  off = align256(off + sizeof(unsigned int) * (4 + (size_t)PSEG * ngrids));
  long long cnt[BK_N] = {};
  for (int i = 0; i < ngrids; ++i) {
    const geno_grid* g = &grids[i];
    const size_t ncell = (size_t)g->nx * g->ny;
    const size_t f = faces_of(g, 0) + faces_of(g, 1);
    const long long nbk[BK_N] = {
        nblocks_bs(ncell, t.block_update),
        nblocks_bs(normal_threads(g, 0), t.block_normal),
        nblocks_bs(2 * faces_of(g, 0), t.block_faces),
        nblocks_bs(normal_threads(g, 1), t.block_normal),
        nblocks_bs(2 * faces_of(g, 1), t.block_faces),
        std::min<long long>(1024, std::max<long long>(1, (long long)((f + t.slow_faces_per_block - 1) /
                                                                  t.slow_faces_per_block))),
        nblocks_bs(ncell, t.block_update),
        fused_blocks(geo_of(g), 0),
        fused_blocks(geo_of(g), 1),
        1};
    for (int k = 0; k < BK_N; ++k) {
      P->offs[(size_t)k * (ngrids + 1) + i] = (int)cnt[k];
      cnt[k] += nbk[k];
      if (cnt[k] > 0x7fffffff / 1024) return fail(GENO_EINVAL, "batch too large");
    }
    P->goff[i] = off;
    const Layout L = layout_of(g);
    off = align256(off + L.total);
    BEntry& e = P->tab[i];
    e.geo = geo_of(g);
    e.npart = (int)nbk[BK_UPDATE];
    e.slow_nb = (int)nbk[BK_SLOW];
    e.fnbu[0] = fused_nbu(e.geo, 0);
    e.fnbu[1] = fused_nbu(e.geo, 1);
  }
  for (int k = 0; k < BK_N; ++k) {
    P->offs[(size_t)k * (ngrids + 1) + ngrids] = (int)cnt[k];
    P->nb[k] = (int)cnt[k];
  }
  P->segs.start[0] = 0;
  const int order[6] = {BK_NORMAL_X, BK_FACES_X, BK_NORMAL_Y, BK_FACES_Y, BK_SLOW, BK_UPDATE};
  for (int q = 0; q < PSEG; ++q) {
    const long long next = (long long)P->segs.start[q] + P->nb[order[q % 6]];
    if (next > 0x7fffffff) return fail(GENO_EINVAL, "batch too large");
    P->segs.start[q + 1] = (int)next;
  }
  P->total = off;
  return GENO_OK;
}

// Device pointers of the table entries for workspace ws.
void bind_batch(BatchPlan* P, char* ws, void* const* W, void* const* dW, const geno_grid* grids) {
  for (int i = 0; i < P->ngrids; ++i) {
    const Layout L = layout_of(&grids[i]);
    char* b = ws + P->goff[i];
    BEntry& e = P->tab[i];
    e.W = (double*)W[i];
    e.dW = dW[i];
    e.ctrl = reinterpret_cast<Ctrl*>(b + L.ctrl);
    e.part = reinterpret_cast<double*>(b + L.part);
    e.queue[0] = reinterpret_cast<unsigned int*>(b + L.queue[0]);
    e.queue[1] = reinterpret_cast<unsigned int*>(b + L.queue[1]);
    e.wst = reinterpret_cast<double*>(b + L.wst);
    e.r = reinterpret_cast<double*>(b + L.r);
    e.dwst = b + L.dwst;
    e.fr[0] = b + L.fr[0];
    e.fr[1] = b + L.fr[1];
    e.fl[0] = b + L.fl[0];
    e.fl[1] = b + L.fl[1];
  }
}

#define GO_BS(BSV, KIND, KERN, NB, ...)                                                  \
  switch (BSV) {                                                                         \
    case 128: return launch_bs(KIND, KERN<128>, NB, 128, s, __VA_ARGS__);                \
    case 512: return launch_bs(KIND, KERN<512>, NB, 512, s, __VA_ARGS__);                \
    default: return launch_bs(KIND, KERN<256>, NB, 256, s, __VA_ARGS__);                 \
  }

template <typename T, bool CHAR = false>
struct BatchK {
  template <int BS> static constexpr auto init = kb_init<T, BS>;
  template <int BS> static constexpr auto nx = kb_normal<0, T, BS, CHAR>;
  template <int BS> static constexpr auto ny = kb_normal<1, T, BS, CHAR>;
  template <int BS> static constexpr auto fx = kb_faces<0, T, BS>;
  template <int BS> static constexpr auto fy = kb_faces<1, T, BS>;
  template <int BS> static constexpr auto slow = kb_slow<T, BS>;
  template <int BS> static constexpr auto up1 = kb_update<1, T, BS>;
  template <int BS> static constexpr auto up2 = kb_update<2, T, BS>;
};

template <typename T>
hipError_t go_init(const BatchPlan& P, const BEntry* tab, const int* offs, double gamma,
                   hipStream_t s) {
  GO_BS(P.bs[BK_INIT], GENO_K_INIT, BatchK<T>::template init, P.nb[BK_INIT], tab, offs, P.ngrids,
        gamma)
}

template <typename T>
hipError_t go_phase(int phase, const BatchPlan& P, const BEntry* tab, const int* offs,
                    const geno::KParams& k, int stage, const Cnt& cnt, hipStream_t s) {
  const int ng = P.ngrids;
  using BC = BatchK<T, true>;   // normal step on characteristic variables
  switch (phase) {
    case BK_NORMAL_X:
      if (k.charvars)
        GO_BS(P.bs[phase], GENO_K_NORMAL_X, BC::template nx, P.nb[phase], tab,
              offs, ng, k, stage, cnt)
      GO_BS(P.bs[phase], GENO_K_NORMAL_X, BatchK<T>::template nx, P.nb[phase], tab, offs, ng, k,
            stage, cnt)
    case BK_FACES_X:
      GO_BS(P.bs[phase], GENO_K_FACES_X, BatchK<T>::template fx, P.nb[phase], tab, offs, ng, k,
            stage, cnt)
    case BK_NORMAL_Y:
      if (k.charvars)
        GO_BS(P.bs[phase], GENO_K_NORMAL_Y, BC::template ny, P.nb[phase], tab,
              offs, ng, k, stage, cnt)
      GO_BS(P.bs[phase], GENO_K_NORMAL_Y, BatchK<T>::template ny, P.nb[phase], tab, offs, ng, k,
            stage, cnt)
    case BK_FACES_Y:
      GO_BS(P.bs[phase], GENO_K_FACES_Y, BatchK<T>::template fy, P.nb[phase], tab, offs, ng, k,
            stage, cnt)
    case BK_SLOW:
      GO_BS(P.bs[phase], GENO_K_SLOW, BatchK<T>::template slow, P.nb[phase], tab, offs, ng, k,
            stage, cnt)
    default:
      if (stage == 1) {
        GO_BS(P.bs[BK_UPDATE], GENO_K_UPDATE_1, BatchK<T>::template up1, P.nb[BK_UPDATE], tab,
              offs, ng, k, cnt)
      } else {
        GO_BS(P.bs[BK_UPDATE], GENO_K_UPDATE_2, BatchK<T>::template up2, P.nb[BK_UPDATE], tab,
              offs, ng, k, cnt)
      }
  }
}

template <typename T>
int batch_step(const BatchPlan& P, const BEntry* tab, const int* offs, const geno::KParams& k,
               const Cnt& cnt, hipStream_t s) {
  const int ng = P.ngrids;
  const bool fused =
      use_fused<T>(k, cnt, (size_t)P.nb[BK_FUSED_X] + (size_t)P.nb[BK_FUSED_Y]);
  for (int stage = 1; stage <= 2; ++stage) {
    if (fused) {
      using TX = FusedTile<0, FX_NT, FX_NN>;
      using TY = FusedTile<1, FY_NT, FY_NN>;
      const bool wf = stage == 1;
      HIP_TRY(launch_bs(-1, kb_prep<T>, (unsigned)ng, 1024, s, tab, k, stage));
      const bool ch = k.charvars != 0;
      HIP_TRY(launch_bs(GENO_K_FUSED_X,
                        wf ? (ch ? kb_fused<0, T, true, FUSED_CHAR> : kb_fused<0, T, true, FUSED_PLAIN>)
                           : (ch ? kb_fused<0, T, false, FUSED_CHAR> : kb_fused<0, T, false, FUSED_PLAIN>),
                        (unsigned)P.nb[BK_FUSED_X], TX::BS, s, tab, offs, ng, k));
      HIP_TRY(launch_bs(GENO_K_FUSED_Y,
                        wf ? (ch ? kb_fused<1, T, true, FUSED_CHAR> : kb_fused<1, T, true, FUSED_PLAIN>)
                           : (ch ? kb_fused<1, T, false, FUSED_CHAR> : kb_fused<1, T, false, FUSED_PLAIN>),
                        (unsigned)P.nb[BK_FUSED_Y], TY::BS, s, tab, offs, ng, k));
      HIP_TRY(go_phase<T>(BK_SLOW, P, tab, offs, k, stage, cnt, s));
      HIP_TRY(go_phase<T>(BK_UPDATE, P, tab, offs, k, stage, cnt, s));
    } else {
      for (int phase : {BK_NORMAL_X, BK_FACES_X, BK_NORMAL_Y, BK_FACES_Y, BK_SLOW, BK_UPDATE})
        HIP_TRY(go_phase<T>(phase, P, tab, offs, k, stage, cnt, s));
    }
  }
  return GENO_OK;
}

// Instantiated graphs of one batched step, kept across calls and looked up by
// everything their kernel arguments are made of (device, workspace, plan,
// method constants, counting slots); at most GRAPH_CACHE, the least recently
// used replaced first.
struct GraphEntry {
  std::vector<unsigned char> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;
};
constexpr size_t GRAPH_CACHE = 8;
std::vector<GraphEntry> g_graphs;
std::mutex g_graphs_mu;
unsigned long long g_graph_clock = 0;
long long g_graph_builds = 0;   // graphs instantiated so far (for tests)

template <typename V>
void key_put(std::vector<unsigned char>& key, const V& v) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
  key.insert(key.end(), b, b + sizeof(V));
}

// persistent step: work-groups of the launch (every CU filled to the kernel's
// occupancy, at most one per item)
template <typename T>
int persist_wgs(const BatchPlan& P, bool charvars, int* nwg) {
  int dev = 0, ncu = 0, per = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (charvars)
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kb_persist<T, true>, PB, 0));
  else
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kb_persist<T, false>, PB, 0));
  int widest = 1;
  for (int q = 0; q < PSEG; ++q) widest = std::max(widest, P.segs.start[q + 1] - P.segs.start[q]);
  const long long n = (long long)std::max(1, ncu) * std::max(1, per);
  *nwg = (int)std::max<long long>(1, std::min<long long>(n, widest));
  return GENO_OK;
}

constexpr unsigned int PERSIST_SPIN = 1u << 21;   // polls of one dependency wait (~1 s)

template <typename T>
int persist_step(const BatchPlan& P, const BEntry* tab, const int* offs, char* ws,
                 const geno::KParams& k, int nwg, hipStream_t s) {
  unsigned int* sched = reinterpret_cast<unsigned int*>(ws + P.sched_off);
  unsigned int* done = sched + 4;
  if (k.charvars)
    HIP_TRY(launch_bs(-1, kb_persist<T, true>, (unsigned)nwg, PB, s, tab, offs, P.ngrids, k,
                      P.segs, sched, done, PERSIST_SPIN));
  else
    HIP_TRY(launch_bs(-1, kb_persist<T, false>, (unsigned)nwg, PB, s, tab, offs, P.ngrids, k,
                      P.segs, sched, done, PERSIST_SPIN));
  return GENO_OK;
}

// one step of the batch in the given mode (GENO_BATCH_*), as launches on s
template <typename T>
int batch_one(int mode, const BatchPlan& P, const BEntry* tab, const int* offs, char* ws,
              const geno::KParams& k, const Cnt& cnt, int nwg, hipStream_t s) {
  if (mode == GENO_BATCH_PERSISTENT) return persist_step<T>(P, tab, offs, ws, k, nwg, s);
  return batch_step<T>(P, tab, offs, k, cnt, s);
}

// the cached graph of one step for this key, captured on s if missing
template <typename T>
int graph_of(int mode, const BatchPlan& P, const BEntry* tab, const int* offs, char* ws,
             const geno::KParams& k, const Cnt& cnt, int nwg, hipStream_t s,
             hipGraphExec_t* out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::vector<unsigned char> key;
  key_put(key, mode);
  key_put(key, (int)sizeof(T));
  key_put(key, dev);
  key_put(key, (const void*)ws);
  key_put(key, P.total);
  key_put(key, P.bs);
  key_put(key, P.segs);
  key_put(key, nwg);
  key_put(key, k);
  key_put(key, (const void*)cnt.p);
  key_put(key, cnt.cap);
  key.insert(key.end(), reinterpret_cast<const unsigned char*>(P.offs.data()),
             reinterpret_cast<const unsigned char*>(P.offs.data() + P.offs.size()));
  std::lock_guard<std::mutex> lock(g_graphs_mu);
  for (auto& e : g_graphs)
    if (e.key == key) {
      e.used = ++g_graph_clock;
      *out = e.exec;
      return GENO_OK;
    }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int rc = GENO_OK;
  g_tim_suspend = 1;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = batch_one<T>(mode, P, tab, offs, ws, k, cnt, nwg, s);
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (rc == GENO_OK && e2 != hipSuccess)
      rc = fail(GENO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    if (rc == GENO_OK) {
      e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) rc = fail(GENO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
  } else {
    rc = fail(GENO_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  g_tim_suspend = 0;
  if (rc != GENO_OK) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (g_graphs.size() >= GRAPH_CACHE) {
    auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
    // a replaced graph may still be queued on some stream: wait for the device
    HIP_TRY(hipDeviceSynchronize());
    (void)hipGraphExecDestroy(lru->exec);
    (void)hipGraphDestroy(lru->graph);
    g_graphs.erase(lru);
  }
  GraphEntry ent;
  ent.key = std::move(key);
  ent.graph = graph;
  ent.exec = exec;
  ent.used = ++g_graph_clock;
  g_graphs.push_back(std::move(ent));
  ++g_graph_builds;
  *out = exec;
  return GENO_OK;
}

// nsteps steps of a planned, bound batch whose table is in ws
template <typename T>
int batch_run(const BatchPlan& P, char* ws, const geno_grid* g0, int nsteps, int mode,
              float* step_ms, const Cnt& cnt, hipStream_t s) {
  const BEntry* tab = reinterpret_cast<const BEntry*>(ws + P.tab_off);
  const int* offs = reinterpret_cast<const int*>(ws + P.offs_off);
  const geno::KParams k = kparams(g0);
  if (mode == GENO_BATCH_PERSISTENT)
    HIP_TRY(launch_bs(GENO_K_INIT, kb_init<T, PB>, P.nb[BK_INIT], PB, s, tab, offs, P.ngrids,
                      k.gamma));
  else
    HIP_TRY(go_init<T>(P, tab, offs, k.gamma, s));
  int nwg = 0;
  if (mode == GENO_BATCH_PERSISTENT) {
    int rc0 = persist_wgs<T>(P, k.charvars != 0, &nwg);
    if (rc0) return rc0;
    unsigned int* sched = reinterpret_cast<unsigned int*>(ws + P.sched_off);
    const int n = PSEG * P.ngrids;
    HIP_TRY(launch_bs(-1, kb_sched_clear, (unsigned)std::min(1024, n / PB + 1), PB, s, sched,
                      sched + 4, n));
  }
  std::vector<hipEvent_t> ev;
  if (step_ms && nsteps > 0) {
    ev.assign(nsteps + 1, nullptr);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  }
  int rc = GENO_OK;
  hipGraphExec_t exec = nullptr;
  if (mode != GENO_BATCH_EAGER && nsteps > 0)
    rc = graph_of<T>(mode, P, tab, offs, ws, k, cnt, nwg, s, &exec);
  for (int n = 0; rc == GENO_OK && n < nsteps; ++n) {
    if (!ev.empty() && n == 0) {
      hipError_t e = hipEventRecord(ev[0], s);
      if (e != hipSuccess) rc = fail(GENO_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
    }
    if (exec) {
      hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) rc = fail(GENO_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
    } else if (rc == GENO_OK) {
      rc = batch_one<T>(mode, P, tab, offs, ws, k, cnt, nwg, s);
    }
    if (rc == GENO_OK && !ev.empty()) {
      hipError_t e = hipEventRecord(ev[n + 1], s);
      if (e != hipSuccess) rc = fail(GENO_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
    }
  }
  {
    hipError_t e = hipStreamSynchronize(s);
    if (rc == GENO_OK && e != hipSuccess) rc = fail(GENO_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  if (rc == GENO_OK && mode == GENO_BATCH_PERSISTENT) {
    unsigned int err = 0;
    hipError_t e = hipMemcpy(&err, ws + P.sched_off + 2 * sizeof(unsigned int), sizeof err,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(GENO_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    else if (err)
      rc = fail(GENO_EHIP, "persistent batched step: a dependency wait exceeded its bound");
  }
  if (rc == GENO_OK && !ev.empty())
    for (int n = 0; n < nsteps; ++n) {
      hipError_t e = hipEventElapsedTime(&step_ms[n], ev[n], ev[n + 1]);
      if (e != hipSuccess) {
        rc = fail(GENO_EHIP, "hipEventElapsedTime: %s", hipGetErrorString(e));
        break;
      }
    }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

// plan, bind and upload the batch table (the call waits for the copy)
int prepare_batch(int ngrids, const geno_grid* grids, void* const* W, void* const* dW, void* ws,
                  const geno_tuning* tune, BatchPlan* P, hipStream_t s, bool persistent = false) {
  int rc = check_batch(ngrids, grids);
  if (rc) return rc;
  if (!W || !dW || !ws) return fail(GENO_EINVAL, "null pointer");
  for (int i = 0; i < ngrids; ++i)
    if (!W[i] || !dW[i]) return fail(GENO_EINVAL, "null state pointer of grid %d", i);
  geno_tuning t;
  rc = tuning_of(tune, &t);
  if (rc) return rc;
  // the persistent step runs every phase in its one-wave work-groups
  if (persistent) t.block_normal = t.block_faces = t.block_slow = t.block_update = PB;
  rc = plan_batch(ngrids, grids, t, P);
  if (rc) return rc;
  bind_batch(P, (char*)ws, W, dW, grids);
  HIP_TRY(hipMemcpyAsync((char*)ws + P->tab_off, P->tab.data(), sizeof(BEntry) * ngrids,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync((char*)ws + P->offs_off, P->offs.data(), sizeof(int) * P->offs.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return GENO_OK;
}

int batch_stats(const BatchPlan& P, char* ws, const geno_grid* grids, geno_stats* stats,
                hipStream_t s) {
  stats->guard = 0;
  stats->nonfinite = 0;
  stats->last_dt = 0.0;
  for (int i = 0; i < P.ngrids; ++i) {
    const Layout L = layout_of(&grids[i]);
    Ctrl h;
    HIP_TRY(hipMemcpyAsync(&h, ws + P.goff[i] + L.ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->guard += (long long)h.guard;
    stats->nonfinite += (long long)h.nonfinite;
    if (i == 0) stats->last_dt = h.dt;
  }
  if (stats->nonfinite)
    return fail(GENO_ENONPHYS, "%lld non-physical cells in the batch", stats->nonfinite);
  return GENO_OK;
}

}  // namespace

// operation costs per work class (opcount.hip)
int geno_op_costs_impl(int ndim, double gamma, int nkinds, int nclass, double* costs);

// Device memory of gks_step_noalloc: its whole workspace, one copy of
// GENO_NOALLOC_SCRATCH_BYTES on every device the library runs on, held until
// the process ends. In host code this name is not a device address; the
// address of each device's copy is taken once with hipGetSymbolAddress and
// kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[GENO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
void* scratch_ptr[SCRATCH_MAX_DEVICES] = {};
std::mutex scratch_mu;

// the device address of the current device's scratch (looked up on the
// first call on that device, with that device current)
int scratch_of_current(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(GENO_EINVAL, "device %d beyond the %d devices the scratch table holds", dev,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GENO_EHIP, "no device address for the scratch array");
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return GENO_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int geno_abi_version(void) { return GENO_ABI_VERSION; }

long long geno_batched_graphs_built(void) {
  std::lock_guard<std::mutex> lock(g_graphs_mu);
  return g_graph_builds;
}

int geno_timing_enable(int max_launches) {
  for (int i = 0; i < 2 * g_tim.cap; ++i) (void)hipEventDestroy(g_tim.ev[i]);
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

int geno_count_enable(int on) {
  g_cnt.on = on ? 1 : 0;
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

int geno_work_read(int nkinds, int nclass, long long* counts, void* stream) {
  if (!counts || nkinds < 1 || nclass < 1) return fail(GENO_EINVAL, "null argument");
  for (int i = 0; i < nkinds * nclass; ++i) counts[i] = 0;
  if (!g_cnt.p) return GENO_OK;
  const size_t n = (size_t)GENO_NKERNELS * GENO_NCLASS * g_cnt.cap;
  unsigned long long* h = (unsigned long long*)malloc(n * sizeof *h);
  if (!h) return fail(GENO_EINVAL, "out of host memory");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(h, g_cnt.p, n * sizeof *h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free(h);
    return fail(GENO_EHIP, "work counters: %s", hipGetErrorString(e));
  }
  for (int a = 0; a < nkinds && a < GENO_NKERNELS; ++a)
    for (int c = 0; c < nclass && c < GENO_NCLASS; ++c) {
      unsigned long long t = 0;
      const unsigned long long* p = h + ((size_t)a * GENO_NCLASS + c) * g_cnt.cap;
      for (int i = 0; i < g_cnt.cap; ++i) t += p[i];
      counts[a * nclass + c] = (long long)t;
    }
  free(h);
  return GENO_OK;
}

int geno_op_costs(const geno_grid* g, int nkinds, int nclass, double* costs) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!costs || nkinds < 1 || nclass < 1) return fail(GENO_EINVAL, "null argument");
  return geno_op_costs_impl(g->ndim, g->params.gamma, nkinds, nclass, costs);
}

const char* geno_kernel_name(int kind) {
  return (kind >= 0 && kind < GENO_NKERNELS) ? KNAMES[kind] : "";
}

const char* geno_last_error(void) { return geno_err::g_err; }

int geno_params_default(geno_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  memset(p, 0, sizeof *p);
  p->version = GENO_ABI_VERSION;
  p->variables = GENO_VARS_CONSERVATIVE;
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
  p->eps_ulps = 64.0;
  p->fuse = 1;
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
  if (g->params.precision == GENO_MIXED)
    return reconstruct_t<float>(g, (double*)W, (float*)dW, dir, (float*)face_state, (double*)chi,
                                ws, s);
  return reconstruct_t<double>(g, (double*)W, (double*)dW, dir, (double*)face_state,
                               (double*)chi, ws, s);
}

int gks_flux(const geno_grid* g, const void* face_state, double dt, int dir, void* F, void* Ft,
             void* Wint, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!face_state) return fail(GENO_EINVAL, "null face_state");
  if (!(dt > 0.0)) return fail(GENO_EINVAL, "dt must be positive");
  if (dir != 0 && !(g->ndim == 2 && dir == 1)) return fail(GENO_EINVAL, "bad direction %d", dir);
  hipStream_t s = (hipStream_t)stream;
  if (g->params.precision == GENO_MIXED)
    return flux_t<float>(g, (const float*)face_state, dt, dir, (float*)F, (float*)Ft,
                         (float*)Wint, s);
  return flux_t<double>(g, (const double*)face_state, dt, dir, (double*)F, (double*)Ft,
                        (double*)Wint, s);
}

int gks_step(const geno_grid* g, void* W, void* dW, void* ws, int nsteps, double* dt_out,
             geno_stats* stats, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !dW || !ws) return fail(GENO_EINVAL, "null pointer");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  rc = check_gate(g);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Cnt cnt{nullptr, 0};
  if (g_cnt.on) {
    // measurement mode: (re)allocate the per-block count slots and clear them
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int cap = count_cap(g);
    if (!g_cnt.p || cap > g_cnt.cap || dev != g_cnt.dev) {
      if (g_cnt.p) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(g_cnt.p));
        g_cnt.p = nullptr;
      }
      HIP_TRY(hipMalloc((void**)&g_cnt.p,
                        (size_t)GENO_NKERNELS * GENO_NCLASS * cap * sizeof(unsigned long long)));
      g_cnt.cap = cap;
      g_cnt.dev = dev;
    }
    HIP_TRY(hipMemsetAsync(g_cnt.p, 0,
                           (size_t)GENO_NKERNELS * GENO_NCLASS * g_cnt.cap *
                               sizeof(unsigned long long),
                           s));
    cnt = Cnt{g_cnt.p, g_cnt.cap};
  }
  Ctrl* ctrl = nullptr;
  if (g->params.precision == GENO_MIXED)
    rc = step_t<float>(g, (double*)W, (float*)dW, ws, nsteps, dt_out, cnt, s, &ctrl);
  else
    rc = step_t<double>(g, (double*)W, (double*)dW, ws, nsteps, dt_out, cnt, s, &ctrl);
  if (rc) return rc;
  if (stats) {
    Ctrl h;
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

int gks_step_noalloc(const geno_grid* g, void* W, void* dW, int nsteps, double* dt_out,
                     geno_stats* stats, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !dW) return fail(GENO_EINVAL, "null pointer");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  rc = check_gate(g);
  if (rc) return rc;
  const size_t need = layout_of(g).total;
  if (need > (size_t)GENO_NOALLOC_SCRATCH_BYTES)
    return fail(GENO_EINVAL,
                "grid needs %zu bytes of workspace, above the %zu bytes of the allocation-free "
                "scratch (use gks_step with a workspace)",
                need, (size_t)GENO_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  rc = scratch_of_current(&ws);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  // no work counting here (its per-block slots are allocated on first use);
  // every workspace entry the step reads is written by it first
  const Cnt cnt{nullptr, 0};
  Ctrl* ctrl = nullptr;
  if (g->params.precision == GENO_MIXED)
    rc = step_t<float>(g, (double*)W, (float*)dW, ws, nsteps, dt_out, cnt, s, &ctrl);
  else
    rc = step_t<double>(g, (double*)W, (double*)dW, ws, nsteps, dt_out, cnt, s, &ctrl);
  if (rc) return rc;
  if (stats) {
    Ctrl h;
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

int geno_linearity(const geno_grid* g, void* W, void* dW, int dir, double* chi3, double teno_ct,
                   void* ws, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !dW || !chi3 || !ws) return fail(GENO_EINVAL, "null pointer");
  if (dir != 0 && !(g->ndim == 2 && dir == 1)) return fail(GENO_EINVAL, "bad direction %d", dir);
  if (!(teno_ct > 0.0 && teno_ct < 1.0)) return fail(GENO_EINVAL, "teno_ct must be in (0, 1)");
  hipStream_t s = (hipStream_t)stream;
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  const int nv = g->ndim == 2 ? 4 : 3;
  const size_t n1 = dir == 0 ? g->nx + 1 : g->nx + 2;
  const size_t n0 = g->ndim == 1 ? 1 : (dir == 0 ? g->ny + 2 : g->ny + 1);
  const unsigned nb = nblocks((size_t)nv * n0 * n1);
  if (g->params.precision == GENO_MIXED) {
    const Bufs<float> B = bufs_of<float>((char*)ws, L, g->ndim);
    rc = launch_init<float>(g, geo, k.gamma, (double*)W, (float*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_linearity<0, float>, nb, s, geo, k, g->ndim, (const double*)W,
                     (const float*)dW, chi3, teno_ct));
    else
      HIP_TRY(launch(-1, k_linearity<1, float>, nb, s, geo, k, g->ndim, (const double*)W,
                     (const float*)dW, chi3, teno_ct));
  } else {
    const Bufs<double> B = bufs_of<double>((char*)ws, L, g->ndim);
    rc = launch_init<double>(g, geo, k.gamma, (double*)W, (double*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_linearity<0, double>, nb, s, geo, k, g->ndim, (const double*)W,
                     (const double*)dW, chi3, teno_ct));
    else
      HIP_TRY(launch(-1, k_linearity<1, double>, nb, s, geo, k, g->ndim, (const double*)W,
                     (const double*)dW, chi3, teno_ct));
  }
  return GENO_OK;
}

int geno_conserved_totals(const geno_grid* g, const void* W, double* totals, void* stream) {
  const int rc = check_grid(g);
  if (rc) return rc;
  if (!W || !totals) return fail(GENO_EINVAL, "null pointer");
  const int nv = g->ndim == 2 ? 4 : 3;
  const double area = g->ndim == 2 ? g->dx * g->dy : g->dx;
  HIP_TRY(launch_bs(-1, k_totals, (unsigned)nv, 1024u, (hipStream_t)stream, geo_of(g),
                    (const double*)W, area, totals));
  return GENO_OK;
}

int geno_tuning_default(geno_tuning* t) {
  if (!t) return fail(GENO_EINVAL, "null tuning");
  return tuning_of(nullptr, t);
}

size_t gks_batched_workspace_bytes(int ngrids, const geno_grid* grids) {
  if (check_batch(ngrids, grids)) return 0;
  geno_tuning t;
  tuning_of(nullptr, &t);
  BatchPlan P;
  if (plan_batch(ngrids, grids, t, &P)) return 0;
  return P.total;
}

int gks_step_batched(int ngrids, const geno_grid* grids, void* const* W, void* const* dW, void* ws,
                     int nsteps, const geno_tuning* tune, int use_graph, float* step_ms,
                     geno_stats* stats, void* stream) {
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  if (use_graph != GENO_BATCH_EAGER && use_graph != GENO_BATCH_GRAPH &&
      use_graph != GENO_BATCH_PERSISTENT)
    return fail(GENO_EINVAL, "unknown batched mode %d", use_graph);
  // The persistent step is switched off: its launches did not finish on the
  // device (before and after the one-wave work-groups and relaxed polling),
  // and the cause is not established.
  if (use_graph == GENO_BATCH_PERSISTENT)
    return fail(GENO_EINVAL, "the persistent batched mode is not available in this build");
  hipStream_t s = (hipStream_t)stream;
  if (use_graph && s == nullptr)
    return fail(GENO_EINVAL, "graph mode needs a stream other than the NULL stream");
  BatchPlan P;
  int rc = prepare_batch(ngrids, grids, W, dW, ws, tune, &P, s,
                         use_graph == GENO_BATCH_PERSISTENT);
  if (rc) return rc;
  Cnt cnt{nullptr, 0};
  if (g_cnt.on && use_graph != GENO_BATCH_PERSISTENT) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cap = 1;
    for (int k = 0; k < BK_N; ++k) cap = std::max(cap, P.nb[k]);
    if (!g_cnt.p || cap > g_cnt.cap || dev != g_cnt.dev) {
      if (g_cnt.p) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(g_cnt.p));
        g_cnt.p = nullptr;
      }
      HIP_TRY(hipMalloc((void**)&g_cnt.p,
                        (size_t)GENO_NKERNELS * GENO_NCLASS * cap * sizeof(unsigned long long)));
      g_cnt.cap = cap;
      g_cnt.dev = dev;
    }
    HIP_TRY(hipMemsetAsync(g_cnt.p, 0,
                           (size_t)GENO_NKERNELS * GENO_NCLASS * g_cnt.cap *
                               sizeof(unsigned long long),
                           s));
    cnt = Cnt{g_cnt.p, g_cnt.cap};
  }
  if (grids[0].params.precision == GENO_MIXED)
    rc = batch_run<float>(P, (char*)ws, &grids[0], nsteps, use_graph, step_ms, cnt, s);
  else
    rc = batch_run<double>(P, (char*)ws, &grids[0], nsteps, use_graph, step_ms, cnt, s);
  if (rc) return rc;
  if (stats) return batch_stats(P, (char*)ws, grids, stats, s);
  return GENO_OK;
}

int geno_autotune_batched(int ngrids, const geno_grid* grids, void* const* W, void* const* dW,
                          void* ws, int trial_steps, geno_tuning* out, void* stream) {
  if (!out) return fail(GENO_EINVAL, "null tuning");
  if (trial_steps < 1) return fail(GENO_EINVAL, "trial_steps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  geno_tuning best;
  tuning_of(nullptr, &best);
  const bool mixed = check_batch(ngrids, grids) == GENO_OK && grids[0].params.precision == GENO_MIXED;
  const Cnt none{nullptr, 0};
  // one run of a candidate: summed kernel time of the given kinds
  auto trial = [&](const geno_tuning& t, std::initializer_list<int> kinds, double* ms) -> int {
    BatchPlan P;
    int rc = prepare_batch(ngrids, grids, W, dW, ws, &t, &P, s);
    if (rc) return rc;
    rc = geno_timing_enable(12 * trial_steps + 4);
    if (rc) return rc;
    rc = mixed ? batch_run<float>(P, (char*)ws, &grids[0], trial_steps, 0, nullptr, none, s)
               : batch_run<double>(P, (char*)ws, &grids[0], trial_steps, 0, nullptr, none, s);
    double tot[GENO_NKERNELS];
    long long nl[GENO_NKERNELS];
    if (rc == GENO_OK) rc = geno_timing_read(GENO_NKERNELS, tot, nl);
    geno_timing_enable(0);
    if (rc) return rc;
    *ms = 0.0;
    for (int k : kinds) *ms += tot[k];
    return GENO_OK;
  };
  double ms = 0.0;
  int rc = trial(best, {GENO_K_INIT}, &ms);   // warm-up
  if (rc) return rc;
  const int sizes[3] = {128, 256, 512};
  struct Field {
    int geno_tuning::*f;
    std::initializer_list<int> kinds;
  };
  const Field fields[3] = {{&geno_tuning::block_normal, {GENO_K_NORMAL_X, GENO_K_NORMAL_Y}},
                           {&geno_tuning::block_faces, {GENO_K_FACES_X, GENO_K_FACES_Y}},
                           {&geno_tuning::block_update,
                            {GENO_K_UPDATE_1, GENO_K_UPDATE_2, GENO_K_INIT}}};
  for (const Field& fd : fields) {
    double bms = 1e300;
    int bsz = best.*fd.f;
    for (int b : sizes) {
      geno_tuning t = best;
      t.*fd.f = b;
      rc = trial(t, fd.kinds, &ms);
      if (rc) return rc;
      if (ms < bms) {
        bms = ms;
        bsz = b;
      }
    }
    best.*fd.f = bsz;
  }
  double bms = 1e300;
  geno_tuning bslow = best;
  for (int b : sizes)
    for (int fpb : {512, 2048, 8192}) {
      geno_tuning t = best;
      t.block_slow = b;
      t.slow_faces_per_block = fpb;
      rc = trial(t, {GENO_K_SLOW}, &ms);
      if (rc) return rc;
      if (ms < bms) {
        bms = ms;
        bslow = t;
      }
    }
  *out = bslow;
  return GENO_OK;
}

int geno_mlp_load(const float* params, void* stream) {
  if (!params) return fail(GENO_EINVAL, "null params");
  hipStream_t s = (hipStream_t)stream;
  std::vector<float> p(mlp::NPARAM);
  HIP_TRY(hipMemcpyAsync(p.data(), params, sizeof(float) * mlp::NPARAM, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (float x : p)
    if (!std::isfinite(x)) return fail(GENO_EINVAL, "non-finite network parameter");
  // B fragments of both layers in lane order (see g_mlp_frag)
  std::vector<unsigned short> frag(16 * 64 * 8, 0);
  for (int layer = 0; layer < 2; ++layer)
    for (int kb = 0; kb < 2; ++kb)
      for (int nt = 0; nt < 4; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < 8; ++e) {
            const int kk = kb * 32 + 8 * (lane / 16) + e, n = nt * 16 + lane % 16;
            float w = 0.0f;
            if (layer == 0 && kk < mlp::NIN) w = p[mlp::OW1 + n * mlp::NIN + kk];
            if (layer == 1) w = p[mlp::OW2 + n * mlp::NH + kk];
            frag[(((size_t)(layer * 8 + kb * 4 + nt) * 64) + lane) * 8 + e] = f2bf(w);
          }
  std::vector<float> vec(3 * mlp::NH + 1);
  for (int q = 0; q < mlp::NH; ++q) {
    vec[q] = p[mlp::OB1 + q];
    vec[mlp::NH + q] = p[mlp::OB2 + q];
    vec[2 * mlp::NH + q] = p[mlp::OW3 + q];
  }
  vec[3 * mlp::NH] = p[mlp::OB3];
  HIP_TRY(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_mlp_frag), frag.data(),
                                 sizeof(unsigned short) * frag.size(), 0, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_mlp_vec), vec.data(), sizeof(float) * vec.size(), 0,
                                 hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64) g_mlp_loaded[dev] = true;
  return GENO_OK;
}

int geno_mlp_infer(const float* X, int n, float* prob, void* stream) {
  if (!X || !prob) return fail(GENO_EINVAL, "null pointer");
  if (n < 0) return fail(GENO_EINVAL, "n must be >= 0");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64 || !g_mlp_loaded[dev]) return fail(GENO_EINVAL, "no network loaded");
  if (n == 0) return GENO_OK;
  const unsigned nb = (unsigned)(((size_t)n + 63) / 64);
  HIP_TRY(launch(-1, k_mlp_infer, nb, (hipStream_t)stream, X, n, prob));
  return GENO_OK;
}

int geno_gate_prob(const geno_grid* g, void* W, void* dW, int dir, float* prob, void* ws,
                   void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (g->ndim != 2) return fail(GENO_EINVAL, "the gate is 2-D only");
  if (!W || !dW || !prob || !ws) return fail(GENO_EINVAL, "null pointer");
  if (dir != 0 && dir != 1) return fail(GENO_EINVAL, "bad direction %d", dir);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64 || !g_mlp_loaded[dev]) return fail(GENO_EINVAL, "no network loaded");
  hipStream_t s = (hipStream_t)stream;
  const Geo geo = geo_of(g);
  const size_t nc = (size_t)g->nx * g->ny;
  const Layout L = layout_of(g);
  if (g->params.precision == GENO_MIXED) {
    const Bufs<float> B = bufs_of<float>((char*)ws, L, 2);
    rc = launch_init<float>(g, geo, g->params.gamma, (double*)W, (float*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_gate<0, float, 1>, gate_blocks(nc), s, geo, (const double*)W,
                     (const float*)dW, 0.0f, (unsigned char*)nullptr, prob));
    else
      HIP_TRY(launch(-1, k_gate<1, float, 1>, gate_blocks(nc), s, geo, (const double*)W,
                     (const float*)dW, 0.0f, (unsigned char*)nullptr, prob));
  } else {
    const Bufs<double> B = bufs_of<double>((char*)ws, L, 2);
    rc = launch_init<double>(g, geo, g->params.gamma, (double*)W, (double*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_gate<0, double, 1>, gate_blocks(nc), s, geo, (const double*)W,
                     (const double*)dW, 0.0f, (unsigned char*)nullptr, prob));
    else
      HIP_TRY(launch(-1, k_gate<1, double, 1>, gate_blocks(nc), s, geo, (const double*)W,
                     (const double*)dW, 0.0f, (unsigned char*)nullptr, prob));
  }
  return GENO_OK;
}

int geno_harvest(const geno_grid* g, void* W, void* dW, int dir, float* X, float* y, void* ws,
                 void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (g->ndim != 2) return fail(GENO_EINVAL, "harvest is 2-D only");
  if (!W || !dW || !X || !ws) return fail(GENO_EINVAL, "null pointer");
  if (dir != 0 && dir != 1) return fail(GENO_EINVAL, "bad direction %d", dir);
  hipStream_t s = (hipStream_t)stream;
  const Geo geo = geo_of(g);
  const geno::KParams k = kparams(g);
  const Layout L = layout_of(g);
  const unsigned nb = nblocks((size_t)g->nx * g->ny);
  if (g->params.precision == GENO_MIXED) {
    const Bufs<float> B = bufs_of<float>((char*)ws, L, 2);
    rc = launch_init<float>(g, geo, k.gamma, (double*)W, (float*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_harvest<0, float>, nb, s, geo, k, (const double*)W, (const float*)dW, X, y));
    else
      HIP_TRY(launch(-1, k_harvest<1, float>, nb, s, geo, k, (const double*)W, (const float*)dW, X, y));
  } else {
    const Bufs<double> B = bufs_of<double>((char*)ws, L, 2);
    rc = launch_init<double>(g, geo, k.gamma, (double*)W, (double*)dW, B, s);
    if (rc) return rc;
    if (dir == 0)
      HIP_TRY(launch(-1, k_harvest<0, double>, nb, s, geo, k, (const double*)W, (const double*)dW, X, y));
    else
      HIP_TRY(launch(-1, k_harvest<1, double>, nb, s, geo, k, (const double*)W, (const double*)dW, X, y));
  }
  return GENO_OK;
}

}  // extern "C"
