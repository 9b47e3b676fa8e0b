// HIP kernels and C ABI of the sixth-order non-compact scheme in 1-D
// (declarations and conventions: geno6.h).
//
// One Runge-Kutta stage is one launch. A work-group of 256 lanes owns 255
// consecutive cells: it stages the averages of its cells and three halo
// cells on each side in LDS (boundary images formed on the fly), each lane
// then reconstructs both sides of one of the 256 faces of the tile (GENO on
// the six-cell stencil for the three variables), guards them and evaluates
// HLLC, the fluxes go back to LDS, and each lane finishes one cell: the flux
// difference and the stage combination of the classical Runge-Kutta method.
// The last stage also folds the work-group maxima of |u| + a of the new
// state into 1024 slots (atomic max), from which a one-work-group launch
// forms the next step's dt on the device.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <tuple>
#include <utility>

#include "geno6.h"
#include "geno6_device.hpp"

namespace geno_err {
int fail(int code, const char* fmt, ...);
}

namespace {

using geno_err::fail;
using geno6::KP6;

constexpr int TB = 256;        // lanes per work-group
constexpr int TC = TB - 1;     // cells per work-group (TB faces)
constexpr int HALO = 3;        // cells needed on each side of a face stencil
constexpr int TL = TC + 2 * HALO;   // staged cells per variable
constexpr int NSLOT = 1024;         // slots of the wave-speed maxima (atomic max, bits of
                                    // non-negative doubles order as unsigned integers)

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(GENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Ctrl6 {
  double dt;
  unsigned long long guard;
  unsigned long long nonfinite;
};

struct Geo6 {
  int n, pitch, bc_lo, bc_hi;
  double dx, inv_dx;
  double ghost[2][3][3];   // GENO6_BC_FIXED states: [end][cell k][field]
};

// ---------------------------------------------------------------------------
// Timing hooks (events bound to the kernel's own dispatch)
// ---------------------------------------------------------------------------
struct Timing6 {
  hipEvent_t* ev = nullptr;
  int* kind = nullptr;
  int cap = 0, used = 0;
};
Timing6 g_tim6;

template <typename... KArgs, typename... Args>
hipError_t launch6_bs(int kind, void (*kern)(KArgs...), unsigned grid, unsigned bs, hipStream_t s,
                      Args&&... args) {
  std::tuple<KArgs...> tup = validateArgsCountType(kern, std::tuple<Args...>{args...});
  void* argv[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
  pArgs<0>(tup, argv);
  if (kind >= 0 && g_tim6.used < g_tim6.cap) {
    const int u = g_tim6.used++;
    g_tim6.kind[u] = kind;
    return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(bs), argv, 0, s,
                              g_tim6.ev[2 * u], g_tim6.ev[2 * u + 1], 0);
  }
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(bs), argv, 0, s);
}

template <typename... KArgs, typename... Args>
hipError_t launch6(int kind, void (*kern)(KArgs...), unsigned grid, hipStream_t s, Args&&... args) {
  return launch6_bs(kind, kern, grid, TB, s, std::forward<Args>(args)...);
}

// ---------------------------------------------------------------------------
// Boundary images: value of field f at cell i in [-3, n + 3)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_at(const Geo6& g, const double* __restrict__ U, int f, int i) {
  int src = i;
  double sign = 1.0;
  if (i < 0 && g.bc_lo == GENO6_BC_FIXED) return g.ghost[0][-i - 1][f];
  if (i >= g.n && g.bc_hi == GENO6_BC_FIXED) return g.ghost[1][i - g.n][f];
  if (i < 0) {
    src = g.bc_lo == GENO_BC_PERIODIC ? i + g.n : (g.bc_lo == GENO_BC_REFLECTING ? -i - 1 : 0);
    if (g.bc_lo == GENO_BC_REFLECTING && f == 1) sign = -1.0;
  } else if (i >= g.n) {
    src = g.bc_hi == GENO_BC_PERIODIC ? i - g.n
                                      : (g.bc_hi == GENO_BC_REFLECTING ? 2 * g.n - 1 - i : g.n - 1);
    if (g.bc_hi == GENO_BC_REFLECTING && f == 1) sign = -1.0;
  }
  return sign * U[(size_t)f * g.pitch + src];
}

__device__ __forceinline__ double wave_speed(double gamma, double r, double m, double E) {
  const double ir = 1.0 / r, u = m * ir;
  const double p = (gamma - 1.0) * (E - 0.5 * m * u);
  return fabs(u) + sqrt(gamma * p * ir);
}

__device__ __forceinline__ bool physical(double r, double m, double E) {
  return isfinite(r) && isfinite(m) && isfinite(E) && r > 0.0 && r * E - 0.5 * m * m > 0.0;
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < TB / 64; ++w) m = fmax(m, red[w]);
  return m;
}

__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned s = 0;
#pragma unroll
  for (int w = 0; w < TB / 64; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Start of geno6_step: counters and maxima slots cleared (one work-group).
__global__ void __launch_bounds__(TB) k6_clear(unsigned long long* __restrict__ slots, Ctrl6* ctrl) {
  if (slots)
    for (int q = threadIdx.x; q < NSLOT; q += TB) slots[q] = 0ull;
  if (threadIdx.x == 0) {
    ctrl->guard = 0;
    ctrl->nonfinite = 0;
  }
}

// Work-group maximum s >= 0 into its slot (work-groups share a slot round
// robin).
__device__ __forceinline__ void slot_max(unsigned long long* slots, double s) {
  if (threadIdx.x == 0)
    atomicMax(&slots[blockIdx.x & (NSLOT - 1)], (unsigned long long)__double_as_longlong(s));
}

// Maxima of |u| + a of the initial state (same tiling as the stage kernel).
__global__ void __launch_bounds__(TB) k6_init(Geo6 g, double gamma, const double* __restrict__ U,
                                               unsigned long long* __restrict__ slots) {
  __shared__ double red[TB / 64];
  const int c = (int)blockIdx.x * TC + (int)threadIdx.x;
  double s = 0.0;
  if (threadIdx.x < TC && c < g.n)
    s = wave_speed(gamma, U[c], U[(size_t)g.pitch + c], U[2 * (size_t)g.pitch + c]);
  s = block_max(s, red);
  slot_max(slots, s);
}

// dt of a step: cfl dx / max of the slots (or dt_fixed); the slots are
// cleared for the maxima of the step's last stage. One work-group of TB
// lanes, NSLOT / TB slots each.
__global__ void __launch_bounds__(TB) k6_dt(unsigned long long* __restrict__ slots, double dx,
                                             double cfl, double dt_fixed, Ctrl6* ctrl,
                                             double* dt_out, int step) {
  __shared__ double red[TB / 64];
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < NSLOT / TB; ++q) {
    unsigned long long& sl = slots[q * TB + threadIdx.x];
    m = fmax(m, __longlong_as_double((long long)sl));
    sl = 0ull;
  }
  m = block_max(m, red);
  if (threadIdx.x == 0) {
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl * dx / m;
    ctrl->dt = dt;
    if (dt_out) dt_out[step] = dt;
  }
}

// MODE 0..3: Runge-Kutta stages; MODE 4: right-hand side only (Yout = L).
//   0: acc = Y + dt/6 L, Yout = Y + dt/2 L    (Y = U)
//   1: acc += dt/3 L,    Yout = U0 + dt/2 L
//   2: acc += dt/3 L,    Yout = U0 + dt L
//   3: Yout = acc + dt/6 L (= the new U), maxima of |u| + a, non-physical
//      cells counted
template <int MODE, bool CHAR>
__global__ void __launch_bounds__(TB) k6_stage(Geo6 g, KP6 k, const double* __restrict__ Y,
                                                const double* __restrict__ U0,
                                                double* __restrict__ acc, double* __restrict__ Yout,
                                                Ctrl6* ctrl, unsigned long long* __restrict__ slots) {
  __shared__ double su[3][TL];
  __shared__ double sf[3][TB];
  __shared__ double redd[TB / 64];
  __shared__ unsigned redu[TB / 64];
  const int t = (int)threadIdx.x;
  const int c0 = (int)blockIdx.x * TC;
  // stage cells c0-3 .. c0+TC+2 (those past n + 2 are never read)
  for (int q = t; q < TL; q += TB) {
    const int i = c0 - HALO + q;
    if (i <= g.n + 2) {
#pragma unroll
      for (int f = 0; f < 3; ++f) su[f][q] = cell_at(g, Y, f, i);
    }
  }
  __syncthreads();
  // face s = c0 + t between cells s-1 and s: stencil cells s-3..s+2 = LDS t..t+5
  unsigned guard = 0;
  if (c0 + t <= g.n) {
    const auto get = [&](int f, int m) { return su[f][t + m]; };
    double WL[3], WR[3], F[3];
    guard = (unsigned)geno6::face6<double, CHAR>(get, k, WL, WR, F, nullptr);
#pragma unroll
    for (int f = 0; f < 3; ++f) sf[f][t] = F[f];
  }
  __syncthreads();
  const int c = c0 + t;
  const bool own = t < TC && c < g.n;
  double L[3] = {0.0, 0.0, 0.0};
  if (own) {
#pragma unroll
    for (int f = 0; f < 3; ++f) L[f] = -(sf[f][t + 1] - sf[f][t]) * g.inv_dx;
  }
  if (MODE == 4) {
    if (own) {
#pragma unroll
      for (int f = 0; f < 3; ++f) Yout[(size_t)f * g.pitch + c] = L[f];
    }
    return;
  }
  const double dt = ctrl->dt;
  double wnew[3] = {0.0, 0.0, 0.0};
  if (own) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const size_t o = (size_t)f * g.pitch + c;
      if (MODE == 0) {
        const double y = su[f][t + HALO];
        acc[o] = y + (dt * (1.0 / 6.0)) * L[f];
        Yout[o] = y + (0.5 * dt) * L[f];
      } else if (MODE == 1) {
        acc[o] = acc[o] + (dt * (1.0 / 3.0)) * L[f];
        Yout[o] = U0[o] + (0.5 * dt) * L[f];
      } else if (MODE == 2) {
        acc[o] = acc[o] + (dt * (1.0 / 3.0)) * L[f];
        Yout[o] = U0[o] + dt * L[f];
      } else {
        wnew[f] = acc[o] + (dt * (1.0 / 6.0)) * L[f];
        Yout[o] = wnew[f];
      }
    }
  }
  const unsigned gsum = block_sum(guard, redu);
  if (t == 0 && gsum) atomicAdd(&ctrl->guard, (unsigned long long)gsum);
  if (MODE == 3) {
    double s = 0.0;
    unsigned bad = 0;
    if (own) {
      if (physical(wnew[0], wnew[1], wnew[2])) s = wave_speed(k.gamma, wnew[0], wnew[1], wnew[2]);
      else bad = 1;
    }
    s = block_max(s, redd);
    const unsigned nbad = block_sum(bad, redu);
    slot_max(slots, s);
    if (t == 0 && nbad) atomicAdd(&ctrl->nonfinite, (unsigned long long)nbad);
  }
}

// Reconstruction and flux of every face (output form of geno6_faces).
template <bool CHAR>
__global__ void __launch_bounds__(TB) k6_faces(Geo6 g, KP6 k, const double* __restrict__ U,
                                                double* __restrict__ UL, double* __restrict__ UR,
                                                double* __restrict__ F, double* __restrict__ chi) {
  const int s = (int)blockIdx.x * TB + (int)threadIdx.x;
  if (s > g.n) return;
  double u[3][6];
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int m = 0; m < 6; ++m) u[f][m] = cell_at(g, U, f, s - HALO + m);
  const auto get = [&](int f, int m) { return u[f][m]; };
  double WL[3], WR[3], FF[3], X[6];
  geno6::face6<double, CHAR>(get, k, WL, WR, FF, X);
  const size_t nf = (size_t)g.n + 1;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (UL) UL[f * nf + s] = WL[f];
    if (UR) UR[f * nf + s] = WR[f];
    if (F) F[f * nf + s] = FF[f];
    if (chi) {
      chi[f * nf + s] = X[f];
      chi[(3 + f) * nf + s] = X[3 + f];
    }
  }
}

// ---------------------------------------------------------------------------
// Small grids (the paper's 1-D problems have 200 to 1800 cells): one
// work-group of SB lanes per grid runs all steps and stages of the call in
// one launch. Each stage sweeps the grid in passes of SB - 1 cells (stage
// the pass's cells and halo in LDS, reconstruct and flux its SB faces, flux
// difference and stage combination of its cells); a barrier between stages
// makes the stage's writes visible to the work-group (its waves share one
// CU's caches). The arithmetic is the stage kernel's, in the same order, so
// each grid's result is the one geno6_step gives.
// ---------------------------------------------------------------------------
// Lanes per work-group (one grid): 1024 with conservative variables; 512
// with characteristic ones, whose face code needs more than the 128 VGPRs a
// 1024-lane work-group leaves each lane.
template <bool CHAR>
struct SmallShape {
  static constexpr int SB = CHAR ? 512 : 1024;
  static constexpr int SC = SB - 1;               // cells per pass
  static constexpr int SL = SC + 2 * HALO;        // staged cells per variable
};

template <int SB>
__device__ __forceinline__ double block_max_s(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < SB / 64; ++w) m = fmax(m, red[w]);
  return m;
}

template <int SB>
__device__ __forceinline__ unsigned block_sum_s(unsigned v, unsigned* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned s = 0;
#pragma unroll
  for (int w = 0; w < SB / 64; ++w) s += red[w];
  return s;
}

template <bool CHAR>
__global__ void __launch_bounds__(SmallShape<CHAR>::SB) k6_small(Geo6 g, KP6 k,
                                                                  double* __restrict__ Ubase,
                                                                  double* __restrict__ wsbase,
                                                                  size_t stride, int nsteps,
                                                                  double* __restrict__ dt_out,
                                                                  Ctrl6* ctrl) {
  constexpr int SB = SmallShape<CHAR>::SB, SC = SmallShape<CHAR>::SC, SL = SmallShape<CHAR>::SL;
  __shared__ double su[3][SL];
  __shared__ double sf[3][SB];
  __shared__ double redd[SB / 64];
  __shared__ unsigned redu[SB / 64];
  const int t = (int)threadIdx.x;
  const size_t gi = blockIdx.x;
  double* U = Ubase + gi * stride;
  double* acc = wsbase + gi * 3 * stride;
  double* ya = acc + stride;
  double* yb = ya + stride;
  // wave-speed maximum of the initial state
  double smax = 0.0;
  for (int c = t; c < g.n; c += SB)
    smax = fmax(smax, wave_speed(k.gamma, U[c], U[(size_t)g.pitch + c], U[2 * (size_t)g.pitch + c]));
  smax = block_max_s<SB>(smax, redd);
  unsigned guard = 0, bad = 0;
  for (int step = 0; step < nsteps; ++step) {
    const double dt = k.dt_fixed > 0.0 ? k.dt_fixed : k.cfl * g.dx / smax;
    if (t == 0 && dt_out) dt_out[gi * nsteps + step] = dt;
    double snew = 0.0;
#pragma unroll 1
    for (int stage = 0; stage < 4; ++stage) {
      const double* Y = stage == 0 ? U : (stage == 2 ? yb : ya);
      double* Yout = stage == 0 ? ya : (stage == 1 ? yb : (stage == 2 ? ya : U));
      for (int c0 = 0; c0 < g.n; c0 += SC) {
        for (int q = t; q < SL; q += SB) {
          const int i = c0 - HALO + q;
          if (i <= g.n + 2) {
#pragma unroll
            for (int f = 0; f < 3; ++f) su[f][q] = cell_at(g, Y, f, i);
          }
        }
        __syncthreads();
        if (c0 + t <= g.n) {
          const auto get = [&](int f, int m) { return su[f][t + m]; };
          double WL[3], WR[3], F[3];
          guard += (unsigned)geno6::face6<double, CHAR>(get, k, WL, WR, F, nullptr);
#pragma unroll
          for (int f = 0; f < 3; ++f) sf[f][t] = F[f];
        }
        __syncthreads();
        const int c = c0 + t;
        if (t < SC && c < g.n) {
          double wnew[3];
#pragma unroll
          for (int f = 0; f < 3; ++f) {
            const double L = -(sf[f][t + 1] - sf[f][t]) * g.inv_dx;
            const size_t o = (size_t)f * g.pitch + c;
            if (stage == 0) {
              const double y = su[f][t + HALO];
              acc[o] = y + (dt * (1.0 / 6.0)) * L;
              Yout[o] = y + (0.5 * dt) * L;
            } else if (stage == 1) {
              acc[o] = acc[o] + (dt * (1.0 / 3.0)) * L;
              Yout[o] = U[o] + (0.5 * dt) * L;
            } else if (stage == 2) {
              acc[o] = acc[o] + (dt * (1.0 / 3.0)) * L;
              Yout[o] = U[o] + dt * L;
            } else {
              wnew[f] = acc[o] + (dt * (1.0 / 6.0)) * L;
              Yout[o] = wnew[f];
            }
          }
          if (stage == 3) {
            if (physical(wnew[0], wnew[1], wnew[2]))
              snew = fmax(snew, wave_speed(k.gamma, wnew[0], wnew[1], wnew[2]));
            else
              ++bad;
          }
        }
        __syncthreads();   // the pass's LDS is reused; its global writes are read next stage
      }
    }
    smax = block_max_s<SB>(snew, redd);
  }
  const unsigned gsum = block_sum_s<SB>(guard, redu);
  const unsigned nbad = block_sum_s<SB>(bad, redu);
  if (t == 0) {
    if (gsum) atomicAdd(&ctrl->guard, (unsigned long long)gsum);
    if (nbad) atomicAdd(&ctrl->nonfinite, (unsigned long long)nbad);
    if (gi == 0 && nsteps > 0) ctrl->dt = k.dt_fixed > 0.0 ? k.dt_fixed : k.cfl * g.dx / smax;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int check_params6(const geno6_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  if (p->version != GENO6_ABI_VERSION)
    return fail(GENO_EVERSION, "params version %d != %d", p->version, GENO6_ABI_VERSION);
  if (!(p->gamma > 1.0) || !(p->eps > 0.0) || !(p->C > 0.0) || !(p->cfl > 0.0))
    return fail(GENO_EINVAL, "gamma > 1, eps > 0, C > 0 and cfl > 0 are required");
  for (int i = 0; i < 4; ++i)
    if (!(p->d[i] > 0.0)) return fail(GENO_EINVAL, "linear weights d must be positive");
  if (!(p->dt_fixed >= 0.0)) return fail(GENO_EINVAL, "dt_fixed must be >= 0");
  if (p->variables != GENO6_VARS_CONSERVATIVE && p->variables != GENO6_VARS_CHARACTERISTIC)
    return fail(GENO_EINVAL, "bad variables code %d", p->variables);
  for (int i = 0; i < 2; ++i)
    if (p->bc[i] != GENO_BC_PERIODIC && p->bc[i] != GENO_BC_TRANSMISSIVE &&
        p->bc[i] != GENO_BC_REFLECTING && p->bc[i] != GENO6_BC_FIXED)
      return fail(GENO_EINVAL, "bad boundary code %d", p->bc[i]);
  if ((p->bc[0] == GENO_BC_PERIODIC) != (p->bc[1] == GENO_BC_PERIODIC))
    return fail(GENO_EINVAL, "periodic boundaries must be set on both ends");
  return GENO_OK;
}

int check_grid6(const geno6_grid* g) {
  if (!g) return fail(GENO_EINVAL, "null grid");
  const int rc = check_params6(&g->params);
  if (rc) return rc;
  if (g->n < 3) return fail(GENO_EINVAL, "at least 3 cells are required");
  if (g->pitch != ((g->n + 63) / 64) * 64) return fail(GENO_EINVAL, "pitch inconsistent (use geno6_grid_init)");
  if (!(g->dx > 0.0)) return fail(GENO_EINVAL, "bad cell size");
  return GENO_OK;
}

Geo6 geo6(const geno6_grid* g) {
  Geo6 o;
  o.n = g->n;
  o.pitch = g->pitch;
  o.bc_lo = g->params.bc[0];
  o.bc_hi = g->params.bc[1];
  o.dx = g->dx;
  o.inv_dx = 1.0 / g->dx;
  for (int e = 0; e < 2; ++e)
    for (int c = 0; c < 3; ++c)
      for (int f = 0; f < 3; ++f) o.ghost[e][c][f] = g->params.ghost[e][c][f];
  return o;
}

KP6 kp6(const geno6_params& p) {
  KP6 k;
  k.gamma = p.gamma;
  k.C = p.C;
  k.inv_tanhC = 1.0 / std::tanh(p.C);
  k.t2_cut = 2.0 * (1.0 - 19.8 / p.C) / (19.8 / p.C);
  k.eps = p.eps;
  for (int i = 0; i < 4; ++i) k.d[i] = p.d[i];
  k.cfl = p.cfl;
  k.dt_fixed = p.dt_fixed;
  k.characteristic = p.variables == GENO6_VARS_CHARACTERISTIC;
  return k;
}

unsigned tiles(const geno6_grid* g) { return (unsigned)((g->n + TC - 1) / TC); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WS6 {
  size_t slots, ya, yb, acc, total;
};

WS6 ws_layout(const geno6_grid* g) {
  WS6 w;
  size_t off = align256(sizeof(Ctrl6));
  w.slots = off;
  off = align256(off + sizeof(unsigned long long) * NSLOT);
  const size_t arr = align256(sizeof(double) * 3 * (size_t)g->pitch);
  w.ya = off;
  off += arr;
  w.yb = off;
  off += arr;
  w.acc = off;
  off += arr;
  w.total = off;
  return w;
}

}  // namespace

extern "C" {

int geno6_params_default(geno6_params* p) {
  if (!p) return fail(GENO_EINVAL, "null params");
  p->version = GENO6_ABI_VERSION;
  p->gamma = 1.4;
  p->C = 20.0;
  p->eps = 1e-15;
  p->d[0] = 1.0;
  p->d[1] = 8.0;
  p->d[2] = 1.0;
  p->d[3] = 1.0;
  p->cfl = 0.5;
  p->bc[0] = p->bc[1] = GENO_BC_PERIODIC;
  p->dt_fixed = 0.0;
  p->variables = GENO6_VARS_CONSERVATIVE;
  for (int e = 0; e < 2; ++e)
    for (int c = 0; c < 3; ++c)
      for (int f = 0; f < 3; ++f) p->ghost[e][c][f] = 0.0;
  return GENO_OK;
}

int geno6_grid_init(geno6_grid* g, int n, double x0, double x1, const geno6_params* p) {
  if (!g) return fail(GENO_EINVAL, "null grid");
  const int rc = check_params6(p);
  if (rc) return rc;
  if (n < 3) return fail(GENO_EINVAL, "at least 3 cells are required");
  if (n > 0x7fffffff - 1024) return fail(GENO_EINVAL, "too many cells for 32-bit indexing");
  if (!(x1 > x0)) return fail(GENO_EINVAL, "x1 must exceed x0");
  g->n = n;
  g->pitch = ((n + 63) / 64) * 64;
  g->x0 = x0;
  g->x1 = x1;
  g->dx = (x1 - x0) / n;
  g->params = *p;
  return GENO_OK;
}

size_t geno6_workspace_bytes(const geno6_grid* g) {
  if (check_grid6(g)) return 0;
  return ws_layout(g).total;
}

int geno6_faces(const geno6_grid* g, const double* U, double* UL, double* UR, double* F,
                double* chi, void* stream) {
  const int rc = check_grid6(g);
  if (rc) return rc;
  if (!U) return fail(GENO_EINVAL, "null state");
  const unsigned nb = (unsigned)((g->n + 1 + TB - 1) / TB);
  const KP6 k = kp6(g->params);
  if (k.characteristic)
    HIP_TRY(launch6(-1, k6_faces<true>, nb, (hipStream_t)stream, geo6(g), k, U, UL, UR, F, chi));
  else
    HIP_TRY(launch6(-1, k6_faces<false>, nb, (hipStream_t)stream, geo6(g), k, U, UL, UR, F, chi));
  return GENO_OK;
}

int geno6_rhs(const geno6_grid* g, const double* U, double* L, void* stream) {
  const int rc = check_grid6(g);
  if (rc) return rc;
  if (!U || !L) return fail(GENO_EINVAL, "null state");
  const KP6 k = kp6(g->params);
  auto kern = k.characteristic ? k6_stage<4, true> : k6_stage<4, false>;
  HIP_TRY(launch6(-1, kern, tiles(g), (hipStream_t)stream, geo6(g), k, U, (const double*)nullptr,
                  (double*)nullptr, L, (Ctrl6*)nullptr, (unsigned long long*)nullptr));
  return GENO_OK;
}

int geno6_step(const geno6_grid* g, double* U, void* ws, int nsteps, double* dt_out,
               geno_stats* stats, void* stream) {
  int rc = check_grid6(g);
  if (rc) return rc;
  if (!U || !ws) return fail(GENO_EINVAL, "null state or workspace");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const WS6 L = ws_layout(g);
  char* base = (char*)ws;
  Ctrl6* ctrl = (Ctrl6*)base;
  unsigned long long* slots = (unsigned long long*)(base + L.slots);
  double* ya = (double*)(base + L.ya);
  double* yb = (double*)(base + L.yb);
  double* acc = (double*)(base + L.acc);
  const Geo6 geo = geo6(g);
  const KP6 k = kp6(g->params);
  const unsigned nb = tiles(g);
  HIP_TRY(launch6(-1, k6_clear, 1, s, slots, ctrl));
  HIP_TRY(launch6(GENO6_K_INIT, k6_init, nb, s, geo, k.gamma, (const double*)U, slots));
  const bool ch = k.characteristic;
  auto s0 = ch ? k6_stage<0, true> : k6_stage<0, false>;
  auto s1 = ch ? k6_stage<1, true> : k6_stage<1, false>;
  auto s2 = ch ? k6_stage<2, true> : k6_stage<2, false>;
  auto s3 = ch ? k6_stage<3, true> : k6_stage<3, false>;
  for (int st = 0; st < nsteps; ++st) {
    HIP_TRY(launch6(GENO6_K_DT, k6_dt, 1, s, slots, g->dx, k.cfl, k.dt_fixed, ctrl, dt_out, st));
    HIP_TRY(launch6(GENO6_K_STAGE, s0, nb, s, geo, k, (const double*)U, (const double*)U, acc, ya,
                    ctrl, slots));
    HIP_TRY(launch6(GENO6_K_STAGE, s1, nb, s, geo, k, (const double*)ya, (const double*)U, acc, yb,
                    ctrl, slots));
    HIP_TRY(launch6(GENO6_K_STAGE, s2, nb, s, geo, k, (const double*)yb, (const double*)U, acc, ya,
                    ctrl, slots));
    HIP_TRY(launch6(GENO6_K_STAGE, s3, nb, s, geo, k, (const double*)ya, (const double*)U, acc, U,
                    ctrl, slots));
  }
  if (stats) {
    Ctrl6 h;
    HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->guard = (long long)h.guard;
    stats->nonfinite = (long long)h.nonfinite;
    stats->last_dt = nsteps > 0 ? h.dt : 0.0;
    if (h.nonfinite) return fail(GENO_ENONPHYS, "%llu non-physical cells", h.nonfinite);
  }
  return GENO_OK;
}

size_t geno6_batch_workspace_bytes(const geno6_grid* g, int ngrids) {
  if (check_grid6(g) || ngrids < 1) return 0;
  return align256(sizeof(Ctrl6)) + (size_t)ngrids * 3 * 3 * (size_t)g->pitch * sizeof(double);
}

int geno6_step_batch(const geno6_grid* g, int ngrids, double* U, void* ws, int nsteps,
                     double* dt_out, geno_stats* stats, void* stream) {
  int rc = check_grid6(g);
  if (rc) return rc;
  if (ngrids < 1 || ngrids > GENO6_BATCH_MAX) return fail(GENO_EINVAL, "ngrids must be in [1, %d]", GENO6_BATCH_MAX);
  if (!U || !ws) return fail(GENO_EINVAL, "null state or workspace");
  if (nsteps < 0) return fail(GENO_EINVAL, "nsteps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  Ctrl6* ctrl = (Ctrl6*)base;
  double* arrays = (double*)(base + align256(sizeof(Ctrl6)));
  const Geo6 geo = geo6(g);
  const KP6 k = kp6(g->params);
  const size_t stride = 3 * (size_t)g->pitch;
  HIP_TRY(launch6(-1, k6_clear, 1, s, (unsigned long long*)nullptr, ctrl));
  if (k.characteristic)
    HIP_TRY(launch6_bs(GENO6_K_SMALL, k6_small<true>, (unsigned)ngrids, SmallShape<true>::SB, s, geo,
                       k, U, arrays, stride, nsteps, dt_out, ctrl));
  else
    HIP_TRY(launch6_bs(GENO6_K_SMALL, k6_small<false>, (unsigned)ngrids, SmallShape<false>::SB, s,
                       geo, k, U, arrays, stride, nsteps, dt_out, ctrl));
  if (stats) {
    Ctrl6 h;
    HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    stats->guard = (long long)h.guard;
    stats->nonfinite = (long long)h.nonfinite;
    stats->last_dt = nsteps > 0 ? h.dt : 0.0;
    if (h.nonfinite) return fail(GENO_ENONPHYS, "%llu non-physical cells", h.nonfinite);
  }
  return GENO_OK;
}

int geno6_timing_enable(int max_launches) {
  for (int i = 0; i < 2 * g_tim6.cap; ++i) (void)hipEventDestroy(g_tim6.ev[i]);
  free(g_tim6.ev);
  free(g_tim6.kind);
  g_tim6 = Timing6{};
  if (max_launches <= 0) return GENO_OK;
  g_tim6.ev = (hipEvent_t*)calloc((size_t)2 * max_launches, sizeof(hipEvent_t));
  g_tim6.kind = (int*)calloc((size_t)max_launches, sizeof(int));
  if (!g_tim6.ev || !g_tim6.kind) return fail(GENO_EINVAL, "out of host memory");
  for (int i = 0; i < 2 * max_launches; ++i) {
    const hipError_t e = hipEventCreate(&g_tim6.ev[i]);
    if (e != hipSuccess) {
      g_tim6.cap = i / 2;
      return fail(GENO_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  g_tim6.cap = max_launches;
  return GENO_OK;
}

int geno6_timing_read(int nkinds, double* ms_total, long long* launches) {
  if (!ms_total || !launches || nkinds < 1) return fail(GENO_EINVAL, "null argument");
  for (int q = 0; q < nkinds; ++q) {
    ms_total[q] = 0.0;
    launches[q] = 0;
  }
  for (int i = 0; i < g_tim6.used; ++i) {
    HIP_TRY(hipEventSynchronize(g_tim6.ev[2 * i + 1]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, g_tim6.ev[2 * i], g_tim6.ev[2 * i + 1]));
    const int q = g_tim6.kind[i];
    if (q < nkinds) {
      ms_total[q] += ms;
      launches[q] += 1;
    }
  }
  g_tim6.used = 0;
  return GENO_OK;
}

}  // extern "C"
