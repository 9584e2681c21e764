// The advection step of the energy equation (Sec. 2.4, Eq. energy_advection):
// one explicit Euler step of dT/dt + u . grad T = 0 in each phase,
//
//   T*_k = T_k - dt * (u_0 D_0 + u_1 D_1 + u_2 D_2),
//
// each cell with its own phase's temperature field (the caller's fields
// carry the values extended across the interface) and its own phase's
// velocity at the centre (the mean of its two faces per axis).  D_a is the
// third-order WENO derivative of Jiang & Shu: the difference over h of the
// values at the cell's two a-faces, each reconstructed from the upwind side
// (the sign of u_a) from the two candidate stencils (m, 0) and (0, p) with
// linear weights 1/3 and 2/3 and smoothness indicators (T_0 - T_m)^2 and
// (T_p - T_0)^2.  A stencil cell beyond a wall takes the nearest cell's
// value; periodic axes wrap.  A zero velocity component contributes
// nothing.
//
// Layout and launch: one thread per cell in the natural order; each thread
// reads its colour byte, its phase's 2 faces per axis, the centre and the 4
// cells at distance 1 and 2 along each axis (the y and z neighbours come
// from the L2: the blocks of one XCD take a contiguous range of rows).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {
namespace {

constexpr int EN_BLOCK = 256;

struct EnergyArgs {
  Dims d;
  double h, dt, eps;
  const uint8_t* ccol;
  const double* T[2];     // [0] vapour, [1] liquid
  const double* u[2][3];  // face fields per phase and axis
  double* out;
};

// Face value from the upwind cells (m, 0) and the downwind cell p.  The
// weights alpha_r = d_r / (eps + beta_r)^2 enter only through their ratio,
// so both are multiplied by (eps + beta0)^2 (eps + beta1)^2: one division.
__device__ inline double weno3_face(double tm, double t0, double tp, double eps) {
  const double q0 = 0.5 * (3.0 * t0 - tm);
  const double q1 = 0.5 * (t0 + tp);
  const double g0 = t0 - tm, g1 = tp - t0;
  const double e0 = eps + g0 * g0, e1 = eps + g1 * g1;
  const double w0 = (1.0 / 3.0) * (e1 * e1), w1 = (2.0 / 3.0) * (e0 * e0);
  return (w0 * q0 + w1 * q1) / (w0 + w1);
}

// index v (at most two steps outside [0, n)) wrapped or clamped
__device__ inline int wrap_clamp(int v, int n, bool per) {
  if (per) {
    if (v < 0) v += n;
    if (v < 0) v += n;
    if (v >= n) v -= n;
    if (v >= n) v -= n;
    return v;
  }
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

template <int DIM>
__global__ __launch_bounds__(EN_BLOCK) void k_advect_energy(EnergyArgs g) {
  const long long c = (long long)xcd_tile(blockIdx.x, gridDim.x) * EN_BLOCK + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N) return;
  int ijk[3];
  cell_ijk(d, c, ijk[0], ijk[1], ijk[2]);
  const int ph = g.ccol[c] ? 1 : 0;
  const double* __restrict__ T = g.T[ph];
  const long long st[3] = {1, d.n[0], (long long)d.n[0] * d.n[1]};
  const double tc = T[c];
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    // the cell's velocity component: the mean of its two a-faces
    const long long fn0 = d.n[0] + (a == 0 ? 1 : 0), fn1 = d.n[1] + (a == 1 ? 1 : 0);
    const long long lo = (long long)ijk[0] + fn0 * ((long long)ijk[1] + fn1 * ijk[2]);
    const long long up = lo + (a == 0 ? 1LL : a == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1]);
    const double* __restrict__ f = g.u[ph][a];
    const double ua = 0.5 * (f[lo] + f[up]);
    // the four stencil cells along a (offsets -2, -1, +1, +2)
    const bool per = d.per[a] != 0;
    const int n = d.n[a], ia = ijk[a];
    const long long base = c - (long long)ia * st[a];
    const double tm2 = T[base + (long long)wrap_clamp(ia - 2, n, per) * st[a]];
    const double tm1 = T[base + (long long)wrap_clamp(ia - 1, n, per) * st[a]];
    const double tp1 = T[base + (long long)wrap_clamp(ia + 1, n, per) * st[a]];
    const double tp2 = T[base + (long long)wrap_clamp(ia + 2, n, per) * st[a]];
    double D = 0.0;
    if (ua > 0.0)
      D = (weno3_face(tm1, tc, tp1, g.eps) - weno3_face(tm2, tm1, tc, g.eps)) / g.h;
    else if (ua < 0.0)
      D = (weno3_face(tp2, tp1, tc, g.eps) - weno3_face(tp1, tc, tm1, g.eps)) / g.h;
    acc = a == 0 ? ua * D : acc + ua * D;
  }
  g.out[c] = tc - g.dt * acc;
}

}  // namespace
}  // namespace ebit

using namespace ebit;

extern "C" hipError_t ebit_launch_advect_energy(const Dims* d, double h, const double* T_liq, const double* T_vap,
                                                const double* const u_l[3], const double* const u_v[3],
                                                const uint8_t* ccol, double dt, double eps, double* out,
                                                hipStream_t st) {
  EnergyArgs g;
  g.d = *d;
  g.h = h;
  g.dt = dt;
  g.eps = eps;
  g.ccol = ccol;
  g.T[0] = T_vap;
  g.T[1] = T_liq;
  for (int a = 0; a < 3; ++a) {
    g.u[1][a] = a < d->dim ? u_l[a] : nullptr;
    g.u[0][a] = a < d->dim ? u_v[a] : nullptr;
  }
  g.out = out;
  const long long blocks = (d->N + EN_BLOCK - 1) / EN_BLOCK;
  if (blocks == 0) return hipSuccess;
  if (d->dim == 3)
    hipLaunchKernelGGL(k_advect_energy<3>, dim3((unsigned)blocks), dim3(EN_BLOCK), 0, st, g);
  else
    hipLaunchKernelGGL(k_advect_energy<2>, dim3((unsigned)blocks), dim3(EN_BLOCK), 0, st, g);
  return hipGetLastError();
}
