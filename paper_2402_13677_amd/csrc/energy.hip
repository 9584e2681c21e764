// The advection step of the energy equation (Sec. 2.4, Eq. energy_advection):
// one explicit Euler step of dT/dt + u . grad T = 0 in each phase,
//
//   T*_k = T_k - dt * (u_0 D_0 + u_1 D_1 + u_2 D_2),
//
// each cell with its own phase's temperature field (the caller's fields
// carry the values extended across the interface) and its own phase's
// velocity at the centre (the mean of its two faces per axis).  D_a is the
// third-order WENO derivative of Jiang & Shu: the difference of the values
// at the cell's two a-faces times 1/h, each reconstructed from the upwind side
// (the sign of u_a) from the two candidate stencils (m, 0) and (0, p) with
// linear weights 1/3 and 2/3 and smoothness indicators (T_0 - T_m)^2 and
// (T_p - T_0)^2.  A stencil cell beyond a wall takes the nearest cell's
// value; periodic axes wrap.  A zero velocity component contributes
// nothing.
//
// Layout and launch: one thread per cell, a block per 16 x 16 tile of an
// x-y plane.  The tile rows are grouped into eight strips (as many as there
// are XCDs, each with its own L2); the blocks are ordered strip by strip,
// within a strip plane by plane from the bottom, and within a plane tile by
// tile, so the contiguous range of blocks an XCD takes is one strip climbed
// plane by plane.  Each thread reads its colour byte, its phase's 2 faces
// per axis, the centre and the 4 cells at distance 1 and 2 along each axis:
// the x and y neighbours of a tile come from tiles of the same strip and
// plane, just read into the same L2, and the z neighbours from the planes
// just below; only the rows next to another strip are fetched twice.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {
namespace {

constexpr int EN_TX = 16, EN_TY = 16, EN_BLOCK = EN_TX * EN_TY;

struct EnergyArgs {
  Dims d;
  double inv_h, dt, eps;
  const uint8_t* ccol;
  const double* T[2];     // [0] vapour, [1] liquid
  const double* u[2][3];  // face fields per phase and axis
  double* out;
};

// The difference of the two face values a cell's derivative takes, seen
// from the upwind side: with the stencil ordered upwind to downwind as
// (a, b, c, e) (c the cell), the face c|e from (b, c | e) and the face b|c
// from (a, b | c).  Each face value is written as its upwind cell plus half
// the weighted mean of the two one-sided differences,
//   face = t0 + (w0 (t0 - tm) + w1 (tp - t0)) / (2 (w0 + w1)),
// the Jiang & Shu weights alpha_r = d_r / (eps + beta_r)^2 scaled by the
// common factor (eps + beta0)^2 (eps + beta1)^2 (w0 = d0 (eps + beta1)^2,
// w1 = d1 (eps + beta0)^2); both faces' quotients share one division.
__device__ inline double weno3_diff(double a, double b, double c, double e, double eps) {
  const double g_ab = b - a, g_bc = c - b, g_ce = e - c;
  const double e_ab = eps + g_ab * g_ab, e_bc = eps + g_bc * g_bc, e_ce = eps + g_ce * g_ce;
  // face c|e: (m, 0, p) = (b, c, e); face b|c: (a, b, c)
  const double wu0 = (1.0 / 3.0) * (e_ce * e_ce), wu1 = (2.0 / 3.0) * (e_bc * e_bc);
  const double wl0 = (1.0 / 3.0) * (e_bc * e_bc), wl1 = (2.0 / 3.0) * (e_ab * e_ab);
  const double nu = wu0 * g_bc + wu1 * g_ce, du = wu0 + wu1;
  const double nl = wl0 * g_ab + wl1 * g_bc, dl = wl0 + wl1;
  return g_bc + 0.5 * ((nu * dl - nl * du) / (du * dl));
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
  // a context's grid has fewer than 2^31 cells (and fewer than 2^32 faces
  // per axis): 32-bit offsets throughout.  Block t: strip s = t / (n2 gx sh),
  // then the plane and the tile within the strip's sh rows of gx tiles.
  const Dims& d = g.d;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int n2 = d.n[2];
  const int gx = (d.n[0] + EN_TX - 1) / EN_TX, gy = (d.n[1] + EN_TY - 1) / EN_TY;
  const int sh = (gy + 7) / 8;
  const int per_plane = gx * sh, per_strip = per_plane * n2;
  const int st_i = t / per_strip, r = t - st_i * per_strip;
  const int kz = r / per_plane, q = r - kz * per_plane;
  const int ty = st_i * sh + q / gx, tx = q % gx;
  const int ijk[3] = {tx * EN_TX + (int)(threadIdx.x % EN_TX), ty * EN_TY + (int)(threadIdx.x / EN_TX), kz};
  if (ty >= gy || ijk[0] >= d.n[0] || ijk[1] >= d.n[1]) return;
  const unsigned n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
  const unsigned c = (unsigned)ijk[0] + n0 * ((unsigned)ijk[1] + n1 * (unsigned)kz);
  const int ph = g.ccol[c] ? 1 : 0;
  const double* __restrict__ T = g.T[ph];
  const unsigned st[3] = {1u, n0, n0 * n1};
  const double tc = T[c];
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    // the cell's velocity component: the mean of its two a-faces
    const unsigned fn0 = n0 + (a == 0 ? 1u : 0u), fn1 = n1 + (a == 1 ? 1u : 0u);
    const unsigned lo = (unsigned)ijk[0] + fn0 * ((unsigned)ijk[1] + fn1 * (unsigned)ijk[2]);
    const unsigned up = lo + (a == 0 ? 1u : a == 1 ? n0 : n0 * n1);
    const double* __restrict__ f = g.u[ph][a];
    const double ua = 0.5 * (f[lo] + f[up]);
    // the four stencil cells along a (offsets -2, -1, +1, +2)
    const bool per = d.per[a] != 0;
    const int n = d.n[a], ia = ijk[a];
    const unsigned base = c - (unsigned)ia * st[a];
    const double tm2 = T[base + (unsigned)wrap_clamp(ia - 2, n, per) * st[a]];
    const double tm1 = T[base + (unsigned)wrap_clamp(ia - 1, n, per) * st[a]];
    const double tp1 = T[base + (unsigned)wrap_clamp(ia + 1, n, per) * st[a]];
    const double tp2 = T[base + (unsigned)wrap_clamp(ia + 2, n, per) * st[a]];
    // the stencil ordered from the upwind side (u > 0: i-2, i-1, i, i+1;
    // u < 0: i+2, i+1, i, i-1), selected rather than branched on; the
    // downstream face minus the upstream one is then D_a h in the direction
    // of the flow, so u_a D_a = |u_a| weno3_diff / h.  A zero component
    // contributes exactly 0, whatever its stencil holds.
    const bool pos = ua > 0.0;
    const double df = weno3_diff(pos ? tm2 : tp2, pos ? tm1 : tp1, tc, pos ? tp1 : tm1, g.eps);
    const double t = ua != 0.0 ? fabs(ua) * (df * g.inv_h) : 0.0;
    acc = a == 0 ? t : acc + t;
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
  g.inv_h = 1.0 / h;
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
  const long long gx = (d->n[0] + EN_TX - 1) / EN_TX, gy = (d->n[1] + EN_TY - 1) / EN_TY;
  const long long sh = (gy + 7) / 8;
  const long long blocks = ((gy + sh - 1) / sh) * sh * gx * d->n[2];
  if (blocks == 0) return hipSuccess;
  if (d->dim == 3)
    hipLaunchKernelGGL(k_advect_energy<3>, dim3((unsigned)blocks), dim3(EN_BLOCK), 0, st, g);
  else
    hipLaunchKernelGGL(k_advect_energy<2>, dim3((unsigned)blocks), dim3(EN_BLOCK), 0, st, g);
  return hipGetLastError();
}
