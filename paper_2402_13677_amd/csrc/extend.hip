// Narrow-band extension of a cell field across the interface (Sec. 2.4,
// Eq. extrapolation): explicit pseudo-time steps of first-order upwind
// transport along the interface normal, pointing out of the region that holds
// the data.
//
// Discretisation (the paper gives the equation and the band only):
//   * band: cells whose 3^d block (the cell included) holds an interface cell;
//   * band normal: the normalised sum of those interface cells' facet normals
//     (vapour -> liquid), visited with the x offset slowest, z fastest;
//   * velocity a = +n in liquid cells, -n in vapour cells;
//   * targets: the vapour band cells (liquid -> vapour), the liquid band cells
//     (vapour -> liquid) or the band cells off the interface (interface ->
//     band), each with a non-zero normal sum;
//   * f(c) <- f(c) - (1/d) sum_d |a_d| (f(c) - f(up_d(c))), up_d the upwind
//     neighbour along axis d (c - e_d for a_d > 0, c + e_d for a_d < 0), a
//     term kept only when that neighbour exists (walls stop, periodic axes
//     wrap) and holds data or is a target; all targets from the previous
//     iterate.
//
// Layout.  Per cell a 16-bit code: bit 0 target; per axis d three bits at
// 1 + 3d: term kept, upwind side is c + e_d, upwind cell is a target.  The
// weights |a_d| sit in three cell arrays (only targets' entries are written
// or read).  The iterate alternates between q and a work array: a target
// reads targets from the current source and every other cell from q, whose
// non-target entries never change.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {
namespace {

constexpr int EXT_BLOCK = 256;

__device__ inline bool ext_data(int mode, uint8_t fl) {
  if (mode == EBIT_EXT_LIQ_TO_VAP) return (fl >> 6) & 1;
  if (mode == EBIT_EXT_VAP_TO_LIQ) return !((fl >> 6) & 1);
  return (fl >> 7) & 1;
}

__device__ inline bool ext_candidate(int mode, uint8_t fl) {
  // a band cell of this colour (or off the interface) is updated
  if (mode == EBIT_EXT_LIQ_TO_VAP) return !((fl >> 6) & 1);
  if (mode == EBIT_EXT_VAP_TO_LIQ) return (fl >> 6) & 1;
  return !((fl >> 7) & 1);
}

// neighbour of (i, j, k) at offsets (di, dj, dk); false beyond a wall
__device__ inline bool ext_nbr(const Dims& d, int i, int j, int k, int di, int dj, int dk, long long& m) {
  int p[3] = {i + di, j + dj, k + dk};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= d.dim) continue;
    if (p[a] < 0 || p[a] >= d.n[a]) {
      if (!d.per[a]) return false;
      p[a] = p[a] < 0 ? p[a] + d.n[a] : p[a] - d.n[a];
    }
  }
  m = (long long)p[0] + (long long)d.n[0] * ((long long)p[1] + (long long)d.n[1] * p[2]);
  return true;
}

struct ExtArgs {
  Dims d;
  int mode;
  const uint8_t* flags;
  const double* nF;  // 3 arrays of N: x, y, z
  uint16_t* code;
  double* w[3];
};

// pass 1: target bit and the signed velocity a = +-n per target
__global__ void k_ext_mark(ExtArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N) return;
  const uint8_t fc = g.flags[c];
  uint16_t out = 0;
  if (ext_candidate(g.mode, fc)) {
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const int rz = d.dim == 3 ? 1 : 0;
    bool inb = false;
    double s[3] = {0.0, 0.0, 0.0};
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj)
        for (int dk = -rz; dk <= rz; ++dk) {
          long long m;
          if (!ext_nbr(d, i, j, k, di, dj, dk, m)) continue;
          if (!((g.flags[m] >> 7) & 1)) continue;
          inb = true;
          s[0] += g.nF[m];
          s[1] += g.nF[d.N + m];
          if (d.dim == 3) s[2] += g.nF[2 * d.N + m];
        }
    const double L = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (inb && L > 0.0) {
      out = 1;
      const double sg = ((fc >> 6) & 1) ? 1.0 : -1.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a < d.dim) g.w[a][c] = sg * (s[a] / L);
    }
  }
  g.code[c] = out;
}

// pass 2: which upwind terms a target keeps, and where they are read from.
// It reads neighbours' target bits and rewrites its own code; a rewrite
// keeps bit 0, so what a neighbour reads does not depend on the order.
__global__ void k_ext_terms(ExtArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N) return;
  uint16_t code = g.code[c];
  if (!(code & 1)) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= d.dim) continue;
    const double av = g.w[a][c];
    bool keep = false, plus = av < 0.0, tgt = false;
    if (av != 0.0) {
      const int s = plus ? 1 : -1;
      long long m;
      if (ext_nbr(d, i, j, k, a == 0 ? s : 0, a == 1 ? s : 0, a == 2 ? s : 0, m)) {
        tgt = g.code[m] & 1;
        keep = tgt || ext_data(g.mode, g.flags[m]);
      }
    }
    g.w[a][c] = keep ? fabs(av) : 0.0;
    code |= (uint16_t)((keep ? 1 : 0) | (plus ? 2 : 0) | (tgt ? 4 : 0)) << (1 + 3 * a);
  }
  g.code[c] = code;
}

template <int DIM>
__global__ __launch_bounds__(EXT_BLOCK) void k_ext_step(Dims d, const uint16_t* __restrict__ code,
                                                        const double* __restrict__ w0, const double* __restrict__ w1,
                                                        const double* __restrict__ w2, const double* q,
                                                        const double* src, double* dst, double lam) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  const uint16_t cd = code[c];
  if (!(cd & 1)) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const double f = src[c];
  double up[DIM], wt[DIM];
  // every load first
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int bits = (cd >> (1 + 3 * a)) & 7;
    up[a] = f;
    wt[a] = 0.0;
    if (bits & 1) {
      const int s = (bits & 2) ? 1 : -1;
      long long m = c;
      ext_nbr(d, i, j, k, a == 0 ? s : 0, a == 1 ? s : 0, a == 2 ? s : 0, m);
      up[a] = (bits & 4) ? src[m] : q[m];
      wt[a] = (a == 0 ? w0 : a == 1 ? w1 : w2)[c];
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) acc += wt[a] * (f - up[a]);
  dst[c] = f - lam * acc;
}

__global__ void k_ext_copy(long long N, const uint16_t* __restrict__ code, const double* __restrict__ src,
                           double* __restrict__ dst) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N && (code[c] & 1)) dst[c] = src[c];
}

}  // namespace
}  // namespace ebit

using namespace ebit;

extern "C" hipError_t ebit_launch_extend(const Dims* d, int mode, int iters, const uint8_t* flags, const double* nF,
                                         double* q, double* work, uint16_t* code, double* const w[3],
                                         hipStream_t st) {
  ExtArgs g;
  g.d = *d;
  g.mode = mode;
  g.flags = flags;
  g.nF = nF;
  g.code = code;
  for (int a = 0; a < 3; ++a) g.w[a] = w[a];
  const unsigned nb = (unsigned)((d->N + EXT_BLOCK - 1) / EXT_BLOCK);
  hipLaunchKernelGGL(k_ext_mark, dim3(nb), dim3(EXT_BLOCK), 0, st, g);
  hipLaunchKernelGGL(k_ext_terms, dim3(nb), dim3(EXT_BLOCK), 0, st, g);
  const double lam = 1.0 / d->dim;
  const double* w2 = d->dim == 3 ? w[2] : w[0];
  const double* src = q;
  double* dst = work;
  for (int t = 0; t < iters; ++t) {
    if (d->dim == 3)
      hipLaunchKernelGGL(k_ext_step<3>, dim3(nb), dim3(EXT_BLOCK), 0, st, *d, (const uint16_t*)code,
                         (const double*)w[0], (const double*)w[1], w2, (const double*)q, src, dst, lam);
    else
      hipLaunchKernelGGL(k_ext_step<2>, dim3(nb), dim3(EXT_BLOCK), 0, st, *d, (const uint16_t*)code,
                         (const double*)w[0], (const double*)w[1], w2, (const double*)q, src, dst, lam);
    src = dst;
    dst = (dst == work) ? q : work;
  }
  // an odd count leaves the last iterate in the work array
  if (src == work)
    hipLaunchKernelGGL(k_ext_copy, dim3(nb), dim3(EXT_BLOCK), 0, st, d->N, (const uint16_t*)code,
                       (const double*)work, q);
  return hipGetLastError();
}
