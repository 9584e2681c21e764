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
// Layout.  The band comes from a separable dilation of the interface bit
// (one pass per axis over byte arrays), then a byte per cell marks the
// targets.  The targets are then listed compactly (order immaterial: every
// target is updated from the previous iterate): per entry the cell index and
// a code (per axis d three bits at 3d: term kept, upwind side is c + e_d,
// upwind cell is a target), and per axis the weight |a_d| (0 when the term
// is dropped).  A step touches only the listed cells.  The iterate
// alternates between q and a work array: a target reads targets from the
// current source and every other cell from q, whose non-target entries
// never change.
//
// The same band carries Eq. ghost_velocity from the extended mass flux to
// every face whose two cells are band cells (k_ghost_band): cut faces by the
// projection's rule, uncut faces with the means of the two cells' mass flux
// and unit band normals.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebit_internal.h"
#include "ghost.h"

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

// OR of the per-cell bit over the three cells c - e_AX, c, c + e_AX; the
// first pass takes the interface bit of the flags (and clears the list
// counter).  Block b takes EXT_BLOCK cells of one x row (rows of more cells
// take several blocks): the cell index comes from a row number and an
// offset, with no per-thread division.
__global__ __launch_bounds__(EXT_BLOCK) void k_ext_dilate(Dims d, int ax, const uint8_t* __restrict__ flags,
                                                          const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                          int* counter) {
  const unsigned n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
  const unsigned per_row = (n0 + EXT_BLOCK - 1) / EXT_BLOCK;
  const unsigned row = blockIdx.x / per_row;
  const unsigned i = (blockIdx.x - row * per_row) * EXT_BLOCK + threadIdx.x;
  if (i >= n0) return;
  const unsigned c = row * n0 + i;
  if (!in && c == 0) *counter = 0;
  const unsigned j = row % n1, k = row / n1;
  const unsigned ia = ax == 0 ? i : (ax == 1 ? j : k);
  const unsigned na = (unsigned)d.n[ax];
  const unsigned st = ax == 0 ? 1u : (ax == 1 ? n0 : n0 * n1);
  const bool per = d.per[ax] != 0;
  // the two neighbours along AX (the cell itself where there is none)
  const unsigned lo = ia > 0 ? c - st : (per ? c + (na - 1) * st : c);
  const unsigned hi = ia + 1 < na ? c + st : (per ? c - (na - 1) * st : c);
  uint8_t v;
  if (in)
    v = in[lo] | in[c] | in[hi];
  else
    v = (uint8_t)(((flags[lo] | flags[c] | flags[hi]) >> 7) & 1);
  out[c] = v;
}

// The same pass four cells at a time, for rows of a multiple of 4 cells (so
// every row starts on a 4-byte boundary): thread t takes the 32-bit word of
// cells 4t .. 4t+3 (byte b of the word is cell 4t+b).  Along x the word is
// ORed with itself shifted by one byte either way and with the bytes of the
// cells just outside it; along y or z with the words of the rows either side.
__global__ __launch_bounds__(EXT_BLOCK) void k_ext_dilate4(Dims d, int ax, const uint8_t* __restrict__ flags,
                                                           const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                           int* counter) {
  const unsigned t = blockIdx.x * EXT_BLOCK + threadIdx.x;
  const unsigned N = (unsigned)d.N;
  if (t >= N / 4) return;
  const unsigned c = 4 * t;
  if (!in && c == 0) *counter = 0;
  const unsigned n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
  const unsigned row = c / n0, i = c - row * n0;
  const uint8_t* src = in ? in : flags;
  // the interface bit of each byte on the first pass, the byte itself after
  auto bits = [&](unsigned w) { return in ? w : (w >> 7) & 0x01010101u; };
  const unsigned w = bits(*reinterpret_cast<const unsigned*>(src + c));
  unsigned v;
  if (ax == 0) {
    const bool per = d.per[0] != 0;
    unsigned left = 0, right = 0;
    if (i > 0)
      left = src[c - 1];
    else if (per)
      left = src[c + n0 - 1];
    if (i + 4 < n0)
      right = src[c + 4];
    else if (per)
      right = src[c + 4 - n0];
    left = bits(left) & 0xffu;
    right = bits(right) & 0xffu;
    v = w | (w << 8) | (w >> 8) | left | (right << 24);
  } else {
    const unsigned j = row % n1, k = row / n1;
    const unsigned ia = ax == 1 ? j : k;
    const unsigned na = (unsigned)d.n[ax];
    const unsigned st = ax == 1 ? n0 : n0 * n1;
    const bool per = d.per[ax] != 0;
    const unsigned lo = ia > 0 ? c - st : (per ? c + (na - 1) * st : c);
    const unsigned hi = ia + 1 < na ? c + st : (per ? c - (na - 1) * st : c);
    v = w | bits(*reinterpret_cast<const unsigned*>(src + lo)) | bits(*reinterpret_cast<const unsigned*>(src + hi));
  }
  *reinterpret_cast<unsigned*>(out + c) = v;
}

// blocks of k_ext_dilate (whole rows of EXT_BLOCK-cell chunks) or, for rows
// of a multiple of 4 cells, of k_ext_dilate4
inline bool dilate_by_words(const Dims* d) { return d->n[0] % 4 == 0; }
inline unsigned dilate_blocks(const Dims* d) {
  if (dilate_by_words(d)) return (unsigned)((d->N / 4 + EXT_BLOCK - 1) / EXT_BLOCK);
  const unsigned per_row = ((unsigned)d->n[0] + EXT_BLOCK - 1) / EXT_BLOCK;
  return per_row * (unsigned)d->n[1] * (unsigned)d->n[2];
}
inline void launch_dilate(const Dims* d, int ax, const uint8_t* flags, const uint8_t* in, uint8_t* out, int* counter,
                          hipStream_t st) {
  if (dilate_by_words(d))
    hipLaunchKernelGGL(k_ext_dilate4, dim3(dilate_blocks(d)), dim3(EXT_BLOCK), 0, st, *d, ax, flags, in, out, counter);
  else
    hipLaunchKernelGGL(k_ext_dilate, dim3(dilate_blocks(d)), dim3(EXT_BLOCK), 0, st, *d, ax, flags, in, out, counter);
}

struct ExtArgs {
  Dims d;
  int mode;
  const uint8_t* flags;
  const double* nF;  // 3 arrays of N: x, y, z
  const uint8_t* band;
  uint8_t* tgt;
  unsigned long long* list;
  double* w[3];
  double* ns[3];  // the band normal sum of every target (scratch, cells)
  int* counter;
};

// target byte per cell: in the band, of the mode's colour, a normal
__global__ void k_ext_mark(ExtArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N) return;
  uint8_t t = 0;
  if (g.band[c] && ext_candidate(g.mode, g.flags[c])) {
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    double s[3];
    t = band_normal_sum(d, g.flags, g.nF, i, j, k, s) ? 1 : 0;
    // kept for the list pass (read back for targets only)
    if (t)
      for (int a = 0; a < d.dim; ++a) g.ns[a][c] = s[a];
  }
  g.tgt[c] = t;
}

// the list: every target's kept upwind terms and weights, appended at a slot
// taken per wave
__global__ __launch_bounds__(EXT_BLOCK) void k_ext_list(ExtArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  const bool act = c < d.N && g.tgt[c];
  unsigned code = 0;
  double wt[3] = {0.0, 0.0, 0.0};
  if (act) {
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    // the band normal sum the mark pass computed
    const double s[3] = {g.ns[0][c], g.ns[1][c], d.dim == 3 ? g.ns[2][c] : 0.0};
    const double L = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double sg = ((g.flags[c] >> 6) & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= d.dim) continue;
      const double av = sg * (s[a] / L);
      bool keep = false, tg = false;
      const bool plus = av < 0.0;
      if (av != 0.0) {
        const int sd = plus ? 1 : -1;
        long long m;
        if (nbr_cell(d, i, j, k, a == 0 ? sd : 0, a == 1 ? sd : 0, a == 2 ? sd : 0, m)) {
          tg = g.tgt[m] != 0;
          keep = tg || ext_data(g.mode, g.flags[m]);
        }
      }
      wt[a] = keep ? fabs(av) : 0.0;
      code |= (unsigned)((keep ? 1 : 0) | (plus ? 2 : 0) | (tg ? 4 : 0)) << (3 * a);
    }
  }
  // one atomic per wave for the wave's targets
  const unsigned long long mask = __ballot(act);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(g.counter, __popcll(mask));
  base = __shfl(base, leader);
  if (!act) return;
  const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
  g.list[slot] = (unsigned long long)c | ((unsigned long long)code << 40);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < d.dim) g.w[a][slot] = wt[a];
}

template <int DIM>
__global__ __launch_bounds__(EXT_BLOCK) void k_ext_step(Dims d, const unsigned long long* __restrict__ list,
                                                        const int* __restrict__ counter,
                                                        const double* __restrict__ w0, const double* __restrict__ w1,
                                                        const double* __restrict__ w2, const double* q,
                                                        const double* src, double* dst, double lam) {
  const int T = *counter;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (long long)gridDim.x * blockDim.x) {
    const unsigned long long e = list[t];
    const long long c = (long long)(e & ((1ull << 40) - 1));
    const unsigned cd = (unsigned)(e >> 40);
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const double f = src[c];
    double up[DIM], wt[DIM];
    // every load first
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const unsigned bits = (cd >> (3 * a)) & 7;
      up[a] = f;
      wt[a] = (a == 0 ? w0 : a == 1 ? w1 : w2)[t];
      if (bits & 1) {
        const int s = (bits & 2) ? 1 : -1;
        long long m = c;
        nbr_cell(d, i, j, k, a == 0 ? s : 0, a == 1 ? s : 0, a == 2 ? s : 0, m);
        up[a] = (bits & 4) ? src[m] : q[m];
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc += wt[a] * (f - up[a]);
    dst[c] = f - lam * acc;
  }
}

__global__ void k_ext_copy(const unsigned long long* __restrict__ list, const int* __restrict__ counter,
                           const double* __restrict__ src, double* __restrict__ dst) {
  const int T = *counter;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (long long)gridDim.x * blockDim.x) {
    const long long c = (long long)(list[t] & ((1ull << 40) - 1));
    dst[c] = src[c];
  }
}

struct GhostBandArgs {
  Dims d;
  double jump;  // [1/rho] = 1/rho_l - 1/rho_v
  const uint8_t* flags;
  const uint8_t* band;
  const double* th[3];
  const double* nF;
  const double* mdot;  // the mass flux carried to the band
  double* nb[3];       // the unit band normal of every band cell (scratch)
  double* ul[3];
  double* uv[3];
};

// The unit band normal of every band cell (zero where the sum of its
// block's facet normals vanishes), for k_ghost_band to read for both cells
// of a face.
__global__ __launch_bounds__(EXT_BLOCK) void k_ghost_band_normal(GhostBandArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N || !g.band[c]) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  double s[3];
  const bool on = band_normal_sum(d, g.flags, g.nF, i, j, k, s);
  const double L = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  for (int a = 0; a < d.dim; ++a) g.nb[a][c] = on ? s[a] / L : 0.0;
}

// Eq. ghost_velocity on the band faces.  Each band cell handles its + faces
// and, on the first layer, face 0 (the periodic copy of face n), as the
// projection's ghost kernel does; every cut face has two band cells (its
// holder carries a facet, the other cell lies in the holder's block), so the
// cut faces handled here are exactly the projection's.
__global__ __launch_bounds__(EXT_BLOCK) void k_ghost_band(GhostBandArgs g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Dims& d = g.d;
  if (c >= d.N || !g.band[c]) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const uint8_t f = g.flags[c];
  for (int s = 0; s < 2 * d.dim; ++s) {
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    if (!(up || ia == 0)) continue;
    const int sd = up ? 1 : -1;
    long long m;
    if (!nbr_cell(d, i, j, k, a == 0 ? sd : 0, a == 1 ? sd : 0, a == 2 ? sd : 0, m)) continue;  // a wall
    const long long fi = face_of_side(d, i, j, k, s);
    if ((f >> s) & 1) {
      const long long lo = up ? c : m, hi = up ? m : c;
      cut_face_ghost(d, g.flags, g.nF, g.mdot, g.jump, a, lo, hi, g.th[a][fi], fi, g.ul[a], g.uv[a]);
      continue;
    }
    if (!g.band[m]) continue;
    const double mf = 0.5 * (g.mdot[c] + g.mdot[m]);
    const double nf = 0.5 * (g.nb[a][c] + g.nb[a][m]);
    const double jmp = mf * g.jump * nf;
    if (f & F_LIQ)
      g.uv[a][fi] = g.ul[a][fi] + jmp;
    else
      g.ul[a][fi] = g.uv[a][fi] - jmp;
  }
}

}  // namespace
}  // namespace ebit

using namespace ebit;

extern "C" hipError_t ebit_launch_extend(const Dims* d, int mode, int iters, const uint8_t* flags, const double* nF,
                                         double* q, double* work, uint8_t* bytes, unsigned long long* list,
                                         double* const w[3], double* const ns[3], int* counter, hipStream_t st) {
  const unsigned nb = (unsigned)((d->N + EXT_BLOCK - 1) / EXT_BLOCK);
  const unsigned nl = nb < 2048u ? nb : 2048u;
  uint8_t* A = bytes;
  uint8_t* B = bytes + d->N;
  // band = the interface bit dilated along each axis in turn
  const uint8_t* in = nullptr;
  uint8_t* out = A;
  for (int ax = 0; ax < d->dim; ++ax) {
    launch_dilate(d, ax, flags, in, out, counter, st);
    in = out;
    out = (out == A) ? B : A;
  }
  ExtArgs g;
  g.d = *d;
  g.mode = mode;
  g.flags = flags;
  g.nF = nF;
  g.band = in;
  g.tgt = out;
  g.list = list;
  for (int a = 0; a < 3; ++a) {
    g.w[a] = w[a];
    g.ns[a] = a < d->dim ? ns[a] : nullptr;
  }
  g.counter = counter;
  hipLaunchKernelGGL(k_ext_mark, dim3(nb), dim3(EXT_BLOCK), 0, st, g);
  hipLaunchKernelGGL(k_ext_list, dim3(nb), dim3(EXT_BLOCK), 0, st, g);
  const double lam = 1.0 / d->dim;
  const double* w2 = d->dim == 3 ? w[2] : w[0];
  const double* src = q;
  double* dst = work;
  for (int t = 0; t < iters; ++t) {
    if (d->dim == 3)
      hipLaunchKernelGGL(k_ext_step<3>, dim3(nl), dim3(EXT_BLOCK), 0, st, *d, (const unsigned long long*)list,
                         (const int*)counter, (const double*)w[0], (const double*)w[1], w2, (const double*)q, src,
                         dst, lam);
    else
      hipLaunchKernelGGL(k_ext_step<2>, dim3(nl), dim3(EXT_BLOCK), 0, st, *d, (const unsigned long long*)list,
                         (const int*)counter, (const double*)w[0], (const double*)w[1], w2, (const double*)q, src,
                         dst, lam);
    src = dst;
    dst = (dst == work) ? q : work;
  }
  // an odd count leaves the last iterate in the work array
  if (src == work)
    hipLaunchKernelGGL(k_ext_copy, dim3(nl), dim3(EXT_BLOCK), 0, st, (const unsigned long long*)list,
                       (const int*)counter, (const double*)work, q);
  return hipGetLastError();
}

extern "C" hipError_t ebit_launch_ghost_band(const Dims* d, double jump, const uint8_t* flags,
                                             const double* const th[3], const double* nF, const double* mdot,
                                             double* const ul[3], double* const uv[3], uint8_t* bytes,
                                             double* const nb[3], int* counter, hipStream_t st) {
  const unsigned nblk = (unsigned)((d->N + EXT_BLOCK - 1) / EXT_BLOCK);
  uint8_t* A = bytes;
  uint8_t* B = bytes + d->N;
  const uint8_t* in = nullptr;
  uint8_t* out = A;
  for (int ax = 0; ax < d->dim; ++ax) {
    launch_dilate(d, ax, flags, in, out, counter, st);
    in = out;
    out = (out == A) ? B : A;
  }
  GhostBandArgs g;
  g.d = *d;
  g.jump = jump;
  g.flags = flags;
  g.band = in;
  g.nF = nF;
  g.mdot = mdot;
  for (int a = 0; a < 3; ++a) {
    g.th[a] = a < d->dim ? th[a] : nullptr;
    g.nb[a] = a < d->dim ? nb[a] : nullptr;
    g.ul[a] = a < d->dim ? ul[a] : nullptr;
    g.uv[a] = a < d->dim ? uv[a] : nullptr;
  }
  hipLaunchKernelGGL(k_ghost_band_normal, dim3(nblk), dim3(EXT_BLOCK), 0, st, g);
  hipLaunchKernelGGL(k_ghost_band, dim3(nblk), dim3(EXT_BLOCK), 0, st, g);
  return hipGetLastError();
}
