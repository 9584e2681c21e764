// EBIT marker motion (Sec. 2.1, Eqs. marker_motion and discrete_marker_motion)
// and the interfacial velocity (Sec. 2.3, Eq. jump_interfacial_vel).
//
// Interfacial velocity, per cell (2D and 3D): the cell's own phase velocity
// (the mean of its two faces per axis in that phase's face field) plus
// mdot / rho_k times the band normal (the normalised sum of the facet
// normals, vapour -> liquid, of the interface cells in the 3^d block; zero
// off the band).
//
// Marker motion (2D): an x pass, then a y pass over the same cell field.
// In the pass along axis a:
//   * every marker moves along a by u_G,a dt, u_G,a bilinear in the four
//     nearest cell centres (kept inside walls, wrapped on periodic axes); a
//     marker on a wall across a stays on it;
//   * an aligned marker (on a grid line along a) lands on the edge of its
//     line that holds its new coordinate; two landings on one edge cancel;
//     the vertices between the old and the new edge change colour;
//   * an unaligned edge (across a) holds a marker when its end vertices now
//     differ in colour, at the mean of the moved interface's crossings with
//     its line, each crossing the mean over the circles through a moved
//     segment and the far end of each neighbouring segment (the chord when
//     there is none);
//   * afterwards each cell takes its corners' colour, or for a two-marker
//     cell the side of its segment's line that the corners mark as liquid.
//
// Layout.  Each pass is three launches over flat index spaces: every edge
// of both families (the moved coordinate along a and the fixed one across
// a, NaN where no marker sits), every (aligned line, position) (one vertex
// and one edge: the flips and the landing are gathered from the four edges
// of the line that can reach them within one cell), every unaligned edge
// (the crossings are gathered from the four cells of its row that can
// reach its line).  Gathers make the result independent of thread order;
// a displacement above one cell is reported instead of being handled.
// No contraction of products into fused multiply-adds in this file: the
// landing edge and the colour tests are decided by plain IEEE products and
// sums.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {
namespace {

constexpr int ADV_BLOCK = 256;

__device__ inline long long face_index(const Dims& d, int a, int i, int j, int k) {
  const long long n0 = d.n[0] + (a == 0 ? 1 : 0);
  const long long n1 = d.n[1] + (a == 1 ? 1 : 0);
  return (long long)i + n0 * ((long long)j + n1 * k);
}

// Whether the 3^d block of (i, j, k) holds an interface cell: every flag of
// the block is loaded at once with 32-bit offsets (walls stop, periodic axes
// wrap), so the cells far from the interface (nearly all) need no ordered
// sum of normals.
template <int DIM>
__device__ inline bool block_has_iface(const Dims& d, const uint8_t* __restrict__ flags, int i, int j, int k) {
  const int p[3] = {i, j, k};
  unsigned idx[3][3];
  bool ok[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      int q = p[a] + o - 1;
      bool v = a < DIM || o == 1;
      if (a < DIM && (q < 0 || q >= d.n[a])) {
        v = d.per[a] != 0;
        q = q < 0 ? q + d.n[a] : q - d.n[a];
      }
      ok[a][o] = v;
      idx[a][o] = v ? (unsigned)q : 0u;
    }
  const unsigned n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
  uint8_t acc = 0;
#pragma unroll
  for (int oz = 0; oz < 3; ++oz)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int ox = 0; ox < 3; ++ox) {
        if (DIM == 2 && oz != 1) continue;
        if (ok[0][ox] && ok[1][oy] && ok[2][oz]) acc |= flags[idx[0][ox] + n0 * (idx[1][oy] + n1 * idx[2][oz])];
      }
  return (acc >> 7) & 1;
}

template <int DIM>
__global__ __launch_bounds__(ADV_BLOCK) void k_iface_velocity(Dims d, const uint8_t* __restrict__ flags,
                                                              const double* __restrict__ nF, const double* ul0,
                                                              const double* ul1, const double* ul2,
                                                              const double* uv0, const double* uv1,
                                                              const double* uv2, const double* __restrict__ mdot,
                                                              double rho_l, double rho_v, double* out0,
                                                              double* out1, double* out2) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const bool liquid = (flags[c] >> 6) & 1;
  double s[3] = {0.0, 0.0, 0.0};
  const bool band = block_has_iface<DIM>(d, flags, i, j, k) && band_normal_sum(d, flags, nF, i, j, k, s);
  const double L = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  const double mr = mdot[c] / (liquid ? rho_l : rho_v);
  const double* ul[3] = {ul0, ul1, ul2};
  const double* uv[3] = {uv0, uv1, uv2};
  double* out[3] = {out0, out1, out2};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double* f = liquid ? ul[a] : uv[a];
    const long long lo = face_index(d, a, i, j, k);
    const long long up = lo + (a == 0 ? 1LL : a == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1]);
    const double uc = 0.5 * (f[lo] + f[up]);
    const double n = band ? s[a] / L : 0.0;
    out[a][c] = uc + mr * n;
  }
}

// ---------------------------------------------------------------------------
// marker motion, 2D
// ---------------------------------------------------------------------------

// Error bits of a motion call.
constexpr int ADV_ERR_CFL = 1;   // a displacement above one cell, or not finite
constexpr int ADV_ERR_GEOM = 2;  // a cell with other than 0 or 2 markers, or a marker outside [0, 1]
constexpr int ADV_LIST_BLOCKS = 512;

struct Adv {
  int nx, ny;
  int per[2];
  double h, dt;
  int a;                        // pass axis
  double* mk[2];                // markers: x-edges [ny+1][nx], y-edges [ny][nx+1]
  uint8_t* vcol;                // [ny+1][nx+1]
  uint8_t* ccol;                // [ny][nx]
  const double* ug;             // cell field, component a
  double* X[2];                 // per edge: moved coordinate along a (NaN: no marker)
  double* Y[2];                 // per edge: coordinate across a (NaN: no marker)
  int* list[2];                 // marker edge ids: before the x pass, before the y pass
  int* count;                   // [2] list lengths
  int* err;
  int cur, next;                // list this pass reads; list it fills (-1: none)
};

__device__ inline long long xedge(const Adv& A, int i, int j) { return (long long)i + (long long)A.nx * j; }
__device__ inline long long yedge(const Adv& A, int i, int j) { return (long long)i + (long long)(A.nx + 1) * j; }
__device__ inline long long vtx(const Adv& A, int i, int j) { return (long long)i + (long long)(A.nx + 1) * j; }
// global edge id: the x-edges, then the y-edges
__device__ inline int xedge_id(const Adv& A, int i, int j) { return i + A.nx * j; }
__device__ inline int yedge_id(const Adv& A, int i, int j) { return A.nx * (A.ny + 1) + i + (A.nx + 1) * j; }

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Append id to a list, one atomic per wave (the wave's active lanes).
__device__ inline void append(int* list, int* count, int id, bool act) {
  const unsigned long long mask = __ballot(act);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, leader);
  if (act) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = id;
}

// Bilinear value of the cell field at (px, py): the four centres around the
// point, kept inside walls (linear extrapolation there), wrapped on
// periodic axes.
__device__ inline double bilinear(const Adv& A, const double* g, double px, double py) {
  int c0[2], c1[2];
  double f[2];
  const double P[2] = {px, py};
  const int n[2] = {A.nx, A.ny};
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    const double t = P[ax] / A.h - 0.5;
    const double fl = floor(t);
    int lo = (int)fl;
    double fr = t - fl;
    if (A.per[ax]) {
      c1[ax] = wrapi(lo + 1, n[ax]);
      c0[ax] = wrapi(lo, n[ax]);
    } else {
      if (lo < 0) {
        lo = 0;
        fr = t;
      }
      if (lo > n[ax] - 2) {
        fr = t - (double)(n[ax] - 2);
        lo = n[ax] - 2;
      }
      c0[ax] = lo;
      c1[ax] = lo + 1;
    }
    f[ax] = fr;
  }
  const double fx = f[0], fy = f[1];
  const double g00 = g[c0[0] + (long long)A.nx * c0[1]];
  const double g10 = g[c0[0] + (long long)A.nx * c1[1]];
  const double g01 = g[c1[0] + (long long)A.nx * c0[1]];
  const double g11 = g[c1[0] + (long long)A.nx * c1[1]];
  return (1.0 - fx) * (1.0 - fy) * g00 + (1.0 - fx) * fy * g10 + fx * (1.0 - fy) * g01 + fx * fy * g11;
}

// Move the marker s of edge e of family fam along a: its moved coordinate
// along a and its coordinate across a.  False (and X, Y left NaN) for a
// displacement above one cell.
__device__ inline bool move_marker(const Adv& A, int fam, long long e, double s) {
  double px, py;
  if (fam == 0) {
    const int i = (int)(e % A.nx), j = (int)(e / A.nx);
    px = ((double)i + s) * A.h;
    py = (double)j * A.h;
  } else {
    const int i = (int)(e % (A.nx + 1)), j = (int)(e / (A.nx + 1));
    px = (double)i * A.h;
    py = ((double)j + s) * A.h;
  }
  const int a = A.a;
  const double pa = a == 0 ? px : py;
  const double La = (double)(a == 0 ? A.nx : A.ny) * A.h;
  double x1 = pa;
  if (A.per[a] || (pa != 0.0 && pa != La)) {
    const double u = bilinear(A, A.ug, px, py);
    x1 = pa + u * A.dt;
    if (!(fabs(x1 - pa) <= A.h)) {
      // reported; the marker is dropped so that every later index stays
      // within one cell of where it was
      atomicOr(A.err, ADV_ERR_CFL);
      return false;
    }
  }
  A.X[fam][e] = x1;
  A.Y[fam][e] = a == 0 ? py : px;
  return true;
}

// x pass: every edge of both families; each marker is moved and listed.
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_scan(Adv A) {
  const long long E0 = (long long)A.nx * (A.ny + 1);
  const long long E1 = (long long)(A.nx + 1) * A.ny;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool listed = false;
  if (t < E0 + E1) {
    const int fam = t < E0 ? 0 : 1;
    const long long e = fam == 0 ? t : t - E0;
    const double s = A.mk[fam][e];
    if (!isnan(s)) {
      if (!(s >= 0.0 && s <= 1.0))
        atomicOr(A.err, ADV_ERR_GEOM);  // reported and dropped
      else
        listed = move_marker(A, fam, e, s);
    }
  }
  append(A.list[0], &A.count[0], (int)t, listed);
}

// y pass: the markers the x pass wrote, from its list.
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_move_list(Adv A) {
  const int T = A.count[A.cur];
  const int E0 = A.nx * (A.ny + 1);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < T; q += gridDim.x * blockDim.x) {
    const int t = A.list[A.cur][q];
    const int fam = t < E0 ? 0 : 1;
    const long long e = fam == 0 ? t : t - E0;
    move_marker(A, fam, e, A.mk[fam][e]);
  }
}

// Aligned marker at the moved coordinate x1, old edge e: its landing edge
// relative to e (unwrapped) and its fraction.
__device__ inline void landing(const Adv& A, double x1, int n, int& dk, double& s, int e) {
  const double L = (double)n * A.h;
  const int per = A.per[A.a];
  int k;
  double xh;
  if (per) {
    int shift = 0;
    double xw = x1;
    if (x1 < 0.0) {
      xw = x1 + L;
      shift = -n;
    } else if (x1 >= L) {
      xw = x1 - L;
      shift = n;
    }
    xh = xw / A.h;
    k = (int)floor(xh);
    if (k > n - 1) k = n - 1;
    s = xh - (double)k;
    k += shift;
  } else {
    const double xc = fmin(fmax(x1, 0.0), L);
    xh = xc / A.h;
    k = (int)floor(xh);
    if (k > n - 1) k = n - 1;
    s = xh - (double)k;
  }
  dk = k - e;
}

// Moved coordinate of the aligned marker on edge position e of line `line`
// (NaN: none); false beyond a wall.
__device__ inline bool aligned_x(const Adv& A, int line, int eu, int n, int& e, double& x1) {
  e = eu;
  if (A.per[A.a])
    e = wrapi(eu, n);
  else if (eu < 0 || eu >= n)
    return false;
  x1 = A.X[A.a][A.a == 0 ? xedge(A, e, line) : yedge(A, line, e)];
  return true;
}

// Aligned markers: each listed marker of the pass family at edge p of its
// line settles the positions v = p-1 .. p+2 it can reach (vertex v, edge v)
// that no marker at a smaller offset in v-2 .. v+1 settles: the vertex
// changes colour once per marker whose old and new edges lie on either side
// of it, the edge takes the one marker landing on it (none if two do).  The
// seam line of a periodic axis across a is computed from line 0, and the
// seam vertex of a periodic axis along a is written with vertex 0.
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_aligned(Adv A) {
  const int a = A.a;
  const int n = a == 0 ? A.nx : A.ny;          // edges per aligned line
  const int nb = a == 0 ? A.ny : A.nx;         // index of the last aligned line
  const int T = A.count[A.cur];
  const int E0 = A.nx * (A.ny + 1);
  // one thread per (listed marker, position offset dv = -1 .. 2)
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < 4LL * T;
       q += (long long)gridDim.x * blockDim.x) {
    const int t = A.list[A.cur][q >> 2];
    const int fam = t < E0 ? 0 : 1;
    if (fam != a) continue;
    const int e0 = fam == 0 ? t : t - E0;
    const int line = a == 0 ? e0 / A.nx : e0 % (A.nx + 1);
    const int pos = a == 0 ? e0 % A.nx : e0 / (A.nx + 1);
    const int src = (A.per[1 - a] && line == nb) ? 0 : line;
    {
      const int dv = (int)(q & 3) - 1;
      const int vu = pos + dv;
      int v = vu;
      if (A.per[a])
        v = wrapi(vu, n);
      else if (vu < 0 || vu > n)
        continue;
      // settled by the marker at the smallest offset o in -2 .. 1 from v
      bool mine = true;
      for (int o = -2; o < -dv; ++o) {
        int e;
        double x1;
        if (aligned_x(A, src, v + o, n, e, x1) && !isnan(x1)) {
          mine = false;
          break;
        }
      }
      if (!mine) continue;
      int par = 0, cnt = 0;
      double snew = NAN;
      for (int o = -2; o <= 1; ++o) {
        const int eu = v + o;
        int e;
        double x1;
        if (!aligned_x(A, src, eu, n, e, x1) || isnan(x1)) continue;
        int dk;
        double s;
        landing(A, x1, n, dk, s, e);
        const int land = eu + dk;
        if (land > eu) {
          if (eu < v && v <= land) par ^= 1;
        } else if (land < eu) {
          if (land < v && v <= eu) par ^= 1;
        }
        if (v < n && land == v) {
          ++cnt;
          snew = s;
        }
      }
      const long long vi = a == 0 ? vtx(A, v, line) : vtx(A, line, v);
      const uint8_t nc = (uint8_t)(A.vcol[vi] ^ par);
      A.vcol[vi] = nc;
      if (A.per[a] && v == 0) A.vcol[a == 0 ? vtx(A, n, line) : vtx(A, line, n)] = nc;
      bool wrote = false;
      int id = 0;
      if (v < n) {
        const double m = cnt == 1 ? snew : NAN;
        A.mk[a][a == 0 ? xedge(A, v, line) : yedge(A, line, v)] = m;
        wrote = !isnan(m);
        id = a == 0 ? xedge_id(A, v, line) : yedge_id(A, line, v);
      }
      if (A.next >= 0) append(A.list[A.next], &A.count[A.next], id, wrote);
    }
  }
}

// The up to four markers of cell (i, j), in the order bottom, top (x-edges),
// left, right (y-edges), as positions (x, y) after the moves of this pass.
__device__ inline int cell_markers(const Adv& A, int i, int j, double px[4], double py[4], int side[4]) {
  int m = 0;
  const long long e[4] = {xedge(A, i, j), xedge(A, i, j + 1), yedge(A, i, j), yedge(A, i + 1, j)};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int fam = q < 2 ? 0 : 1;
    const double xm = A.X[fam][e[q]];
    if (isnan(xm)) continue;
    if (m < 4) {
      const double ym = A.Y[fam][e[q]];
      px[m] = A.a == 0 ? xm : ym;
      py[m] = A.a == 0 ? ym : xm;
      side[m] = q;
    }
    ++m;
  }
  return m;
}

__device__ inline bool cell_has_marker(const Adv& A, int i, int j) {
  return !isnan(A.X[0][xedge(A, i, j)]) || !isnan(A.X[0][xedge(A, i, j + 1)]) || !isnan(A.X[1][yedge(A, i, j)]) ||
         !isnan(A.X[1][yedge(A, i + 1, j)]);
}

// The far end of the segment continuing cell (i, j)'s segment through its
// marker on side q (0 bottom, 1 top, 2 left, 3 right), in the cell's frame.
__device__ inline bool neighbour_end(const Adv& A, int i, int j, int q, double& qx, double& qy) {
  int di = 0, dj = 0;
  if (q == 0) dj = -1;
  else if (q == 1) dj = 1;
  else if (q == 2) di = -1;
  else di = 1;
  int in = i + di, jn = j + dj;
  double sx = 0.0, sy = 0.0;
  if (in < 0 || in >= A.nx) {
    if (!A.per[0]) return false;
    const int w = wrapi(in, A.nx);
    sx = (double)(in - w) * A.h;
    in = w;
  }
  if (jn < 0 || jn >= A.ny) {
    if (!A.per[1]) return false;
    const int w = wrapi(jn, A.ny);
    sy = (double)(jn - w) * A.h;
    jn = w;
  }
  double px[4], py[4];
  int side[4];
  if (cell_markers(A, in, jn, px, py, side) != 2) return false;
  // the shared edge is the neighbour's opposite side
  const int shared = q ^ 1;
  int far = -1, nfar = 0;
  for (int m = 0; m < 2; ++m)
    if (side[m] != shared) {
      far = m;
      ++nfar;
    }
  if (nfar != 1) return false;
  qx = px[far] + sx;
  qy = py[far] + sy;
  return true;
}

// The arc from P1 to P2 of the circle through P1, P2 and C, met with the
// line x_a = xg: the coordinate across a.  Chord frame: u along P1->P2, w
// across, w(u) = -2 k q / (1 + sqrt(1 + 4 k^2 q)), q = u (L - u); the chord
// crossing starts four Newton steps.
__device__ inline double arc_point(double ax, double ay, double bx, double by, double cx, double cy, int a,
                                   double xg) {
  const double dx = bx - ax, dy = by - ay;
  const double L = sqrt(dx * dx + dy * dy);
  const double tx = dx / L, ty = dy / L;
  const double nx = -ty, ny = tx;
  const double ex = cx - ax, ey = cy - ay;
  const double uc = ex * tx + ey * ty;
  const double wc = ex * nx + ey * ny;
  const double D = wc * wc + uc * (uc - L);
  const double k = D != 0.0 ? wc / D : 0.0;
  const double ta = a == 0 ? tx : ty;
  const double na = a == 0 ? nx : ny;
  const double Aa = a == 0 ? ax : ay;
  double u = (xg - Aa) / ta;
  u = fmin(fmax(u, 0.0), L);
  for (int it = 0; it < 4; ++it) {
    const double q = u * (L - u);
    const double S = sqrt(1.0 + 4.0 * k * k * q);
    const double w = -2.0 * k * q / (1.0 + S);
    const double dwdq = -2.0 * k / (1.0 + S) * (1.0 - 2.0 * k * k * q / (S * (1.0 + S)));
    const double f = Aa + u * ta + w * na - xg;
    const double fp = ta + dwdq * (L - 2.0 * u) * na;
    if (fp != 0.0) u = fmin(fmax(u - f / fp, 0.0), L);
  }
  const double q = u * (L - u);
  const double w = -2.0 * k * q / (1.0 + sqrt(1.0 + 4.0 * k * k * q));
  return a == 0 ? (ay + u * ty + w * ny) : (ax + u * tx + w * nx);
}

// The marker of unaligned edge (row, g) after the pass: NaN unless its end
// vertices (on aligned lines row and row + 1) now differ in colour, else the
// mean crossing of the moved segments of cells g-2 .. g+1 of its row.
__device__ inline double unaligned_marker(const Adv& A, int row, int g, int n) {
  const int a = A.a;
  const uint8_t c0 = a == 0 ? A.vcol[vtx(A, g, row)] : A.vcol[vtx(A, row, g)];
  const uint8_t c1 = a == 0 ? A.vcol[vtx(A, g, row + 1)] : A.vcol[vtx(A, row + 1, g)];
  if (c0 == c1) return NAN;
  double px[4], py[4];
  int side[4];
  double sum = 0.0;
  int cnt = 0;
#pragma unroll
  for (int o = -2; o <= 1; ++o) {
    const int iu = g + o;
    int ic = iu;
    if (A.per[a])
      ic = wrapi(iu, n);
    else if (iu < 0 || iu >= n)
      continue;
    const int ci = a == 0 ? ic : row, cj = a == 0 ? row : ic;
    if (cell_markers(A, ci, cj, px, py, side) != 2) continue;
    const double p1a = a == 0 ? px[0] : py[0], p2a = a == 0 ? px[1] : py[1];
    if (p1a == p2a) continue;
    const double lo = fmin(p1a, p2a), hi = fmax(p1a, p2a);
    const double xg = (double)(g - iu + ic) * A.h;  // the line in the cell's frame
    if (!(lo <= xg && xg <= hi)) continue;
    double q1x, q1y, q2x, q2y;
    const bool h1 = neighbour_end(A, ci, cj, side[0], q1x, q1y);
    const bool h2 = neighbour_end(A, ci, cj, side[1], q2x, q2y);
    double yb;
    if (h1 && h2) {
      const double v0 = arc_point(px[0], py[0], px[1], py[1], q1x, q1y, a, xg);
      const double v1 = arc_point(px[0], py[0], px[1], py[1], q2x, q2y, a, xg);
      yb = 0.5 * (v0 + v1);
    } else if (h1) {
      yb = arc_point(px[0], py[0], px[1], py[1], q1x, q1y, a, xg);
    } else if (h2) {
      yb = arc_point(px[0], py[0], px[1], py[1], q2x, q2y, a, xg);
    } else {
      const double p1b = a == 0 ? py[0] : px[0], p2b = a == 0 ? py[1] : px[1];
      yb = p1b + (xg - p1a) * (p2b - p1b) / (p2a - p1a);
    }
    sum += yb / A.h - (double)row;
    ++cnt;
  }
  const double sb = cnt ? sum / (double)cnt : 0.5;
  return fmin(fmax(sb, 0.0), 1.0);
}

// Unaligned markers: each listed marker settles, for each cell it borders
// whose first marker (bottom, top, left, right) it is, that cell's check
// (0 or 2 markers) and the unaligned edges g = i-1 .. i+2 of the cell's row
// (i its index along a) whose first cell with a marker in g-2 .. g+1 is
// this cell.  Every unaligned edge that can hold a marker after the pass,
// or held one before it, is such an edge.  The seam edge of a periodic axis
// along a is written with edge 0.
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_unaligned(Adv A) {
  const int a = A.a;
  const int b = 1 - a;
  const int n = a == 0 ? A.nx : A.ny;          // cells along a
  const int T = A.count[A.cur];
  const int E0 = A.nx * (A.ny + 1);
  // one thread per (listed marker, cell side, edge offset dg = -1 .. 2)
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < 8LL * T;
       q += (long long)gridDim.x * blockDim.x) {
    const int t = A.list[A.cur][q >> 3];
    const int fam = t < E0 ? 0 : 1;
    const int e0 = fam == 0 ? t : t - E0;
    int ei, ej;                                 // the edge's (i, j)
    if (fam == 0) {
      ei = e0 % A.nx;
      ej = e0 / A.nx;
    } else {
      ei = e0 % (A.nx + 1);
      ej = e0 / (A.nx + 1);
    }
    {
      const int side = (int)((q >> 2) & 1);
      // the cells this edge bounds (below / above an x-edge, left / right of a y-edge)
      int ci = ei, cj = ej;
      if (fam == 0) {
        cj = ej - 1 + side;
        if (cj < 0 || cj >= A.ny) continue;
      } else {
        ci = ei - 1 + side;
        if (ci < 0 || ci >= A.nx) continue;
      }
      // the cell's first marker must be this one
      const int ids[4] = {xedge_id(A, ci, cj), xedge_id(A, ci, cj + 1), yedge_id(A, ci, cj),
                          yedge_id(A, ci + 1, cj)};
      const double xs[4] = {A.X[0][xedge(A, ci, cj)], A.X[0][xedge(A, ci, cj + 1)], A.X[1][yedge(A, ci, cj)],
                            A.X[1][yedge(A, ci + 1, cj)]};
      int first = -1, m = 0;
      for (int k = 0; k < 4; ++k)
        if (!isnan(xs[k])) {
          if (first < 0) first = ids[k];
          ++m;
        }
      if (first != t) continue;
      const int dg = (int)(q & 3) - 1;
      if (m != 2 && dg == -1) atomicOr(A.err, ADV_ERR_GEOM);
      const int row = a == 0 ? cj : ci;
      const int ipos = a == 0 ? ci : cj;
      {
        const int gu = ipos + dg;
        int g = gu;
        if (A.per[a])
          g = wrapi(gu, n);
        else if (gu < 0 || gu > n)
          continue;
        // settled by the cell with a marker at the smallest offset in g-2 .. g+1
        bool mine = true;
        for (int o = -2; o < -dg; ++o) {
          const int iu = g + o;
          int ic = iu;
          if (A.per[a])
            ic = wrapi(iu, n);
          else if (iu < 0 || iu >= n)
            continue;
          if (a == 0 ? cell_has_marker(A, ic, row) : cell_has_marker(A, row, ic)) {
            mine = false;
            break;
          }
        }
        if (!mine) continue;
        const double mv = unaligned_marker(A, row, g, n);
        A.mk[b][a == 0 ? yedge(A, g, row) : xedge(A, row, g)] = mv;
        const bool seam = A.per[a] && g == 0;
        if (seam) A.mk[b][a == 0 ? yedge(A, n, row) : xedge(A, row, n)] = mv;
        if (A.next >= 0) {
          append(A.list[A.next], &A.count[A.next], a == 0 ? yedge_id(A, g, row) : xedge_id(A, row, g), !isnan(mv));
          append(A.list[A.next], &A.count[A.next], a == 0 ? yedge_id(A, n, row) : xedge_id(A, row, n),
                 seam && !isnan(mv));
        }
      }
    }
  }
}

// Back to the no-marker state of the coordinate arrays for a list's edges.
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_reset(Adv A, int which) {
  const int T = A.count[which];
  const int E0 = A.nx * (A.ny + 1);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < T; q += gridDim.x * blockDim.x) {
    const int t = A.list[which][q];
    const int fam = t < E0 ? 0 : 1;
    const int e = fam == 0 ? t : t - E0;
    A.X[fam][e] = NAN;
    A.Y[fam][e] = NAN;
  }
}

// Colour of cell (i, j) from the final markers and its corners.
__device__ inline void cell_colour(const Adv& A, int i, int j) {
  const double h = A.h;
  const long long e[4] = {xedge(A, i, j), xedge(A, i, j + 1), yedge(A, i, j), yedge(A, i + 1, j)};
  double x[2], y[2];
  int m = 0;
  for (int q = 0; q < 4; ++q) {
    const double s = A.mk[q < 2 ? 0 : 1][e[q]];
    if (isnan(s)) continue;
    if (m < 2) {
      if (q < 2) {
        x[m] = ((double)i + s) * h;
        y[m] = (double)(j + (q == 1)) * h;
      } else {
        x[m] = (double)(i + (q == 3)) * h;
        y[m] = ((double)j + s) * h;
      }
    }
    ++m;
  }
  const long long c = (long long)i + (long long)A.nx * j;
  const uint8_t v00 = A.vcol[vtx(A, i, j)], v10 = A.vcol[vtx(A, i + 1, j)];
  const uint8_t v01 = A.vcol[vtx(A, i, j + 1)], v11 = A.vcol[vtx(A, i + 1, j + 1)];
  if (m == 0) {
    A.ccol[c] = v00;
    return;
  }
  if (m != 2) {
    atomicOr(A.err, ADV_ERR_GEOM);
    A.ccol[c] = v00;
    return;
  }
  double nxs = -(y[1] - y[0]), nys = x[1] - x[0];
  const uint8_t cols[4] = {v00, v10, v01, v11};
  const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
  double side = 0.0;
  for (int q = 0; q < 4; ++q)
    side += (double)(2 * (int)cols[q] - 1) *
            (nxs * ((double)(i + dx[q]) * h - x[0]) + nys * ((double)(j + dy[q]) * h - y[0]));
  if (side < 0.0) {
    nxs = -nxs;
    nys = -nys;
  }
  const double centre = nxs * (((double)i + 0.5) * h - x[0]) + nys * (((double)j + 0.5) * h - y[0]);
  A.ccol[c] = centre >= 0.0 ? 1 : 0;
}

// Cell colours after both passes: the cells within 3 of a marker of either
// list (every cell whose corners or markers the step changed); a cell away
// from them keeps its colour.
constexpr int ADV_COLOUR_R = 3;
__global__ __launch_bounds__(ADV_BLOCK) void k_adv_colours(Adv A) {
  const int T0 = A.count[0], T = T0 + A.count[1];
  const int E0 = A.nx * (A.ny + 1);
  constexpr int W = 2 * ADV_COLOUR_R + 1;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < (long long)T * W * W;
       q += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(q / (W * W));
    const int w = (int)(q % (W * W));
    const int t = k < T0 ? A.list[0][k] : A.list[1][k - T0];
    const int fam = t < E0 ? 0 : 1;
    const int e0 = fam == 0 ? t : t - E0;
    int ci = fam == 0 ? e0 % A.nx : e0 % (A.nx + 1);
    int cj = fam == 0 ? e0 / A.nx : e0 / (A.nx + 1);
    ci += w % W - ADV_COLOUR_R;
    cj += w / W - ADV_COLOUR_R;
    if (ci < 0 || ci >= A.nx) {
      if (!A.per[0]) continue;
      ci = wrapi(ci, A.nx);
    }
    if (cj < 0 || cj >= A.ny) {
      if (!A.per[1]) continue;
      cj = wrapi(cj, A.ny);
    }
    cell_colour(A, ci, cj);
  }
}

__global__ void k_adv_clear(int* err, int* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *err = 0;
    count[0] = 0;
    count[1] = 0;
  }
}

unsigned blocks_for(long long n) { return (unsigned)((n + ADV_BLOCK - 1) / ADV_BLOCK); }

// Liquid volume fraction of every cell (2D; Secs. 2.2 and 3.1: the integral
// of H over the cell, from the piecewise-linear EBIT reconstruction).  The
// liquid part of a two-marker cell is the polygon of its liquid corners and
// its two markers, taken counter-clockwise round the cell from (0, 0) in
// cell units; its shoelace area is summed term by term in that order, from
// 0.0, and halved.  A cell with no marker takes its corners' colour.  A
// cell with other than 0 or 2 markers, or whose corner colours do not change
// exactly at its markers, sets the geometry error bit and gets NaN.
__global__ __launch_bounds__(ADV_BLOCK) void k_volume_fraction(int nx, int ny, const double* __restrict__ mx,
                                                               const double* __restrict__ my,
                                                               const uint8_t* __restrict__ vcol,
                                                               double* __restrict__ frac, int* err) {
  // fewer than 2^31 cells and edges: 32-bit offsets
  const unsigned t = blockIdx.x * ADV_BLOCK + threadIdx.x;
  const unsigned N = (unsigned)nx * (unsigned)ny;
  if (t >= N) return;
  const unsigned j = t / (unsigned)nx, i = t - j * (unsigned)nx;
  const unsigned nx1 = (unsigned)nx + 1;
  // corners (0,0), (1,0), (1,1), (0,1) and the edge after each: bottom,
  // right, top, left (each marker s measured from the edge's lower vertex)
  const int col[4] = {vcol[j * nx1 + i], vcol[j * nx1 + i + 1], vcol[(j + 1) * nx1 + i + 1], vcol[(j + 1) * nx1 + i]};
  const double s[4] = {mx[j * (unsigned)nx + i], my[j * nx1 + i + 1], mx[(j + 1) * (unsigned)nx + i], my[j * nx1 + i]};
  bool bad = false;
  int nm = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool has = !isnan(s[e]);
    nm += has ? 1 : 0;
    if ((col[e] != col[(e + 1) & 3]) != has) bad = true;
  }
  double f;
  if (bad || (nm != 0 && nm != 2)) {
    atomicOr(err, ADV_ERR_GEOM);
    f = NAN;
  } else if (nm == 0) {
    f = col[0] ? 1.0 : 0.0;
  } else {
    const double cx[4] = {0.0, 1.0, 1.0, 0.0}, cy[4] = {0.0, 0.0, 1.0, 1.0};
    const double px[4] = {s[0], 1.0, s[2], 0.0}, py[4] = {0.0, s[1], 1.0, s[3]};
    double fx = 0.0, fy = 0.0, lx = 0.0, ly = 0.0, acc = 0.0;
    bool first = true;
    // append a vertex: the term of the previous one and this one
    auto add = [&](double x, double y) {
      if (first) {
        fx = x;
        fy = y;
        first = false;
      } else {
        acc += lx * y - x * ly;
      }
      lx = x;
      ly = y;
    };
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (col[e]) add(cx[e], cy[e]);
      if (!isnan(s[e])) add(px[e], py[e]);
    }
    acc += lx * fy - fx * ly;
    f = 0.5 * acc;
  }
  frac[t] = f;
}

__global__ void k_vf_clear(int* err) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *err = 0;
}

}  // namespace
}  // namespace ebit

using namespace ebit;

extern "C" hipError_t ebit_launch_iface_velocity(const Dims* d, const uint8_t* flags, const double* nF,
                                                 const double* const ul[3], const double* const uv[3],
                                                 const double* mdot, double rho_l, double rho_v,
                                                 double* const out[3], hipStream_t st) {
  const unsigned nb = blocks_for(d->N);
  if (d->dim == 3)
    hipLaunchKernelGGL(k_iface_velocity<3>, dim3(nb), dim3(ADV_BLOCK), 0, st, *d, flags, nF, ul[0], ul[1], ul[2],
                       uv[0], uv[1], uv[2], mdot, rho_l, rho_v, out[0], out[1], out[2]);
  else
    hipLaunchKernelGGL(k_iface_velocity<2>, dim3(nb), dim3(ADV_BLOCK), 0, st, *d, flags, nF, ul[0], ul[1], ul[1],
                       uv[0], uv[1], uv[1], mdot, rho_l, rho_v, out[0], out[1], out[1]);
  return hipGetLastError();
}

extern "C" size_t ebit_advect_scratch_bytes(const Dims* d) {
  const long long E = (long long)d->n[0] * (d->n[1] + 1) + (long long)(d->n[0] + 1) * d->n[1];
  return (size_t)(2 * E) * sizeof(double) + (size_t)(2 * E) * sizeof(int) + 4 * sizeof(int);
}

extern "C" hipError_t ebit_launch_advect(const Dims* d, double h, double dt, const double* const ug[3],
                                         double* const mk[3], uint8_t* vcol, uint8_t* ccol, void* scratch,
                                         int init, int* err, hipStream_t st) {
  Adv A;
  A.nx = d->n[0];
  A.ny = d->n[1];
  A.per[0] = d->per[0];
  A.per[1] = d->per[1];
  A.h = h;
  A.dt = dt;
  A.mk[0] = mk[0];
  A.mk[1] = mk[1];
  A.vcol = vcol;
  A.ccol = ccol;
  A.err = err;
  const long long E0 = (long long)A.nx * (A.ny + 1), E1 = (long long)(A.nx + 1) * A.ny;
  double* xy = (double*)scratch;
  A.X[0] = xy;
  A.X[1] = xy + E0;
  A.Y[0] = xy + E0 + E1;
  A.Y[1] = xy + 2 * E0 + E1;
  int* li = (int*)(xy + 2 * (E0 + E1));
  A.list[0] = li;
  A.list[1] = li + (E0 + E1);
  A.count = li + 2 * (E0 + E1);
  // the coordinate arrays hold NaN between calls; set once per context
  if (init) {
    hipError_t e = ebit_launch_fill_f64(2 * (E0 + E1), xy, NAN, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adv_clear, dim3(1), dim3(64), 0, st, err, A.count);
  const unsigned lb = blocks_for(8 * (E0 + E1)) < (unsigned)ADV_LIST_BLOCKS ? blocks_for(8 * (E0 + E1))
                                                                             : ADV_LIST_BLOCKS;
  for (int a = 0; a < 2; ++a) {
    A.a = a;
    A.ug = ug[a];
    A.cur = a;
    A.next = a == 0 ? 1 : -1;
    if (a == 0)
      hipLaunchKernelGGL(k_adv_scan, dim3(blocks_for(E0 + E1)), dim3(ADV_BLOCK), 0, st, A);
    else
      hipLaunchKernelGGL(k_adv_move_list, dim3(lb), dim3(ADV_BLOCK), 0, st, A);
    hipLaunchKernelGGL(k_adv_aligned, dim3(lb), dim3(ADV_BLOCK), 0, st, A);
    hipLaunchKernelGGL(k_adv_unaligned, dim3(lb), dim3(ADV_BLOCK), 0, st, A);
    hipLaunchKernelGGL(k_adv_reset, dim3(lb), dim3(ADV_BLOCK), 0, st, A, a);
  }
  hipLaunchKernelGGL(k_adv_colours, dim3(lb), dim3(ADV_BLOCK), 0, st, A);
  return hipGetLastError();
}

extern "C" hipError_t ebit_launch_volume_fraction(const Dims* d, const double* const mk[3], const uint8_t* vcol,
                                                 double* frac, int* err, hipStream_t st) {
  hipLaunchKernelGGL(k_vf_clear, dim3(1), dim3(64), 0, st, err);
  if (d->N > 0)
    hipLaunchKernelGGL(k_volume_fraction, dim3(blocks_for(d->N)), dim3(ADV_BLOCK), 0, st, d->n[0], d->n[1], mk[0],
                       mk[1], vcol, frac, err);
  return hipGetLastError();
}
