// Geometric multigrid for the two interface-aware elliptic operators, and the
// FP64 outer loop (flexible preconditioned CG, or defect correction).
//
// Fine level: matrix-free (flags + sparse theta reads give every row).
// Coarse levels: 2^d box aggregation; the coarse operator keeps the summed
// mass part and half of the aggregated flux part (couplings, interface and
// wall terms), i.e. A_c = P^T M P + 1/2 P^T (A - M) P, which stays 5/7-point,
// symmetric and scales like a re-discretisation on the coarse grid.
// Smoother: red-black Gauss-Seidel.  The launched levels sweep red then black
// both before and after the coarse correction (the single-work-group tail
// sweeps black then red after it), so the V-cycle is not a symmetric
// preconditioner; the outer loop is flexible CG (Polak-Ribiere beta), which
// does not need one.
#include <cstdlib>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "ebit_internal.h"

namespace ebit {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ inline bool red_black_cell(const Dims& d, long long t, int color, int& i, int& j, int& k) {
  const int hx = (d.n[0] + 1) >> 1;
  const int ih = (int)(t % hx);
  j = (int)((t / hx) % d.n[1]);
  k = (int)(t / ((long long)hx * d.n[1]));
  if (k >= d.n[2]) return false;
  i = 2 * ih + ((j + k + color) & 1);
  return i < d.n[0];
}

__host__ inline long long half_count(const Dims& d) {
  return (long long)((d.n[0] + 1) >> 1) * d.n[1] * d.n[2];
}

template <typename T>
__global__ void k_fill(long long n, T* x, T v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

// ---------------------------------------------------------------------------
// fine level (matrix-free)
// ---------------------------------------------------------------------------
// Cells across sides s = 0 .. 2 dim - 1 of cell c = (i, j, k) (side 2a is
// the lower one along axis a, 2a + 1 the upper, as in neighbour()), wrapped
// around every axis: the neighbour() cell where there is one; across a wall
// some in-range cell, whose term the caller drops (fine_row gives a wall
// side a zero coupling).  Lets a kernel issue the neighbour loads together
// with the flag byte instead of after fine_row has read it.
__device__ inline void fine_nbrs(const Dims& d, int i, int j, int k, long long c, long long (&m)[6]) {
  const long long s1 = d.n[0], s2 = (long long)d.n[0] * d.n[1];
  m[0] = i > 0 ? c - 1 : c - 1 + d.n[0];
  m[1] = i + 1 < d.n[0] ? c + 1 : c + 1 - d.n[0];
  m[2] = j > 0 ? c - s1 : c - s1 + s2;
  m[3] = j + 1 < d.n[1] ? c + s1 : c + s1 - s2;
  m[4] = k > 0 ? c - s2 : c - s2 + d.N;
  m[5] = k + 1 < d.n[2] ? c + s2 : c + s2 - d.N;
}

template <typename T, typename TB>
__device__ inline T fine_residual_at(const FineOp& op, int i, int j, int k, long long c, const TB* b,
                                     const T* x) {
  long long m[6];
  fine_nbrs(op.d, i, j, k, c, m);
  T xn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) xn[q] = (q < 2 * op.d.dim) ? x[m[q]] : (T)0;
  const T xc = x[c];
  const T bc = (T)b[c];
  T diag, off[6], mass, rb = 0;
  fine_row<T>(op, i, j, k, op.flags[c], diag, off, mass, rb);
  T s = bc - diag * xc;
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q < 2 * op.d.dim && off[q] != (T)0) s -= off[q] * xn[q];
  return s;
}

// per-block partial sums of NV values: row q, slot lb of nb
template <int NV>
__device__ inline void write_partials(double (&v)[NV], double* partial, int lb, int nb) {
  __shared__ double sh[NV * 4];
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < NV; ++q) partial[q * nb + lb] = v[q];
}

// ---------------------------------------------------------------------------
// coarse levels (explicit symmetric coefficients)
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T coarse_offsum(const CoarseOp<T>& op, int i, int j, int k, long long c, const T* x) {
  T s = 0;
  for (int a = 0; a < op.d.dim; ++a) {
    int ni, nj, nk;
    if (neighbour(op.d, i, j, k, 2 * a + 1, ni, nj, nk)) s += op.off[a][c] * x[cell_index(op.d, ni, nj, nk)];
    if (neighbour(op.d, i, j, k, 2 * a, ni, nj, nk)) {
      const long long m = cell_index(op.d, ni, nj, nk);
      s += op.off[a][m] * x[m];
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Fused red-black Gauss-Seidel sweep: one HBM pass per full sweep.
//
// A work-group owns a TX x TY tile of an x-y plane and marches along z over
// a chunk of planes, holding four planes (tile + 2-cell ring) in LDS.  For
// each plane k it first updates the red cells of plane k+1 on the tile + 1
// ring (from the old black values), then the black cells of plane k on the
// tile (from the new red values of planes k-1, k, k+1), and writes plane k.
// Red cells on the ring are recomputed by every tile that needs them from
// the same old values, so the result equals a red half-sweep over the whole
// grid followed by a black one.  Reads x_in, writes x_out (a different
// buffer: neighbouring tiles read x_in while this one writes).  x_in may be
// null (zero initial guess) and a coarse correction xc may be added on load
// (fused prolongation).
// ---------------------------------------------------------------------------
#define RB_TX 64
#define RB_TY 4
// tile of the 2D coarse-level double sweep (the 3D z-march uses RB_TX x
// RB_TY): small tiles give a small coarse level more work-groups
#define RB_CTY 2
#define RB_CTX 32
#define RB_PX (RB_TX + 4)
#define RB_PY (RB_TY + 4)
#define RB_PLANE (RB_PX * RB_PY)
#define RB_THREADS 256

// row of an explicit coarse level
template <typename T>
struct CoarseRows {
  CoarseOp<T> op;
  const T* b;
  __device__ const Dims& dims() const { return op.d; }
  // the coupling across the upper side of axis a is stored at the cell, the
  // one across the lower side at the lower neighbour (wrapped on a periodic
  // axis); none across a wall or along an axis of one cell
  __device__ inline void row(int i, int j, int k, long long c, T& diag, T off[6], T& rhs) const {
    const Dims& d = op.d;
    const long long s1 = d.n[0], s2 = (long long)d.n[0] * d.n[1];
    const int ia[3] = {i, j, k};
    const long long st[3] = {1, s1, s2}, ln[3] = {s1, s2, d.N};
    diag = op.diag[c];
    rhs = b[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      off[2 * a] = off[2 * a + 1] = (T)0;
      if (a >= d.dim || d.n[a] < 2) continue;
      if (ia[a] + 1 < d.n[a] || d.per[a]) off[2 * a + 1] = op.off[a][c];
      if (ia[a] > 0)
        off[2 * a] = op.off[a][c - st[a]];
      else if (d.per[a])
        off[2 * a] = op.off[a][c - st[a] + ln[a]];
    }
  }
};

template <typename T, typename R>
__device__ inline void rb_load_plane(const R& rows, int kk, int tx0, int ty0, const T* __restrict__ xin,
                                     const T* __restrict__ xc, const Dims& cd, T* plane) {
  const Dims& d = rows.dims();
  int k = kk;
  bool present = true;
  if (k < 0 || k >= d.n[2]) {
    if (d.per[2] && d.dim == 3)
      k = (k % d.n[2] + d.n[2]) % d.n[2];
    else
      present = false;
  }
  for (int t = threadIdx.x; t < RB_PLANE; t += RB_THREADS) {
    const int ly = t / RB_PX - 2, lx = t % RB_PX - 2;
    int i = tx0 + lx, j = ty0 + ly;
    T v = (T)0;
    bool ok = present;
    if (ok && (i < 0 || i >= d.n[0])) {
      if (d.per[0]) i = (i % d.n[0] + d.n[0]) % d.n[0];
      else ok = false;
    }
    if (ok && (j < 0 || j >= d.n[1])) {
      if (d.per[1]) j = (j % d.n[1] + d.n[1]) % d.n[1];
      else ok = false;
    }
    if (ok) {
      const long long c = cell_index(d, i, j, k);
      if (xin) v = xin[c];
      if (xc) v += xc[cell_index(cd, i >> 1, j >> 1, k >> 1)];
    }
    plane[t] = v;
  }
}

// rb_load_plane in two halves: the loads into registers (issued a plane
// ahead of their use) and the stores into the LDS plane
#define RB_NPL ((RB_PLANE + RB_THREADS - 1) / RB_THREADS)
template <typename T, typename R>
__device__ inline void rb_issue_plane(const R& rows, int kk, int tx0, int ty0, const T* __restrict__ xin,
                                      const T* __restrict__ xc, const Dims& cd, T (&v)[RB_NPL]) {
  const Dims& d = rows.dims();
  int k = kk;
  bool present = true;
  if (k < 0 || k >= d.n[2]) {
    if (d.per[2] && d.dim == 3)
      k = (k % d.n[2] + d.n[2]) % d.n[2];
    else
      present = false;
  }
#pragma unroll
  for (int e = 0; e < RB_NPL; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    const int ly = t / RB_PX - 2, lx = t % RB_PX - 2;
    int i = tx0 + lx, j = ty0 + ly;
    T w = (T)0;
    bool ok = present && t < RB_PLANE;
    if (ok && (i < 0 || i >= d.n[0])) {
      if (d.per[0]) i = (i % d.n[0] + d.n[0]) % d.n[0];
      else ok = false;
    }
    if (ok && (j < 0 || j >= d.n[1])) {
      if (d.per[1]) j = (j % d.n[1] + d.n[1]) % d.n[1];
      else ok = false;
    }
    if (ok) {
      const long long c = cell_index(d, i, j, k);
      if (xin) w = xin[c];
      if (xc) w += xc[cell_index(cd, i >> 1, j >> 1, k >> 1)];
    }
    v[e] = w;
  }
}

template <typename T>
__device__ inline void rb_put_plane(const T (&v)[RB_NPL], T* plane) {
#pragma unroll
  for (int e = 0; e < RB_NPL; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < RB_PLANE) plane[t] = v[e];
  }
}

// update the cells of one colour of plane k on the tile (RING = 0) or on the
// tile + 1 ring (RING = 1); threads walk only the cells of the colour
template <typename T, int RING, typename R>
__device__ inline void rb_update_plane(const R& rows, int k, int tx0, int ty0, int color, T* pm, T* p0, T* pp) {
  constexpr int WX = RB_TX + 2 * RING, WY = RB_TY + 2 * RING, HX = WX / 2;
  const Dims& d = rows.dims();
  if (k < 0 || k >= d.n[2]) {
    if (!(d.per[2] && d.dim == 3)) return;
  }
  const int kw = (k % d.n[2] + d.n[2]) % d.n[2];
  for (int t = threadIdx.x; t < HX * WY; t += RB_THREADS) {
    const int ly = t / HX - RING;
    const int j = ty0 + ly;
    const int lx = 2 * (t % HX) - RING + ((color + tx0 - RING + j + k) & 1);
    const int i = tx0 + lx;
    // cells outside the domain along a non-periodic axis are not updated
    int iw = i, jw = j;
    if (iw < 0 || iw >= d.n[0]) {
      if (!d.per[0]) continue;
      iw = (iw % d.n[0] + d.n[0]) % d.n[0];
    }
    if (jw < 0 || jw >= d.n[1]) {
      if (!d.per[1]) continue;
      jw = (jw % d.n[1] + d.n[1]) % d.n[1];
    }
    const long long c = cell_index(d, iw, jw, kw);
    T diag, off[6], rhs;
    rows.row(iw, jw, kw, c, diag, off, rhs);
    const int q = (ly + 2) * RB_PX + (lx + 2);
    T sum = rhs - off[0] * p0[q - 1] - off[1] * p0[q + 1];
    if (d.dim >= 2) sum -= off[2] * p0[q - RB_PX] + off[3] * p0[q + RB_PX];
    if (d.dim == 3) sum -= off[4] * pm[q] + off[5] * pp[q];
    p0[q] = sum / diag;
  }
}

template <typename T, typename R>
__device__ inline void rb_fused_body(const R& rows, const T* __restrict__ xin, const T* __restrict__ xc,
                                     const Dims& cd, T* __restrict__ xout, int zchunk, int bx, int by, int bz,
                                     T (*buf)[RB_PLANE]) {
  const Dims& d = rows.dims();
  const int tx0 = bx * RB_TX, ty0 = by * RB_TY;
  const int z0 = bz * zchunk;
  const int z1 = min(z0 + zchunk, d.n[2]);
  const bool zdim = d.dim == 3;
  auto slot = [&](int k) { return buf[((k % 4) + 4) % 4]; };
  // plane k+2, loaded into registers during plane k-1 (3D)
  T pv[RB_NPL];
  if (zdim) {
    for (int k = z0 - 2; k <= z0 + 1; ++k) rb_load_plane<T>(rows, k, tx0, ty0, xin, xc, cd, slot(k));
    __syncthreads();
    // red on the tile + 1 ring of the two planes before the first black one
    rb_update_plane<T, 1>(rows, z0 - 1, tx0, ty0, 0, slot(z0 - 2), slot(z0 - 1),
                       slot(z0));
    __syncthreads();
    rb_update_plane<T, 1>(rows, z0, tx0, ty0, 0, slot(z0 - 1), slot(z0), slot(z0 + 1));
    rb_issue_plane<T>(rows, z0 + 2, tx0, ty0, xin, xc, cd, pv);
    __syncthreads();
  } else {
    rb_load_plane<T>(rows, 0, tx0, ty0, xin, xc, cd, buf[0]);
    __syncthreads();
    rb_update_plane<T, 1>(rows, 0, tx0, ty0, 0, buf[1], buf[0], buf[2]);
    __syncthreads();
  }
  for (int k = z0; k < z1; ++k) {
    T* p0 = zdim ? slot(k) : buf[0];
    if (zdim) {
      rb_put_plane<T>(pv, slot(k + 2));
      __syncthreads();
      if (k + 1 < z1) rb_issue_plane<T>(rows, k + 3, tx0, ty0, xin, xc, cd, pv);
      rb_update_plane<T, 1>(rows, k + 1, tx0, ty0, 0, slot(k), slot(k + 1), slot(k + 2));
      __syncthreads();
    }
    rb_update_plane<T, 0>(rows, k, tx0, ty0, 1, zdim ? slot(k - 1) : buf[1], p0,
                       zdim ? slot(k + 1) : buf[2]);
    __syncthreads();
    for (int t = threadIdx.x; t < RB_TX * RB_TY; t += RB_THREADS) {
      const int lx = t % RB_TX, ly = t / RB_TX;
      const int i = tx0 + lx, j = ty0 + ly;
      if (i < d.n[0] && j < d.n[1]) xout[cell_index(d, i, j, k)] = p0[(ly + 2) * RB_PX + (lx + 2)];
    }
    __syncthreads();
  }
}

// wrap index v along axis a; false if it lies outside a non-periodic domain
__device__ inline bool wrap_axis(const Dims& d, int a, int& v) {
  if (v >= 0 && v < d.n[a]) return true;
  if (!d.per[a]) return false;
  v = (v % d.n[a] + d.n[a]) % d.n[a];
  return true;
}

// ---------------------------------------------------------------------------
// Fine-level red-black sweep, software pipelined along z.
//
// Same ordering as k_rb_fused (red on the tile + 1 ring of plane k+1, then
// black on the tile of plane k), but the right-hand side and the flag byte
// are staged in LDS with the iterate, and the global loads of plane k+3 (x)
// and k+2 (r, flags) are issued into registers before the two updates of
// plane k, so their latency is hidden behind LDS work.  2D grids are one
// plane: x, r and flags of the tile are loaded in a single phase.
// ---------------------------------------------------------------------------
template <int TX, int TY>
struct FineTile {
  static constexpr int PX = TX + 4, PY = TY + 4, PL = PX * PY;  // iterate: tile + 2-cell ring
  static constexpr int QX = TX + 2, QY = TY + 2, QL = QX * QY;  // r, flags: tile + 1-cell ring
  static constexpr int NX = (PL + RB_THREADS - 1) / RB_THREADS;
  static constexpr int NQ = (QL + RB_THREADS - 1) / RB_THREADS;
};

template <typename T, int TX, int TY>
struct FineGeom;

// Plane-invariant part of one thread's work in a fine sweep: which cells of
// the staged windows it loads (their in-plane offsets, -1 outside the domain
// or the window) and which cells it updates in each phase, for both colour
// parities of a plane (the parity alternates with k).  Computed once per
// work-group; the z-march then only adds plane offsets.
template <int TX, int TY>
struct FineSlots {
  using FT = FineTile<TX, TY>;
  static constexpr int HR = (TX + 2) / 2, NR = (HR * (TY + 2) + RB_THREADS - 1) / RB_THREADS;  // red, tile + ring
  static constexpr int HB = TX / 2, NB = (HB * TY + RB_THREADS - 1) / RB_THREADS;              // black, tile
  static constexpr int NW = (TX * TY + RB_THREADS - 1) / RB_THREADS;                           // write-back
  int xo[FT::NX], xco[FT::NX];  // iterate window: cell offset i + n0 j, parent offset on the coarse level
  int qo[FT::NQ];               // r / flags window
  // update slots: q (P = 0; P = 1 is q + 1), qq = q - dq, wrapped i for
  // both parities, wrapped j, parity base, bits: 1 ok(P=0), 2 ok(P=1),
  // 4 x-wall(P=0), 8 x-wall(P=1), 16 y-wall
  int rq[NR], rdq[NR], ri0[NR], ri1[NR], rj[NR], rp[NR], rbits[NR];
  int bq[NB], bdq[NB], bi0[NB], bi1[NB], bj[NB], bp[NB], bbits[NB];
  int wo[NW], wq[NW];
};

template <int TX, int TY, int RING, int NS>
__device__ inline void slot_setup(const Dims& d, int tx0, int ty0, int color, int (&q)[NS], int (&dq)[NS],
                                  int (&i0)[NS], int (&i1)[NS], int (&jj)[NS], int (&pb)[NS], int (&bits)[NS]) {
  using FT = FineTile<TX, TY>;
  constexpr int HX = (TX + 2 * RING) / 2, WY = TY + 2 * RING;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int t = threadIdx.x + s * RB_THREADS;
    bits[s] = 0;
    q[s] = dq[s] = i0[s] = i1[s] = jj[s] = pb[s] = 0;
    if (t >= HX * WY) continue;
    const int ly = t / HX - RING, m = t % HX;
    int j = ty0 + ly;
    pb[s] = (color + tx0 - RING + j) & 1;
    const int lx0 = 2 * m - RING;
    q[s] = (ly + 2) * FT::PX + (lx0 + 2);
    dq[s] = FT::PX + 3 + 2 * ly;
    const bool okj = wrap_axis(d, 1, j);
    jj[s] = j;
    int a = tx0 + lx0, b = tx0 + lx0 + 1;
    const bool oka = okj && wrap_axis(d, 0, a);
    const bool okb = okj && wrap_axis(d, 0, b);
    i0[s] = a;
    i1[s] = b;
    int bt = (oka ? 1 : 0) | (okb ? 2 : 0);
    if (!d.per[0] && (a == 0 || a == d.n[0] - 1)) bt |= 4;
    if (!d.per[0] && (b == 0 || b == d.n[0] - 1)) bt |= 8;
    if (!d.per[1] && (j == 0 || j == d.n[1] - 1)) bt |= 16;
    bits[s] = bt;
  }
}

template <int TX, int TY>
__device__ inline void fine_slots(const Dims& d, const Dims& cd, int tx0, int ty0, FineSlots<TX, TY>& S) {
  using FT = FineTile<TX, TY>;
  using FS = FineSlots<TX, TY>;
#pragma unroll
  for (int e = 0; e < FT::NX; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    S.xo[e] = -1;
    S.xco[e] = 0;
    if (t >= FT::PL) continue;
    int i = tx0 + t % FT::PX - 2, j = ty0 + t / FT::PX - 2;
    if (wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
      S.xo[e] = i + d.n[0] * j;
      S.xco[e] = (i >> 1) + cd.n[0] * (j >> 1);
    }
  }
#pragma unroll
  for (int e = 0; e < FT::NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    S.qo[e] = -1;
    if (t >= FT::QL) continue;
    int i = tx0 + t % FT::QX - 1, j = ty0 + t / FT::QX - 1;
    if (wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) S.qo[e] = i + d.n[0] * j;
  }
  slot_setup<TX, TY, 1, FS::NR>(d, tx0, ty0, 0, S.rq, S.rdq, S.ri0, S.ri1, S.rj, S.rp, S.rbits);
  slot_setup<TX, TY, 0, FS::NB>(d, tx0, ty0, 1, S.bq, S.bdq, S.bi0, S.bi1, S.bj, S.bp, S.bbits);
#pragma unroll
  for (int e = 0; e < FS::NW; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    const int lx = t % TX, ly = t / TX;
    const int i = tx0 + lx, j = ty0 + ly;
    S.wo[e] = (t < TX * TY && i < d.n[0] && j < d.n[1]) ? i + d.n[0] * j : -1;
    S.wq[e] = (ly + 2) * FT::PX + (lx + 2);
  }
}

// iterate window of plane kk into registers (x_in + coarse correction)
template <typename T, int TX, int TY>
__device__ inline void fine_load_x(const Dims& d, const Dims& cd, const FineSlots<TX, TY>& S, int kk,
                                   const T* __restrict__ xin, const T* __restrict__ xc, T (&v)[FineTile<TX, TY>::NX]) {
  using FT = FineTile<TX, TY>;
  int k = kk;
  const bool pz = wrap_axis(d, 2, k) && (xin || xc);
  const long long base = (long long)k * d.n[0] * d.n[1];
  const long long cbase = (long long)(k >> 1) * cd.n[0] * cd.n[1];
#pragma unroll
  for (int e = 0; e < FT::NX; ++e) {
    T s = (T)0;
    if (pz && S.xo[e] >= 0) {
      if (xin) s = xin[base + S.xo[e]];
      if (xc) s += xc[cbase + S.xco[e]];
    }
    v[e] = s;
  }
}

template <typename T, int TX, int TY>
__device__ inline void fine_load_rf(const Dims& d, const FineSlots<TX, TY>& S, int kk, const T* __restrict__ rhs,
                                    const uint8_t* __restrict__ flags, T (&r)[FineTile<TX, TY>::NQ],
                                    uint8_t (&f)[FineTile<TX, TY>::NQ]) {
  using FT = FineTile<TX, TY>;
  int k = kk;
  const bool pz = wrap_axis(d, 2, k);
  const long long base = (long long)k * d.n[0] * d.n[1];
#pragma unroll
  for (int e = 0; e < FT::NQ; ++e) {
    r[e] = (T)0;
    f[e] = 0;
    if (pz && S.qo[e] >= 0) {
      r[e] = rhs[base + S.qo[e]];
      f[e] = flags[base + S.qo[e]];
    }
  }
}

template <typename T, int TX, int TY>
__device__ inline void fine_store(const T (&v)[FineTile<TX, TY>::NX], T* xs) {
  using FT = FineTile<TX, TY>;
#pragma unroll
  for (int e = 0; e < FT::NX; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < FT::PL) xs[t] = v[e];
  }
}

template <typename T, int TX, int TY>
__device__ inline void fine_store_rf(const T (&r)[FineTile<TX, TY>::NQ], const uint8_t (&f)[FineTile<TX, TY>::NQ],
                                     T* rs, uint8_t* fs) {
  using FT = FineTile<TX, TY>;
#pragma unroll
  for (int e = 0; e < FT::NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < FT::QL) {
      rs[t] = r[e];
      fs[t] = f[e];
    }
  }
}

// Coefficients of a regular fine cell (no cut link, no wall face) of each
// phase: A x = dg x_c - w sum_nb x_nb.
template <typename T>
struct RegularRow {
  T w0, w1, inv0, inv1;  // per phase (0 vapour, 1 liquid)
  T dg0, dg1;            // the diagonal dg of each phase
};

template <typename T>
__device__ inline RegularRow<T> regular_row(const FineOp& op) {
  const T ih2 = (T)op.ih2;
  T w[2], inv[2], dgs[2];
  for (int ph = 0; ph < 2; ++ph) {
    w[ph] = (T)op.coef[ph] * ih2;
    T dg = (op.sys == EBIT_SYS_HEAT) ? (T)op.mass[ph] : (T)0;
    for (int s = 0; s < 2 * op.d.dim; ++s) dg += w[ph];
    dgs[ph] = dg;
    inv[ph] = (T)1 / dg;
  }
  return RegularRow<T>{w[0], w[1], inv[0], inv[1], dgs[0], dgs[1]};
}

// Update this thread's cells of one colour of plane k (slots from
// FineSlots) from LDS.  Regular cells take the per-phase constant row,
// cells with a cut link or a wall face the full row of fine_row.
template <typename T, int TX, int TY, int NS>
__device__ inline void fine_update(const FineOp& op, const RegularRow<T>& rr, int k, const int (&q0)[NS],
                                   const int (&dq)[NS], const int (&i0)[NS], const int (&i1)[NS], const int (&jj)[NS],
                                   const int (&pb)[NS], const int (&bits)[NS], const T* pm, T* p0, const T* pp,
                                   const T* rq, const uint8_t* fq) {
  using FT = FineTile<TX, TY>;
  const Dims& d = op.d;
  int kw = k;
  if (!wrap_axis(d, 2, kw)) return;
  const bool zwall = d.dim == 3 && !d.per[2] && (kw == 0 || kw == d.n[2] - 1);
  const int kp = k & 1;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int P = pb[s] ^ kp;
    const int bt = bits[s];
    if (!(bt & (P ? 2 : 1))) continue;
    const int q = q0[s] + P;
    const int qq = q - dq[s];
    const uint8_t f = fq[qq];
    const bool wall = zwall || (bt & (P ? 8 : 4)) || (bt & 16);
    if (!(f & F_CUT) && !wall) {
      const bool liq = (f & F_LIQ) != 0;
      T xn = (p0[q - 1] + p0[q + 1]) + (p0[q - FT::PX] + p0[q + FT::PX]);
      if (d.dim == 3) xn += pm[q] + pp[q];
      p0[q] = ((T)rq[qq] + (liq ? rr.w1 : rr.w0) * xn) * (liq ? rr.inv1 : rr.inv0);
    } else {
      T diag, off[6], mass, rb = 0;
      fine_row<T>(op, P ? i1[s] : i0[s], jj[s], kw, f, diag, off, mass, rb);
      T sum = (T)rq[qq] - off[0] * p0[q - 1] - off[1] * p0[q + 1];
      sum -= off[2] * p0[q - FT::PX] + off[3] * p0[q + FT::PX];
      if (d.dim == 3) sum -= off[4] * pm[q] + off[5] * pp[q];
      p0[q] = sum / diag;
    }
  }
}

template <typename T, int TX, int TY>
__device__ inline void fine_write(const Dims& d, const FineSlots<TX, TY>& S, int k, const T* p0, T* __restrict__ xout) {
  using FS = FineSlots<TX, TY>;
  const long long base = (long long)k * d.n[0] * d.n[1];
#pragma unroll
  for (int e = 0; e < FS::NW; ++e)
    if (S.wo[e] >= 0) xout[base + S.wo[e]] = p0[S.wq[e]];
}

#define FINE_RED(K, PM, P0, PP, RS, FS_)                                                                          \
  fine_update<T, TX, TY, FS::NR>(op, rr, (K), S.rq, S.rdq, S.ri0, S.ri1, S.rj, S.rp, S.rbits, (PM), (P0), (PP), \
                                 (RS), (FS_))
#define FINE_BLACK(K, PM, P0, PP, RS, FS_)                                                                        \
  fine_update<T, TX, TY, FS::NB>(op, rr, (K), S.bq, S.bdq, S.bi0, S.bi1, S.bj, S.bp, S.bbits, (PM), (P0), (PP), \
                                 (RS), (FS_))

template <typename T, int TX, int TY>
__device__ inline void rb_fine_body(const FineOp& op, const T* __restrict__ rhs, const T* __restrict__ xin,
                                    const T* __restrict__ xc, const Dims& cd, T* __restrict__ xout, int zchunk,
                                    int bx, int by, int bz, T (*xs)[FineTile<TX, TY>::PL],
                                    T (*rs)[FineTile<TX, TY>::QL], uint8_t (*fs)[FineTile<TX, TY>::QL]) {
  using FT = FineTile<TX, TY>;
  using FS = FineSlots<TX, TY>;
  const Dims& d = op.d;
  const RegularRow<T> rr = regular_row<T>(op);
  const int tx0 = bx * TX, ty0 = by * TY;
  FS S;
  fine_slots<TX, TY>(d, cd, tx0, ty0, S);
  T xv[FT::NX];
  T rv[FT::NQ];
  uint8_t fv[FT::NQ];
  if (d.dim < 3) {
    fine_load_x<T, TX, TY>(d, cd, S, 0, xin, xc, xv);
    fine_load_rf<T, TX, TY>(d, S, 0, rhs, op.flags, rv, fv);
    fine_store<T, TX, TY>(xv, xs[0]);
    fine_store_rf<T, TX, TY>(rv, fv, rs[0], fs[0]);
    __syncthreads();
    FINE_RED(0, xs[0], xs[0], xs[0], rs[0], fs[0]);
    __syncthreads();
    FINE_BLACK(0, xs[0], xs[0], xs[0], rs[0], fs[0]);
    __syncthreads();
    fine_write<T, TX, TY>(d, S, 0, xs[0], xout);
    return;
  }
  // slots: x plane p in xs[p & 3], r / flags of plane p in rs[p & 1] (p may be negative)
  const int z0 = bz * zchunk;
  const int z1 = min(z0 + zchunk, d.n[2]);
  {
    T xa[FT::NX], xb[FT::NX];
    T ra[FT::NQ];
    uint8_t fa[FT::NQ];
    fine_load_x<T, TX, TY>(d, cd, S, z0 - 2, xin, xc, xv);
    fine_load_x<T, TX, TY>(d, cd, S, z0 - 1, xin, xc, xa);
    fine_load_x<T, TX, TY>(d, cd, S, z0, xin, xc, xb);
    fine_load_rf<T, TX, TY>(d, S, z0 - 1, rhs, op.flags, rv, fv);
    fine_load_rf<T, TX, TY>(d, S, z0, rhs, op.flags, ra, fa);
    fine_store<T, TX, TY>(xv, xs[(z0 - 2) & 3]);
    fine_store<T, TX, TY>(xa, xs[(z0 - 1) & 3]);
    fine_store<T, TX, TY>(xb, xs[z0 & 3]);
    fine_store_rf<T, TX, TY>(rv, fv, rs[(z0 - 1) & 1], fs[(z0 - 1) & 1]);
    fine_store_rf<T, TX, TY>(ra, fa, rs[z0 & 1], fs[z0 & 1]);
    fine_load_x<T, TX, TY>(d, cd, S, z0 + 1, xin, xc, xv);
    fine_store<T, TX, TY>(xv, xs[(z0 + 1) & 3]);
  }
  __syncthreads();
  FINE_RED(z0 - 1, xs[(z0 - 2) & 3], xs[(z0 - 1) & 3], xs[z0 & 3], rs[(z0 - 1) & 1], fs[(z0 - 1) & 1]);
  __syncthreads();
  FINE_RED(z0, xs[(z0 - 1) & 3], xs[z0 & 3], xs[(z0 + 1) & 3], rs[z0 & 1], fs[z0 & 1]);
  fine_load_x<T, TX, TY>(d, cd, S, z0 + 2, xin, xc, xv);
  fine_load_rf<T, TX, TY>(d, S, z0 + 1, rhs, op.flags, rv, fv);
  __syncthreads();
  for (int k = z0; k < z1; ++k) {
    // plane k+2's iterate replaces plane k-2's, plane k+1's r / flags replace plane k-1's
    fine_store<T, TX, TY>(xv, xs[(k + 2) & 3]);
    fine_store_rf<T, TX, TY>(rv, fv, rs[(k + 1) & 1], fs[(k + 1) & 1]);
    __syncthreads();
    if (k + 1 < z1) {
      fine_load_x<T, TX, TY>(d, cd, S, k + 3, xin, xc, xv);
      fine_load_rf<T, TX, TY>(d, S, k + 2, rhs, op.flags, rv, fv);
    }
    FINE_RED(k + 1, xs[k & 3], xs[(k + 1) & 3], xs[(k + 2) & 3], rs[(k + 1) & 1], fs[(k + 1) & 1]);
    __syncthreads();
    FINE_BLACK(k, xs[(k - 1) & 3], xs[k & 3], xs[(k + 1) & 3], rs[k & 1], fs[k & 1]);
    __syncthreads();
    fine_write<T, TX, TY>(d, S, k, xs[k & 3], xout);
  }
}
#undef FINE_RED
#undef FINE_BLACK

// ---------------------------------------------------------------------------
// 2D sweeps, NSW full red-black sweeps per launch.  A work-group stages its
// tile with a ring of 2 NSW cells (iterate) and 2 NSW - 1 cells (the other
// arrays), then runs 2 NSW colour phases on windows that shrink by one
// cell each: the ring cells are recomputed from the same old values by
// every tile that needs them, so the tile ends exactly as after NSW
// whole-grid sweeps.  One launch and one global-memory wait instead of NSW.
// ---------------------------------------------------------------------------
template <int TX, int TY, int NSW, int E = 0>
struct Win2 {
  static constexpr int H = 2 * NSW + E, QR = 2 * NSW - 1 + E;
  static constexpr int PX = TX + 2 * H, PY = TY + 2 * H, PL = PX * PY;
  static constexpr int QX = TX + 2 * QR, QY = TY + 2 * QR, QL = QX * QY;
};

// one colour phase on the window [-ring, T+ring); cells outside a
// non-periodic domain are not updated; upd(q, qq, iw, jw) does the cell
template <int TX, int TY, int NSW, int E, int RING, typename U>
__device__ inline void phase2(const Dims& d, int tx0, int ty0, int color, const U& upd) {
  using W = Win2<TX, TY, NSW, E>;
  constexpr int HX = (TX + 2 * RING) / 2, WY = TY + 2 * RING;
  for (int t = threadIdx.x; t < HX * WY; t += RB_THREADS) {
    const int ly = t / HX - RING;
    const int j = ty0 + ly;
    const int lx = 2 * (t % HX) - RING + ((color + tx0 - RING + j) & 1);
    int iw = tx0 + lx, jw = j;
    if (!wrap_axis(d, 0, iw) || !wrap_axis(d, 1, jw)) continue;
    upd((ly + W::H) * W::PX + (lx + W::H), (ly + W::QR) * W::QX + (lx + W::QR), iw, jw);
  }
}

template <int TX, int TY, int NSW, int E, int P, typename U>
__device__ inline void phases2(const Dims& d, int tx0, int ty0, const U& upd) {
  if constexpr (P < 2 * NSW) {
    phase2<TX, TY, NSW, E, 2 * NSW - 1 - P + E>(d, tx0, ty0, P & 1, upd);
    __syncthreads();
    phases2<TX, TY, NSW, E, P + 1>(d, tx0, ty0, upd);
  }
}

// Restriction fused into a tile's last pre-smoothing launch (2D): the
// window then carries one more ring, so the last (black) phase also covers
// ring 1 and the residual of every red cell of the tile is exact in LDS.
// Tiles start at even coordinates, so the red children (0,0) and (1,1) of
// each coarse cell of the tile lie in it; res(q, qq, i, j) gives a child's
// residual from the window.
template <typename T, int TX, int TY, int E, typename R>
__device__ inline void restrict2(const Dims& d, const Dims& cd, int tx0, int ty0, int H, int PX, int QR, int QX,
                                 T* __restrict__ bc, T* __restrict__ xcz, int split, const R& res) {
  const long long chs = tail_half(cd);
  constexpr int CX = TX / 2, CY = TY / 2;
  for (int t = threadIdx.x; t < CX * CY; t += RB_THREADS) {
    const int ci = tx0 / 2 + t % CX, cj = ty0 / 2 + t / CX;
    if (ci >= cd.n[0] || cj >= cd.n[1]) continue;
    T sum = 0;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const int i = 2 * ci + ch, j = 2 * cj + ch;
      if (i < d.n[0] && j < d.n[1]) {
        const int lx = i - tx0, ly = j - ty0;
        sum += res((ly + H) * PX + (lx + H), (ly + QR) * QX + (lx + QR), i, j);
      }
    }
    const long long I = ci + (long long)cd.n[0] * cj;
    bc[split ? tail_el(cd, chs, ci, cj, 0) : I] = sum;
    xcz[I] = (T)0;
  }
}

// fine level, 2D
template <typename T, int TX, int TY, int NSW, int RES>
__device__ inline void rb_fine2d_body(const FineOp& op, const T* __restrict__ rhs, const T* __restrict__ xin,
                                      const T* __restrict__ xc, const Dims& cd, T* __restrict__ xout, int bx, int by,
                                      T* xs, T* rs, uint8_t* fs, T* __restrict__ bc, T* __restrict__ xcz,
                                      int split, int dots = 0, const double* __restrict__ qv = nullptr,
                                      double* __restrict__ partial = nullptr, int slot = 0, int nslot = 0,
                                      const double* __restrict__ r64 = nullptr) {
  using W = Win2<TX, TY, NSW, RES>;
  const Dims& d = op.d;
  const RegularRow<T> rr = regular_row<T>(op);
  const int tx0 = bx * TX, ty0 = by * TY;
  constexpr int NP = (W::PL + RB_THREADS - 1) / RB_THREADS, NQ = (W::QL + RB_THREADS - 1) / RB_THREADS;
  T vx[NP];
  T vr[NQ];
  uint8_t vf[NQ];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    vx[e] = (T)0;
    int i = tx0 + t % W::PX - W::H, j = ty0 + t / W::PX - W::H;
    if (t < W::PL && (xin || xc) && wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
      if (xin) vx[e] = xin[i + (long long)d.n[0] * j];
      if (xc) vx[e] += xc[(i >> 1) + (long long)cd.n[0] * (j >> 1)];
    }
  }
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    vr[e] = (T)0;
    vf[e] = 0;
    int i = tx0 + t % W::QX - W::QR, j = ty0 + t / W::QX - W::QR;
    if (t < W::QL && wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
      const long long c = i + (long long)d.n[0] * j;
      vr[e] = rhs[c];
      vf[e] = op.flags[c];
    }
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < W::PL) xs[t] = vx[e];
  }
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < W::QL) {
      rs[t] = vr[e];
      fs[t] = vf[e];
    }
  }
  __syncthreads();
  auto upd = [&](int q, int qq, int iw, int jw) {
    const uint8_t f = fs[qq];
    const bool wall = (!d.per[0] && (iw == 0 || iw == d.n[0] - 1)) || (!d.per[1] && (jw == 0 || jw == d.n[1] - 1));
    if (!(f & F_CUT) && !wall) {
      const bool liq = (f & F_LIQ) != 0;
      const T xn = (xs[q - 1] + xs[q + 1]) + (xs[q - W::PX] + xs[q + W::PX]);
      xs[q] = ((T)rs[qq] + (liq ? rr.w1 : rr.w0) * xn) * (liq ? rr.inv1 : rr.inv0);
    } else {
      T diag, off[6], mass, rb = 0;
      fine_row<T>(op, iw, jw, 0, f, diag, off, mass, rb);
      T sum = (T)rs[qq] - off[0] * xs[q - 1] - off[1] * xs[q + 1];
      sum -= off[2] * xs[q - W::PX] + off[3] * xs[q + W::PX];
      xs[q] = sum / diag;
    }
  };
  phases2<TX, TY, NSW, RES, 0>(d, tx0, ty0, upd);
  for (int t = threadIdx.x; t < TX * TY; t += RB_THREADS) {
    const int lx = t % TX, ly = t / TX;
    const int i = tx0 + lx, j = ty0 + ly;
    if (i < d.n[0] && j < d.n[1]) xout[i + (long long)d.n[0] * j] = xs[(ly + W::H) * W::PX + (lx + W::H)];
  }
  if constexpr (RES) {
    // the fine residual r - A x of a child, as fine_residual_at forms it
    auto res = [&](int q, int qq, int i, int j) {
      T diag, off[6], mass, rb = 0;
      fine_row<T>(op, i, j, 0, fs[qq], diag, off, mass, rb);
      const T xn[4] = {xs[q - 1], xs[q + 1], xs[q - W::PX], xs[q + W::PX]};
      T s = (T)rs[qq] - diag * xs[q];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (off[a] != (T)0) s -= off[a] * xn[a];
      return s;
    };
    restrict2<T, TX, TY, RES>(d, cd, tx0, ty0, W::H, W::PX, W::QR, W::QX, bc, xcz, split, res);
  }
  if (dots) {
    // the outer loop's z.r and (dots == 1) z.q over this tile, from the
    // final iterate and the FP64 r (in LDS when the sweep smooths against
    // it, else read here): one partial per tile
    double v[2] = {0, 0};
    for (int t = threadIdx.x; t < TX * TY; t += RB_THREADS) {
      const int lx = t % TX, ly = t / TX;
      const int i = tx0 + lx, j = ty0 + ly;
      if (i < d.n[0] && j < d.n[1]) {
        const double zc = (double)xs[(ly + W::H) * W::PX + (lx + W::H)];
        if constexpr (std::is_same<T, double>::value)
          v[0] += zc * rs[(ly + W::QR) * W::QX + (lx + W::QR)];
        else
          v[0] += zc * r64[i + (long long)d.n[0] * j];
        if (dots == 1) v[1] += zc * qv[i + (long long)d.n[0] * j];
      }
    }
    write_partials<2>(v, partial, slot, nslot);
  }
}

// explicit coarse level, 2D (couplings staged on the iterate's window: a
// ring cell's lower couplings sit one cell further out)
template <typename T, int NSW, int RES>
__device__ inline void rb_coarse2d_body(const CoarseOp<T>& op, const T* __restrict__ b, const T* __restrict__ xin,
                                        const T* __restrict__ xc, const Dims& cd, T* __restrict__ xout, int bx, int by,
                                        T* sb, T* __restrict__ bc, T* __restrict__ xcz, int split) {
  using W = Win2<RB_CTX, RB_CTY, NSW, RES>;
  const Dims& d = op.d;
  T* xs = sb;
  T* o0 = sb + W::PL;
  T* o1 = sb + 2 * W::PL;
  T* dg = sb + 3 * W::PL;
  T* bb = dg + W::QL;
  const int tx0 = bx * RB_CTX, ty0 = by * RB_CTY;
  constexpr int NP = (W::PL + RB_THREADS - 1) / RB_THREADS, NQ = (W::QL + RB_THREADS - 1) / RB_THREADS;
  T vx[NP], v0[NP], v1[NP], vd[NQ], vb[NQ];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    vx[e] = v0[e] = v1[e] = (T)0;
    int i = tx0 + t % W::PX - W::H, j = ty0 + t / W::PX - W::H;
    if (t < W::PL && wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
      const long long c = i + (long long)d.n[0] * j;
      if (xin) vx[e] = xin[c];
      if (xc) vx[e] += xc[(i >> 1) + (long long)cd.n[0] * (j >> 1)];
      v0[e] = op.off[0][c];
      v1[e] = op.off[1][c];
    }
  }
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    vd[e] = (T)1;
    vb[e] = (T)0;
    int i = tx0 + t % W::QX - W::QR, j = ty0 + t / W::QX - W::QR;
    if (t < W::QL && wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
      const long long c = i + (long long)d.n[0] * j;
      vd[e] = op.diag[c];
      vb[e] = b[c];
    }
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < W::PL) {
      xs[t] = vx[e];
      o0[t] = v0[e];
      o1[t] = v1[e];
    }
  }
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < W::QL) {
      dg[t] = vd[e];
      bb[t] = vb[e];
    }
  }
  __syncthreads();
  auto upd = [&](int q, int qc, int, int) {
    const T sum = bb[qc] - o0[q - 1] * xs[q - 1] - o0[q] * xs[q + 1] -
                  (o1[q - W::PX] * xs[q - W::PX] + o1[q] * xs[q + W::PX]);
    xs[q] = sum / dg[qc];
  };
  phases2<RB_CTX, RB_CTY, NSW, RES, 0>(d, tx0, ty0, upd);
  for (int t = threadIdx.x; t < RB_CTX * RB_CTY; t += RB_THREADS) {
    const int lx = t % RB_CTX, ly = t / RB_CTX;
    const int i = tx0 + lx, j = ty0 + ly;
    if (i < d.n[0] && j < d.n[1]) xout[i + (long long)d.n[0] * j] = xs[(ly + W::H) * W::PX + (lx + W::H)];
  }
  if constexpr (RES) {
    // b - diag x - couplings, in the order of coarse_offsum (a window cell
    // outside a wall holds a zero iterate and couplings, so its term is zero)
    auto res = [&](int q, int qc, int, int) {
      T s = 0;
      s += o0[q] * xs[q + 1];
      s += o0[q - 1] * xs[q - 1];
      s += o1[q] * xs[q + W::PX];
      s += o1[q - W::PX] * xs[q - W::PX];
      return bb[qc] - dg[qc] * xs[q] - s;
    };
    restrict2<T, RB_CTX, RB_CTY, RES>(d, cd, tx0, ty0, W::H, W::PX, W::QR, W::QX, bc, xcz, split, res);
  }
}

// shared buffer of the coarse sweep kernel: the 3D z-march's four planes or
// the 2D double sweep's staged windows
constexpr int RB_SBUF = (3 * Win2<RB_CTX, RB_CTY, 2, 1>::PL + 2 * Win2<RB_CTX, RB_CTY, 2, 1>::QL) > 4 * RB_PLANE
                            ? (3 * Win2<RB_CTX, RB_CTY, 2, 1>::PL + 2 * Win2<RB_CTX, RB_CTY, 2, 1>::QL)
                            : 4 * RB_PLANE;

// Children (di, dj, dk) of a coarse cell whose fine cell has colour 0
// ((i + j + k) even): (0,0,0), (1,1,0), then in 3D (1,0,1), (0,1,1).  Every
// pre-smoothing sweep ends with colour 1, whose residual then vanishes up
// to rounding (a Gauss-Seidel update zeroes its cell's residual and no
// later update touches a neighbour of it), so the restricted residual is
// the sum over these children alone.
__device__ inline void even_child(int ch, int& di, int& dj, int& dk) {
  di = (ch == 1 || ch == 2) ? 1 : 0;
  dj = (ch == 1 || ch == 3) ? 1 : 0;
  dk = ch >= 2 ? 1 : 0;
}

// ---------------------------------------------------------------------------
// tail of the V-cycle: every level small enough to sit in LDS, in one
// work-group (no launch per smoothing sweep on the coarse levels).  The
// hierarchy build leaves the coefficients of these levels and the dense
// coarsest inverse in one contiguous image per system, laid out as the
// kernel's LDS: the kernel starts with a straight 16-byte copy of the
// suffix it needs.
//
// Layout of a tail level: every field (diag, 1/diag, couplings off[a], the
// iterate x, the right-hand side b) keeps the cells of colour 0 (i + j + k
// even) in its first half and those of colour 1 in its second, each half
// in row order with the cells (i, j, k) of a grid row at slots i >> 1:
// element colour * hs + (i >> 1) + hw (j + n1 k), hw = (n0 + 1) / 2.  A
// colour sweep then reads its own cells and its neighbours at consecutive
// addresses across a wavefront (no LDS bank conflicts).
// ---------------------------------------------------------------------------
#define EBIT_TAIL_MAX 16
#define EBIT_TAIL_THREADS 1024
#define TAIL_COPY_BATCH 8
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One tail level in LDS: field f (0 diag, 1 1/diag, 2 + a off[a]) at
// cb + 2 f hs, x at xb and b at bb.  The iterates of all levels form one
// region, [L[0].xb, L[0].bb), the right-hand sides the next.
struct TailLevel {
  Dims d;
  int hs;  // colour half length (hw rows, padded to four)
  int cb;
  int xb;
  int bb;
};

template <typename T>
struct TailArgs {
  int nl;  // levels in the tail; the last one is the coarsest
  int nu1, nu2;
  TailLevel L[EBIT_TAIL_MAX];
  const T* img;        // coefficient image from the top tail level on (16-byte aligned)
  int cvec;            // its length in 16-byte units
  int dl;              // tail level solved exactly by its inverse, or -1
  int inv;             // element offset of that inverse (natural order, transposed) in LDS
  int tmp;             // element offset of EBIT_DENSE_MAX scratch elements in LDS
  const int* inv_ok;   // 1 if the inversion succeeded
  const T* bg;         // right-hand side of the top tail level (colour-split order, 2 hs elements)
  T* xg;               // its correction (output, natural order)
};

// Register copy of one tail level's shape (read once per level visit, so
// the loops below do not go back to the case table), with float
// reciprocals for division-free index decoding.
struct TLev {
  int n0, n1, n2, N, hs, cb, xb, bb, p0, p1, p2;
  int hw, hc;              // colour slots per grid row and per colour
  int rs1, wy, wz;         // slots per z-plane, and the row offsets of a y / z wrap
  float r0, r1, r01, rhw;  // 1/n0, 1/n1, 1/(n0 n1), 1/hw
};

__device__ inline TLev tlev(const TailLevel& L) {
  TLev t;
  t.n0 = L.d.n[0];
  t.n1 = L.d.n[1];
  t.n2 = L.d.n[2];
  t.N = (int)L.d.N;
  t.hs = L.hs;
  t.cb = L.cb;
  t.xb = L.xb;
  t.bb = L.bb;
  t.p0 = L.d.per[0];
  t.p1 = L.d.per[1];
  t.p2 = L.d.per[2];
  t.hw = (t.n0 + 1) >> 1;
  t.hc = t.hw * t.n1 * t.n2;
  t.rs1 = t.hw * t.n1;
  t.wy = t.hw * (t.n1 - 1);
  t.wz = t.rs1 * (t.n2 - 1);
  t.r0 = 1.0f / (float)t.n0;
  t.r1 = 1.0f / (float)t.n1;
  t.r01 = 1.0f / (float)(t.n0 * t.n1);
  t.rhw = 1.0f / (float)t.hw;
  return t;
}

// c / n for 0 <= c < 2^22 given r = 1/n in float: the float quotient is off
// by at most one, which the remainder test corrects.
__device__ inline int qdiv(int c, int n, float r) {
  int q = (int)((float)c * r);
  const int m = c - q * n;
  q += (m >= n) - (m < 0);
  return q;
}

template <int DIM>
__device__ inline void cell_of(const TLev& d, int c, int& i, int& j, int& k) {
  if (DIM == 3) {
    const int s2 = d.n0 * d.n1;
    k = qdiv(c, s2, d.r01);
    c -= k * s2;
  } else {
    k = 0;
  }
  j = qdiv(c, d.n0, d.r0);
  i = c - j * d.n0;
}

// element of cell (i, j, k) within any field of level d
__device__ inline int rb_el(const TLev& d, int i, int j, int k) {
  return ((i + j + k) & 1) * d.hs + (i >> 1) + d.hw * (j + d.n1 * k);
}

__device__ inline float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Elements of the neighbours of cell (i, j, k) across sides +x, -x, +y, -y,
// +z, -z, with the periodic wrap.  Across a wall the wrapped cell is named
// too: the coupling stored there is exactly zero (the build adds no
// coupling across a wall), so its term vanishes without a test.  Each one
// is the cell's row base plus an offset: a neighbour is of the other
// colour, except across a wrap of a row, column or pile of odd length,
// where the parity does not change.
template <int DIM>
__device__ inline void rb_nbrs(const TLev& d, int i, int j, int k, int (&nb)[6]) {
  const int c = (i + j + k) & 1;
  const int R = d.hw * (j + d.n1 * k);
  const int oth = c ? 0 : d.hs;  // base of the other colour
  const int sam = c ? d.hs : 0;  // base of this colour
  const int h = i >> 1;
  const int cx = ((d.n0 - 1) & 1) ? oth : sam;
  nb[0] = R + (i + 1 < d.n0 ? oth + ((i + 1) >> 1) : cx);
  nb[1] = R + (i > 0 ? oth + ((i - 1) >> 1) : cx + ((d.n0 - 1) >> 1));
  const int cy = ((d.n1 - 1) & 1) ? oth : sam;
  nb[2] = h + (j + 1 < d.n1 ? oth + R + d.hw : cy + R - d.wy);
  nb[3] = h + (j > 0 ? oth + R - d.hw : cy + R + d.wy);
  if (DIM == 3) {
    const int cz = ((d.n2 - 1) & 1) ? oth : sam;
    nb[4] = h + (k + 1 < d.n2 ? oth + R + d.rs1 : cz + R - d.wz);
    nb[5] = h + (k > 0 ? oth + R - d.rs1 : cz + R + d.wz);
  }
}

// sum of coupling x neighbour value at element e with neighbours nb, in
// the order +x, -x, +y, -y, +z, -z (a coupling belongs to the cell on the
// lower side of its link)
template <typename T, int DIM>
__device__ inline T rb_nsum(const T* sm, const TLev& d, int e, const int (&nb)[6]) {
  const T* x = sm + d.xb;
  const T* o0 = sm + d.cb + 4 * d.hs;
  const T* o1 = o0 + 2 * d.hs;
  T s = 0;
  s = tfma(o0[e], x[nb[0]], s);
  s = tfma(o0[nb[1]], x[nb[1]], s);
  s = tfma(o1[e], x[nb[2]], s);
  s = tfma(o1[nb[3]], x[nb[3]], s);
  if (DIM == 3) {
    const T* o2 = o1 + 2 * d.hs;
    s = tfma(o2[e], x[nb[4]], s);
    s = tfma(o2[nb[5]], x[nb[5]], s);
  }
  return s;
}

// A thread's colour slot on a level: the elements of its cell and of the
// cell's neighbours for either colour the slot is swept in, computed once
// per level visit; ok bit c: the slot holds a cell in colour c (the last
// slot of a row of odd length does not in one colour; a slot past the end
// holds none); par: the element, on the coarse level, of the parent of the
// slot's colour-0 cell.
template <int DIM>
struct Slot {
  int el[2];
  int nb[2][6];
  int par;
  unsigned ok;
};

template <int DIM>
__device__ inline void slot_make(const TLev& d, int h, Slot<DIM>& s, const TLev* C) {
  s.ok = 0;
  if (h < d.hc) s.ok = 3;
  else h = 0;
  const int row = qdiv(h, d.hw, d.rhw);
  const int m = h - row * d.hw;
  int j = row, k = 0;
  if (DIM == 3) {
    k = qdiv(row, d.n1, d.r1);
    j = row - k * d.n1;
  }
  const int pr = (j + k) & 1;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    int i = 2 * m + (c ^ pr);
    if (i >= d.n0) {
      s.ok &= ~(1u << c);
      i = d.n0 - 1;
    }
    s.el[c] = c * d.hs + h;
    rb_nbrs<DIM>(d, i, j, k, s.nb[c]);
    if (c == 0 && C) s.par = rb_el(*C, i >> 1, j >> 1, k >> 1);
  }
}

// One colour C of a red-black Gauss-Seidel sweep over the slots of this
// thread.  A thread computes the new values of all its cells before storing
// any: within a colour no update reads another, so no load waits for a
// store.  FIRST: the first sweep from a zero iterate, x = b / diag on this
// colour (the neighbour sum vanishes, so nothing needs clearing first).
template <typename T, int DIM, int K, int C, bool FIRST>
__device__ inline void rb_colour(T* sm, const TLev& d, const Slot<DIM> (&sl)[K]) {
  T* x = sm + d.xb;
  const T* b = sm + d.bb;
  const T* di = sm + d.cb + 2 * d.hs;
  T nv[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int e = sl[u].el[C];
    if (FIRST)
      nv[u] = b[e] * di[e];
    else
      nv[u] = (b[e] - rb_nsum<T, DIM>(sm, d, e, sl[u].nb[C])) * di[e];
  }
#pragma unroll
  for (int u = 0; u < K; ++u)
    if ((sl[u].ok >> C) & 1) x[sl[u].el[C]] = nv[u];
}

// Pre-smoothing of level d (nu1 sweeps, colour 0 then 1, from zero) and
// the restriction of its residual into the right-hand side of C: the
// residual of the colour swept last vanishes (up to rounding) after a
// Gauss-Seidel sweep, so only the colour-0 children are summed.
// Slot of thread t: h = t + u nth, or with PAIR (2D, two slots, one
// thread per coarse cell) slot m of rows 2r and 2r + 1 for coarse cell
// t = (m, r), whose colour-0 cells are that coarse cell's two red children.
template <int DIM, bool PAIR>
__device__ inline int slot_of(const TLev& d, int t, int u, int nth) {
  if (!PAIR) return t + u * nth;
  const int r = qdiv(t, d.hw, d.rhw);
  return (t - r * d.hw) + d.hw * (2 * r + u);
}

template <typename T, int DIM, int K, bool PAIR, typename Sync>
__device__ inline void rb_pre(T* sm, const TLev& d, const TLev& C, int nu1, int t, int nth, Sync sync) {
  Slot<DIM> sl[K];
#pragma unroll
  for (int u = 0; u < K; ++u) slot_make<DIM>(d, slot_of<DIM, PAIR>(d, t, u, nth), sl[u], nullptr);
  const bool act = PAIR ? t < C.N : t < d.hc;
  if (act) rb_colour<T, DIM, K, 0, true>(sm, d, sl);
  sync();
  if (act) rb_colour<T, DIM, K, 1, false>(sm, d, sl);
  sync();
  for (int s = 1; s < nu1; ++s) {
    if (act) rb_colour<T, DIM, K, 0, false>(sm, d, sl);
    sync();
    if (act) rb_colour<T, DIM, K, 1, false>(sm, d, sl);
    sync();
  }
  const T* x = sm + d.xb;
  const T* b = sm + d.bb;
  const T* dg = sm + d.cb;
  T* bc = sm + C.bb;
  if constexpr (PAIR) {
    // restriction from the slot tables: the two red children of this
    // thread's coarse cell, (0,0) then (1,1)
    if (act) {
      T sum = 0;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = sl[u].el[0];
        const T r = b[e] - dg[e] * x[e] - rb_nsum<T, DIM>(sm, d, e, sl[u].nb[0]);
        sum = (sl[u].ok & 1) ? sum + r : sum;
      }
      const int cj = qdiv(t, C.n0, C.r0);
      bc[rb_el(C, t - cj * C.n0, cj, 0)] = sum;
    }
    sync();
    return;
  }
  // restriction: coarse cells I = t, t + nth, ... in natural order
  for (int I = t; I < C.N; I += nth) {
    int ci, cj, ck;
    cell_of<DIM>(C, I, ci, cj, ck);
    T sum = 0;
    // (two children at a time, for the registers in 3D)
#pragma unroll 2
    for (int ch = 0; ch < (DIM == 3 ? 4 : 2); ++ch) {
      int di_, dj_, dk_;
      even_child(ch, di_, dj_, dk_);
      int i = 2 * ci + di_, j = 2 * cj + dj_, k = 2 * ck + dk_;
      const bool in = i < d.n0 && j < d.n1 && k < d.n2;
      i = i < d.n0 ? i : d.n0 - 1;
      j = j < d.n1 ? j : d.n1 - 1;
      k = k < d.n2 ? k : d.n2 - 1;
      int nb[6];
      rb_nbrs<DIM>(d, i, j, k, nb);
      const int e = rb_el(d, i, j, k);
      const T r = b[e] - dg[e] * x[e] - rb_nsum<T, DIM>(sm, d, e, nb);
      sum = in ? sum + r : sum;
    }
    bc[rb_el(C, ci, cj, ck)] = sum;
  }
  sync();
}

// Post-smoothing of level d after the coarse level C: the correction of C
// added to the colour-0 cells (the only ones the first sweep, colour 1,
// reads; colour 1 is recomputed from them and colour 0 again after it, so
// neither needs the correction itself), then nu2 sweeps, colour 1 then 0.
template <typename T, int DIM, int K, bool PAIR, typename Sync>
__device__ inline void rb_post(T* sm, const TLev& d, const TLev& C, int nu2, int t, int nth, Sync sync) {
  Slot<DIM> sl[K];
#pragma unroll
  for (int u = 0; u < K; ++u) slot_make<DIM>(d, slot_of<DIM, PAIR>(d, t, u, nth), sl[u], &C);
  const bool act = PAIR ? t < C.N : t < d.hc;
  if (act) {
    T* x = sm + d.xb;
    const T* xc = sm + C.xb;
    T nv[K];
#pragma unroll
    for (int u = 0; u < K; ++u) nv[u] = x[sl[u].el[0]] + xc[sl[u].par];
#pragma unroll
    for (int u = 0; u < K; ++u)
      if (sl[u].ok & 1) x[sl[u].el[0]] = nv[u];
  }
  sync();
  for (int s = 0; s < nu2; ++s) {
    if (act) rb_colour<T, DIM, K, 1, false>(sm, d, sl);
    sync();
    if (act) rb_colour<T, DIM, K, 0, false>(sm, d, sl);
    sync();
  }
}

// colour slots per thread at most: two in FP32, one in FP64 (what the
// registers of a 1024-thread work-group hold; the levels that LDS can take
// need no more)
template <typename T, int DIM>
__host__ __device__ constexpr int tail_kmax() {
  return sizeof(T) == 4 ? 2 : 1;
}

// FP32 in 2D with one thread per coarse cell available: the row-pair
// slots (restriction from the slot tables); else one or two slots per
// thread at stride nth
template <typename T, int DIM, typename Sync>
__device__ inline void tail_pre(T* sm, const TLev& d, const TLev& C, int nu1, int t, int nth, Sync sync) {
  constexpr int KM = tail_kmax<T, DIM>();
  if (DIM == 2 && KM == 2 && C.N <= nth)
    rb_pre<T, DIM, KM, true>(sm, d, C, nu1, t, nth, sync);
  else if (KM == 1 || d.hc <= nth)
    rb_pre<T, DIM, 1, false>(sm, d, C, nu1, t, nth, sync);
  else
    rb_pre<T, DIM, KM, false>(sm, d, C, nu1, t, nth, sync);
}

template <typename T, int DIM, typename Sync>
__device__ inline void tail_post(T* sm, const TLev& d, const TLev& C, int nu2, int t, int nth, Sync sync) {
  constexpr int KM = tail_kmax<T, DIM>();
  if (DIM == 2 && KM == 2 && C.N <= nth)
    rb_post<T, DIM, KM, true>(sm, d, C, nu2, t, nth, sync);
  else if (KM == 1 || d.hc <= nth)
    rb_post<T, DIM, 1, false>(sm, d, C, nu2, t, nth, sync);
  else
    rb_post<T, DIM, KM, false>(sm, d, C, nu2, t, nth, sync);
}

// ---- the smallest tail levels by one wavefront ----------------------------
// Levels of at most tail_kmax x 64 slots per colour are processed by wave 0
// alone: its lanes synchronise through wave-scope fences instead of
// work-group barriers (LDS operations of one wave complete in order).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// V-cycle over tail levels l0 .. nl-1 by wave 0 (the rest of the work-group
// waits at the caller's barrier); level l0's right-hand side is in place.
template <typename T, int DIM>
__device__ inline void tail_wave(const TailArgs<T>& a, T* sm, int l0, int nl, bool dense) {
  const int lane = threadIdx.x;
  auto sync = [] { wave_sync(); };
  for (int l = l0; l < nl - 1; ++l) {
    const TLev L = tlev(a.L[l]);
    const TLev C = tlev(a.L[l + 1]);
    tail_pre<T, DIM>(sm, L, C, a.nu1, lane, 64, sync);
  }
  const TLev L = tlev(a.L[nl - 1]);
  T* x = sm + L.xb;
  const T* b = sm + L.bb;
  if (dense) {
    // coarsest level solved exactly, x = A^-1 b with the inverse in natural
    // order: lane t gathers b of cell t, then forms row t
    T* tb = sm + a.tmp;
    const T* inv = sm + a.inv;
    int e = 0;
    if (lane < L.N) {
      int i, j, k;
      cell_of<DIM>(L, lane, i, j, k);
      e = rb_el(L, i, j, k);
      tb[lane] = b[e];
    }
    wave_sync();
    T acc = 0;
    if (lane < L.N) {
#pragma unroll 8
      for (int j = 0; j < L.N; ++j) acc = tfma(inv[j * L.N + lane], tb[j], acc);
      x[e] = acc;
    }
    wave_sync();
  } else {
    // coarsest level: symmetric Gauss-Seidel from zero by one lane (exact
    // for one cell)
    for (int q = lane; q < 2 * L.hs; q += 64) x[q] = (T)0;
    wave_sync();
    if (lane == 0) {
      const T* di = sm + L.cb + 2 * L.hs;
      const int sweeps = L.N == 1 ? 1 : 50;
      for (int s = 0; s < sweeps; ++s)
        for (int dir = 0; dir < 2; ++dir)
          for (int qq = 0; qq < L.N; ++qq) {
            const int q = dir ? (L.N - 1 - qq) : qq;
            int i, j, k, nb[6];
            cell_of<DIM>(L, q, i, j, k);
            rb_nbrs<DIM>(L, i, j, k, nb);
            const int e = rb_el(L, i, j, k);
            x[e] = (b[e] - rb_nsum<T, DIM>(sm, L, e, nb)) * di[e];
          }
    }
    wave_sync();
  }
  for (int l = nl - 2; l >= l0; --l) {
    const TLev F = tlev(a.L[l]);
    const TLev C = tlev(a.L[l + 1]);
    tail_post<T, DIM>(sm, F, C, a.nu2, lane, 64, sync);
  }
}

template <typename T, int DIM>
__device__ inline void tail_body(const TailArgs<T>& a, T* sm) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nl = a.nl;
  {
    // the coefficient image suffix: all loads of a batch issue before any
    // store (an index past the end is clamped to the batch's first, whose
    // value it then stores again)
    const u32x4* src = reinterpret_cast<const u32x4*>(a.img);
    u32x4* dst = reinterpret_cast<u32x4*>(sm);
    const int nv = a.cvec;
    for (int e0 = tid; e0 < nv; e0 += TAIL_COPY_BATCH * nth) {
      int ei[TAIL_COPY_BATCH];
      u32x4 v[TAIL_COPY_BATCH];
#pragma unroll
      for (int u = 0; u < TAIL_COPY_BATCH; ++u) {
        ei[u] = e0 + u * nth < nv ? e0 + u * nth : e0;
        v[u] = src[ei[u]];
      }
#pragma unroll
      for (int u = 0; u < TAIL_COPY_BATCH; ++u) dst[ei[u]] = v[u];
    }
    // every level's iterate cleared (one region): a sweep may name a cell
    // not yet swept (across a wall, with a zero coupling; on a level of odd
    // length the wrapped cell there has the sweep's own colour); then the
    // top level's right-hand side, already in the colour-split order
    const TLev L = tlev(a.L[0]);
    u32x4* xz = reinterpret_cast<u32x4*>(sm + L.xb);
    const int nz = (L.bb - L.xb) * (int)sizeof(T) / 16;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (int e = tid; e < nz; e += nth) xz[e] = zero;
    const u32x4* bs = reinterpret_cast<const u32x4*>(a.bg);
    u32x4* bd = reinterpret_cast<u32x4*>(sm + L.bb);
    const int nbv = 2 * L.hs * (int)sizeof(T) / 16;
    for (int e0 = tid; e0 < nbv; e0 += 4 * nth) {
      int ei[4];
      u32x4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ei[u] = e0 + u * nth < nbv ? e0 + u * nth : e0;
        v[u] = bs[ei[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) bd[ei[u]] = v[u];
    }
  }
  __syncthreads();
  // with a usable inverse the V-cycle stops at its level
  const bool dense = a.dl >= 0 && *a.inv_ok;
  const int nle = dense ? a.dl + 1 : nl;
  // levels l0 .. nle-1 are small enough for one wavefront
  int l0 = nle - 1;
  while (l0 > 0 && tlev(a.L[l0 - 1]).hc <= tail_kmax<T, DIM>() * 64) --l0;
  auto sync = [] { __syncthreads(); };
  for (int l = 0; l < l0; ++l) {
    const TLev L = tlev(a.L[l]);
    const TLev C = tlev(a.L[l + 1]);
    tail_pre<T, DIM>(sm, L, C, a.nu1, tid, nth, sync);
  }
  if (tid < 64) tail_wave<T, DIM>(a, sm, l0, nle, dense);
  __syncthreads();
  for (int l = l0 - 1; l >= 0; --l) {
    const TLev L = tlev(a.L[l]);
    const TLev C = tlev(a.L[l + 1]);
    tail_post<T, DIM>(sm, L, C, a.nu2, tid, nth, sync);
  }
  {
    const TLev L = tlev(a.L[0]);
    const T* x = sm + L.xb;
    T* xg = a.xg;
    for (int q = tid; q < L.N; q += nth) {
      int i, j, k;
      cell_of<DIM>(L, q, i, j, k);
      xg[q] = x[rb_el(L, i, j, k)];
    }
  }
}

// ---------------------------------------------------------------------------
// hierarchy construction
// ---------------------------------------------------------------------------
__device__ inline void store_built(const BuildOut& o, long long I, int ci, int cj, int ck, double M, double F,
                                   const double (&cross)[3]) {
  const double dg = M + 0.5 * F;
  const long long hs = tail_half(o.cd), P = 2 * hs;
  const long long e = tail_el(o.cd, hs, ci, cj, ck);
  o.diag[I] = dg;
  o.mass[I] = M;
  if (o.d32) o.d32[I] = (float)dg;
  if (o.i32) {
    o.i32[e] = (float)dg;
    o.i32[P + e] = 1.0f / (float)dg;
  }
  if (o.i64) {
    o.i64[e] = dg;
    o.i64[P + e] = 1.0 / dg;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (o.off[a]) {
      const double v = 0.5 * cross[a];
      o.off[a][I] = v;
      if (o.o32[a]) o.o32[a][I] = (float)v;
      if (o.i32) o.i32[(2 + a) * P + e] = (float)v;
      if (o.i64) o.i64[(2 + a) * P + e] = v;
    }
}

// coarse cell I from the matrix-free fine operator (aggregate index of a
// wrapped fine cell along each axis: q >> 1)
__device__ inline void build_cell_from_fine(const FineOp& op, const BuildOut& o, long long I) {
  int ci, cj, ck;
  cell_ijk(o.cd, I, ci, cj, ck);
  double M = 0, F = 0, cross[3] = {0, 0, 0};
  for (int dk = 0; dk < 2; ++dk) {
    const int k = 2 * ck + dk;
    if (k >= op.d.n[2]) break;
    for (int dj = 0; dj < 2; ++dj) {
      const int j = 2 * cj + dj;
      if (j >= op.d.n[1]) break;
      for (int di = 0; di < 2; ++di) {
        const int i = 2 * ci + di;
        if (i >= op.d.n[0]) break;
        const long long c = cell_index(op.d, i, j, k);
        double diag, off[6], mass, rb = 0;
        fine_row<double>(op, i, j, k, op.flags[c], diag, off, mass, rb);
        M += mass;
        F += diag - mass;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          if (s >= 2 * op.d.dim || off[s] == 0.0) continue;
          int ni, nj, nk;
          neighbour(op.d, i, j, k, s, ni, nj, nk);
          const bool same = (ni >> 1) == ci && (nj >> 1) == cj && (nk >> 1) == ck;
          if (same)
            F += off[s];
          else if (s & 1)
            cross[s >> 1] += off[s];
        }
      }
    }
  }
  store_built(o, I, ci, cj, ck, M, F, cross);
}

// coarse cell I from the explicit level above
template <int DIM>
__device__ inline void build_cell_from_coarse(const CoarseOp<double>& op, const BuildOut& o, long long I) {
  int ci, cj, ck;
  cell_ijk(o.cd, I, ci, cj, ck);
  const int n0 = op.d.n[0], n1 = op.d.n[1], n2 = op.d.n[2];
  double M = 0, F = 0, cross[3] = {0, 0, 0};
  // children in order (dk, dj, di), G at a time: every load of a group is
  // issued before any is used.  Sides across a wall name the wrapped cell,
  // whose stored coupling there is zero, so they drop out at the zero test
  // like the missing neighbours they stand for.
  constexpr int G = DIM == 3 ? 2 : 4, NCH = DIM == 3 ? 8 : 4;
#pragma unroll 1
  for (int g = 0; g < NCH; g += G) {
    double mv[G], dv[G], ov[G][2 * DIM];
    int ii[G], jj[G], kk[G];
    bool in[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int ch = g + q;
      int i = 2 * ci + (ch & 1), j = 2 * cj + ((ch >> 1) & 1), k = 2 * ck + (ch >> 2);
      in[q] = i < n0 && j < n1 && k < n2;
      i = i < n0 ? i : n0 - 1;
      j = j < n1 ? j : n1 - 1;
      k = k < n2 ? k : n2 - 1;
      ii[q] = i;
      jj[q] = j;
      kk[q] = k;
      const long long c = cell_index(op.d, i, j, k);
      long long m[6];
      fine_nbrs(op.d, i, j, k, c, m);
      mv[q] = op.mass[c];
      dv[q] = op.diag[c];
#pragma unroll
      for (int s = 0; s < 2 * DIM; ++s) ov[q][s] = (s & 1) ? op.off[s >> 1][c] : op.off[s >> 1][m[s]];
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      if (!in[q]) continue;
      M += mv[q];
      F += dv[q] - mv[q];
#pragma unroll
      for (int s = 0; s < 2 * DIM; ++s) {
        const double off = ov[q][s];
        if (off == 0.0) continue;
        const int a = s >> 1, up = s & 1;
        int ni = ii[q], nj = jj[q], nk = kk[q];
        if (a == 0) ni = up ? (ni + 1 < n0 ? ni + 1 : 0) : (ni > 0 ? ni - 1 : n0 - 1);
        if (a == 1) nj = up ? (nj + 1 < n1 ? nj + 1 : 0) : (nj > 0 ? nj - 1 : n1 - 1);
        if (a == 2) nk = up ? (nk + 1 < n2 ? nk + 1 : 0) : (nk > 0 ? nk - 1 : n2 - 1);
        const bool same = (ni >> 1) == ci && (nj >> 1) == cj && (nk >> 1) == ck;
        if (same)
          F += off;
        else if (up)
          cross[a] += off;
      }
    }
  }
  store_built(o, I, ci, cj, ck, M, F, cross);
}

// One level of both systems in one launch: blocks [0, nb) build the
// heat system's cells, blocks [nb, 2 nb) the pressure system's.
template <bool B>
__global__ void k_build_from_fine2(Many<BuildFineArgs> m) {
  long long lb, nbc;
  const BuildFineArgs& a = many_case<B>(m, lb, nbc);
  const bool s1 = lb >= a.nb;
  const long long I = (lb - (s1 ? a.nb : 0u)) * blockDim.x + threadIdx.x;
  if (I >= a.o[0].cd.N) return;
  if (s1)
    build_cell_from_fine(a.op[1], a.o[1], I);
  else
    build_cell_from_fine(a.op[0], a.o[0], I);
}

template <int DIM, bool B>
__global__ void k_build_from_coarse2(Many<BuildCoarseArgs> m) {
  long long lb, nbc;
  const BuildCoarseArgs& a = many_case<B>(m, lb, nbc);
  const bool s1 = lb >= a.nb;
  const long long I = (lb - (s1 ? a.nb : 0u)) * blockDim.x + threadIdx.x;
  if (I >= a.o[0].cd.N) return;
  if (s1)
    build_cell_from_coarse<DIM>(a.op[1], a.o[1], I);
  else
    build_cell_from_coarse<DIM>(a.op[0], a.o[0], I);
}


// Inverse of the operator of a level of at most EBIT_DENSE_MAX cells (the
// exact coarsest solve): assembled row by row with the couplings of
// coarse_offsum, inverted in place by Gauss-Jordan elimination without
// pivoting (the operator is symmetric positive definite), written
// transposed so that lane t of a wave reads column t contiguously.  A
// pivot that is not positive and finite (a singular level) clears *ok and
// the tail keeps its Gauss-Seidel coarsest solve.
__device__ inline bool dense_inverse(const CoarseOp<double>& op, double* inv64, float* inv32, int* ok,
                                     double (*A)[EBIT_DENSE_MAX + 1], double (*colb)[EBIT_DENSE_MAX],
                                     double (*rowb)[EBIT_DENSE_MAX]) {
  constexpr int M = EBIT_DENSE_MAX;
  constexpr int CW = M / 4;  // columns per owning wave
  const int N = (int)op.d.N;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const bool owner = w < 4;  // waves 0-3 hold the matrix, the others only keep the barriers
  for (int e = tid; e < M * M; e += blockDim.x) A[e / M][e % M] = 0.0;
  __syncthreads();
  if (tid < N) {
    int i, j, k;
    cell_ijk(op.d, tid, i, j, k);
    A[tid][tid] = op.diag[tid];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= op.d.dim) continue;
      int ni, nj, nk;
      if (neighbour(op.d, i, j, k, 2 * a + 1, ni, nj, nk)) A[tid][cell_index(op.d, ni, nj, nk)] += op.off[a][tid];
      if (neighbour(op.d, i, j, k, 2 * a, ni, nj, nk)) {
        const long long m = cell_index(op.d, ni, nj, nk);
        A[tid][m] += op.off[a][m];
      }
    }
  }
  __syncthreads();
  // lane i of wave w keeps A[i][CW w .. CW w + CW - 1] in registers
  double r[CW];
#pragma unroll
  for (int jj = 0; jj < CW; ++jj) r[jj] = owner ? A[lane][CW * w + jj] : 0.0;
  bool good = true;
  for (int pw = 0; pw < 4 && pw * CW < N && good; ++pw) {
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int p = pw * CW + c;
      if (p < N && good) {
        // column p and row p of the current matrix go through LDS; the two
        // buffers alternate so one barrier per pivot suffices
        const int buf = c & 1;
        if (w == pw) colb[buf][lane] = r[c];
        if (owner && lane == p) {
#pragma unroll
          for (int jj = 0; jj < CW; ++jj) rowb[buf][CW * w + jj] = r[jj];
        }
        __syncthreads();
        const double piv = colb[buf][p];
        if (!(piv > 0.0) || !isfinite(piv)) {
          good = false;
        } else if (owner) {
          const double ip = 1.0 / piv;
          const double f = colb[buf][lane];
#pragma unroll
          for (int jj = 0; jj < CW; ++jj) {
            const int j = CW * w + jj;
            const double prj = rowb[buf][j] * ip;
            if (lane == p) r[jj] = (j == p) ? ip : prj;
            else r[jj] = (j == p) ? -f * ip : r[jj] - f * prj;
          }
        }
      }
    }
  }
  if (owner && lane < N) {
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) {
      const int j = CW * w + jj;
      if (j < N) {
        inv64[j * N + lane] = r[jj];
        if (inv32) inv32[j * N + lane] = (float)r[jj];
      }
    }
  }
  if (tid == 0) *ok = good ? 1 : 0;
  return good;
}

// Per system, everything the one-work-group part of a hierarchy build needs
// (filled once per context: the pointers do not change between builds).
struct BuildTable {
  int ls, nlev, dl;  // first level built by k_build_small, level count, dense level (-1: none)
  Dims d[EBIT_MAX_LEVELS];
  double* diag[EBIT_MAX_LEVELS];
  double* mass[EBIT_MAX_LEVELS];
  double* off[EBIT_MAX_LEVELS][3];
  float* d32[EBIT_MAX_LEVELS];
  float* o32[EBIT_MAX_LEVELS][3];
  float* i32[EBIT_MAX_LEVELS];
  double* i64[EBIT_MAX_LEVELS];
  double* inv64;
  float* inv32;
  int* inv_ok;
};

// Levels ls .. nlev-1 (each from the one above) and the inverse of the
// dense level: one work-group per system, a barrier between levels.  The
// levels below the dense one serve only a failed inversion (the tail then
// falls back to Gauss-Seidel on the coarsest level), so they are built
// after it and only in that case.
template <int DIM>
__device__ inline void build_small_level(const BuildTable& t, int l) {
  CoarseOp<double> f;
  f.d = t.d[l - 1];
  f.diag = t.diag[l - 1];
  f.mass = t.mass[l - 1];
#pragma unroll
  for (int a = 0; a < 3; ++a) f.off[a] = t.off[l - 1][a];
  BuildOut o;
  o.cd = t.d[l];
  o.diag = t.diag[l];
  o.mass = t.mass[l];
  o.d32 = t.d32[l];
  o.i32 = t.i32[l];
  o.i64 = t.i64[l];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o.off[a] = t.off[l][a];
    o.o32[a] = t.o32[l][a];
  }
  for (long long I = threadIdx.x; I < o.cd.N; I += blockDim.x) build_cell_from_coarse<DIM>(f, o, I);
  __syncthreads();
}

template <int DIM, bool B>
__global__ __launch_bounds__(1024) void k_build_small(Many<BuildSmallArgs> m) {
  __shared__ double A[EBIT_DENSE_MAX][EBIT_DENSE_MAX + 1];
  __shared__ double colb[2][EBIT_DENSE_MAX], rowb[2][EBIT_DENSE_MAX];
  long long lb, nbc;
  const BuildSmallArgs& a = many_case<B>(m, lb, nbc);
  const BuildTable& t = ((const BuildTable*)a.tabs)[lb];
  const int ls = t.ls, nlev = t.nlev, dl = t.dl;
  const int upto = dl >= 0 ? dl + 1 : nlev;
  for (int l = ls; l < upto; ++l) build_small_level<DIM>(t, l);
  if (dl < 0) return;
  CoarseOp<double> f;
  f.d = t.d[dl];
  f.diag = t.diag[dl];
  f.mass = t.mass[dl];
#pragma unroll
  for (int a = 0; a < 3; ++a) f.off[a] = t.off[dl][a];
  const bool good = dense_inverse(f, t.inv64, t.inv32, t.inv_ok, A, colb, rowb);
  if (!good) {
    __syncthreads();
    for (int l = (ls > dl + 1 ? ls : dl + 1); l < nlev; ++l) build_small_level<DIM>(t, l);
  }
}

// ---------------------------------------------------------------------------
// outer loop (FP64) with deterministic two-stage reductions
// ---------------------------------------------------------------------------

#define GRID_STRIDE(c, N) \
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < (N); c += (long long)gridDim.x * blockDim.x)
// the same over the nb blocks one case owns in a batched launch (this block
// is its lb-th), the blocks of one XCD taking neighbouring rows (xcd_tile)
#define CASE_STRIDE(c, N)                                                                                   \
  for (long long c = (long long)xcd_tile(lb, nb) * blockDim.x + threadIdx.x; c < (N); c += (long long)nb * blockDim.x)


// Error-free transformations (Knuth TwoSum, FMA-based TwoProd) for a
// residual evaluated in double-double arithmetic.
__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ inline void dd_add(double& hi, double& lo, double p, double pe) {
  double s, e;
  two_sum(hi, p, s, e);
  e += lo + pe;
  hi = s + e;
  lo = e - (hi - s);
}

// r = b - A x in flux form, accumulated in double-double and rounded once
// (x may be null: r = b); partials: b.b, r.r and the squared norm of
// |b| + |A||x| (a residual cannot be certified below ~eps of that, since the
// rounding of x itself, eps |x| per entry and not smooth, leaves a residual
// of that size).  With the compensated residual the outer loop's restarts
// steer x to the correctly rounded discrete solution.
template <int SYS, typename T = double>
__device__ inline void resid_init_body(const FineOp& op, const double* __restrict__ b, const double* __restrict__ x,
                                       double* __restrict__ r, double* partial, int lb, int nb,
                                       double* __restrict__ xzero = nullptr, T* __restrict__ rv = nullptr,
                                       int split = 0) {
  const long long H = split ? split_half(op.d) : 0;
  double v[3] = {0, 0, 0};
  CASE_STRIDE(c, op.d.N) {
    const double bc = b[c];
    if (xzero) xzero[c] = 0.0;  // a cold start: x = 0, so r = b
    double rc = bc, ac = fabs(bc);
    if (x) {
      int i, j, k;
      cell_ijk(op.d, c, i, j, k);
      double diag, off[6], mass, rb = 0, mx;
      fine_row<double, SYS>(op, i, j, k, op.flags[c], diag, off, mass, rb, &mx);
      const double xc = x[c];
      double hi = bc, lo = 0.0;
      {
        const double p = mx * xc;
        dd_add(hi, lo, -p, -fma(mx, xc, -p));
      }
      ac += fabs(diag * xc);
      const int ns = 2 * op.d.dim;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        if (q >= ns || off[q] == 0.0) continue;
        int ni, nj, nk;
        neighbour(op.d, i, j, k, q, ni, nj, nk);
        const double xn = x[cell_index(op.d, ni, nj, nk)];
        double dh, dl;
        two_sum(xc, -xn, dh, dl);         // x_c - x_n exactly as dh + dl
        // r += off (x_c - x_n)  (off = -w, so this subtracts w (x_c - x_n))
        const double p = off[q] * dh;
        dd_add(hi, lo, p, fma(off[q], dh, -p) + off[q] * dl);
        ac += fabs(off[q] * xn);
      }
      rc = hi + lo;
    }
    if (r) r[c] = rc;
    if (rv) {
      if (split) {
        int i, j, k;
        cell_ijk(op.d, c, i, j, k);
        rv[split_index(op.d, H, i, j, k)] = (T)rc;
      } else {
        rv[c] = (T)rc;
      }
    }
    v[0] += bc * bc;
    v[1] += rc * rc;
    v[2] += ac * ac;
  }
  write_partials<3>(v, partial, lb, nb);
}

// y = A x (difference form: no cancellation between diagonal and couplings)
__global__ void k_apply(FineOp op, const double* __restrict__ x, double* __restrict__ y) {
  GRID_STRIDE(c, op.d.N) {
    int i, j, k;
    cell_ijk(op.d, c, i, j, k);
    double diag, off[6], mass, rb = 0, mx;
    fine_row<double>(op, i, j, k, op.flags[c], diag, off, mass, rb, &mx);
    const double xc = x[c];
    double s = mx * xc;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q >= 2 * op.d.dim || off[q] == 0.0) continue;
      int ni, nj, nk;
      neighbour(op.d, i, j, k, q, ni, nj, nk);
      s -= off[q] * (xc - x[cell_index(op.d, ni, nj, nk)]);
    }
    y[c] = s;
  }
}

// heat right-hand side: b = rho cp/dt T* + interface and wall terms
template <bool B>
__global__ void k_heat_rhs(Many<HeatRhsArgs> m) {
  long long lb, nb;
  const HeatRhsArgs& a = many_case<B>(m, lb, nb);
  const FineOp& op = a.op;
  const double* __restrict__ Ts = a.Ts;
  double* __restrict__ b = a.b;
  for (long long c = lb * blockDim.x + threadIdx.x; c < op.d.N; c += nb * blockDim.x) {
    int i, j, k;
    cell_ijk(op.d, c, i, j, k);
    const uint8_t f = op.flags[c];
    double diag, off[6], mass;
    double rb = op.mass[(f & F_LIQ) ? 1 : 0] * Ts[c];
    fine_row<double>(op, i, j, k, f, diag, off, mass, rb);
    b[c] = rb;
  }
}


// Sum (or max) of nv rows of nb partials, in a fixed order; result in thread 0.
__device__ inline void reduce_partials(const double* __restrict__ partial, int nb, int nv, bool mx,
                                       double (&v)[3]) {
  __shared__ double sh[4 * 4];
  for (int q = 0; q < 3; ++q) {
    double s = 0;
    if (q < nv) {
      if (mx) {
        for (int t = threadIdx.x; t < nb; t += blockDim.x) s = fmax(s, partial[q * nb + t]);
      } else {
        for (int t = threadIdx.x; t < nb; t += blockDim.x) s += partial[q * nb + t];
      }
    }
    v[q] = s;
  }
  if (mx) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double m = wave_max(v[0]);
    if (lane == 0) sh[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) v[0] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  } else {
    block_sum<3>(v, sh);
  }
}

// single-system reductions outside the solves (divergence maximum)
template <bool B>
__global__ void k_finalize(Many<FinArgs> m) {
  long long lb, nbc;
  const FinArgs& a = many_case<B>(m, lb, nbc);
  double v[3];
  reduce_partials(a.partial, a.nb, a.nv, a.kind == FIN_MAX, v);
  if (threadIdx.x != 0) return;
  if (a.kind == FIN_MAX) a.sc->divmax = v[0];
  if (a.kind == FIN_SUM1) a.sc->red[0] = v[0];
}

// a case's status scalars: cleared (dst null) or copied to dst
template <bool B>
__global__ void k_scal(Many<ScalArgs> m) {
  long long lb, nbc;
  const ScalArgs& a = many_case<B>(m, lb, nbc);
  constexpr int W = (int)(sizeof(Scal) / sizeof(double));
  const double* src = (const double*)a.scal;
  double* dst = a.dst ? (double*)a.dst : (double*)a.scal;
  for (int t = threadIdx.x; t < W; t += blockDim.x) dst[t] = a.dst ? src[t] : 0.0;
}

// ---------------------------------------------------------------------------
// Batched solves.  Every kernel of the solve takes the table of cases and a
// work list that maps its 1D grid onto (case, block of that case), so one
// launch serves every case of a batch; the single-context entry points run
// a batch of one.  Per-case control words carry the active mask, the CG
// restart flag and the search-direction slot: a fixed block of outer
// iterations can be replayed as a graph while converged cases drop out on
// the device.
// ---------------------------------------------------------------------------
struct WorkList {
  const int* start;  // [n + 1]: first block of entry e; start[n] = blocks in the launch
  const int* cid;    // [n]: case of entry e
  int n;
  int c0, total;     // the case and block count when n == 1 (no table lookup)
};

__device__ inline int wl_find(const WorkList& w, int& lb, int& nb) {
  const int b = blockIdx.x;
  if (w.n == 1) {
    lb = b;
    nb = w.total;
    return w.c0;
  }
  int lo = 0, hi = w.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w.start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  lb = b - w.start[lo];
  nb = w.start[lo + 1] - w.start[lo];
  return w.cid[lo];
}

// control word of one case (host writes between iteration blocks, the
// finalize kernels on the device)
struct CaseCtl {
  int active;    // iterating
  int fresh;     // next iteration restarts the CG recurrence (beta = 0)
  int pi;        // p[pi] holds the current search direction
  int recheck;   // 1: selected for a recomputation of the true residual; 2: b = 0, x to be cleared
  int pend;      // the x/r update's r.r is not yet taken (2D: the next V-cycle's first launch takes it)
  int pad;
  double stop2;  // the case stops once r.r falls to this level
};

enum { MASK_ACTIVE = 0, MASK_ALL = 1, MASK_ZERO = 3, MASK_STOPPED = 4 };
__device__ inline bool selected(const CaseCtl& c, int mask) {
  if (mask == MASK_ALL) return true;
  if (mask == MASK_ACTIVE) return c.active != 0;
  if (mask == MASK_ZERO) return c.recheck == 2;
  return c.recheck == 1;  // MASK_STOPPED
}

// Device view of one solve of one case: operator, vectors, hierarchy.
template <typename T>
struct SolveCase {
  FineOp op;
  const double* b;
  double* x;
  double* r;
  T* rv;             // the V-cycle's fine right-hand side: r itself (2D FP64) or its copy (FP32, or 3D
                     // in the colour-split order)
  const uint8_t* fs; // 3D: the flags in the colour-split order
  int split;         // 3D: the fine iterate z[0], rv and fs are in the colour-split order
  T* z[2];           // V-cycle result (z[0]) and the second sweep buffer
  double* p[2];
  double* q;
  double* partial;   // [4][nred]: rows 0-1 z.r, z.q (0-2 at a residual recomputation), 2 p.q, 3 r.r
  Scal* sc;
  int nred;          // reduction blocks of this case
  int ndot;          // > 0: the last fine sweep of a V-cycle writes the z.r, z.q partials (one per tile)
  int nlev, lt;      // levels; levels lt .. nlev-1 are solved by the tail kernel
  int fzc, fgx, fgy; // fine sweep: z-chunk and tile grid
  CoarseOp<T> lev[EBIT_MAX_LEVELS];  // explicit levels 1 .. lt-1 (and lt: its size)
  T* lb[EBIT_MAX_LEVELS];
  T* lx[EBIT_MAX_LEVELS][2];
  int lzc[EBIT_MAX_LEVELS], lgx[EBIT_MAX_LEVELS], lgy[EBIT_MAX_LEVELS];
  TailArgs<T> tail;
};

template <typename T>
__global__ void kb_zero_x(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl,
                          int mask) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!selected(ctl[c], mask)) return;
  const SolveCase<T>& C = cs[c];
  CASE_STRIDE(i, C.op.d.N) C.x[i] = 0.0;
}

// compiled per system (SYS), as the p-update
template <typename T, int SYS>
__global__ void kb_resid_init(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl,
                              int mask, int use_x, int zero_x) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!selected(ctl[c], mask)) return;
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  resid_init_body<SYS, T>(op, C.b, use_x ? (const double*)C.x : nullptr, C.r, C.partial, lb, nb,
                       zero_x ? C.x : nullptr,
                          (C.split || !std::is_same<T, double>::value) ? C.rv : nullptr, C.split);
}

template <typename T>
void launch_resid_init(int blocks, const SolveCase<T>* cs, const CaseCtl* ctl, WorkList w, int sys, int mask,
                       int use_x, int zero_x, hipStream_t st) {
  if (sys == EBIT_SYS_HEAT)
    hipLaunchKernelGGL((kb_resid_init<T, EBIT_SYS_HEAT>), dim3(blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl, w, mask,
                       use_x, zero_x);
  else
    hipLaunchKernelGGL((kb_resid_init<T, EBIT_SYS_PRESSURE>), dim3(blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl, w,
                       mask, use_x, zero_x);
}

template <typename T, int TX, int TY, int NSW, int RES>
__global__ __launch_bounds__(RB_THREADS) void kb_rb_fine(const SolveCase<T>* __restrict__ cs,
                                                         CaseCtl* __restrict__ ctl, WorkList wl, int in_sel,
                                                         int out_sel, int add_xc, int dots, int settle) {
  using FT = FineTile<TX, TY>;
  using W = Win2<TX, TY, NSW, RES>;
  // one set of buffers serves the 3D z-march (four iterate planes, two r /
  // flag planes) and the 2D staged window
  constexpr int QB = W::QL > 2 * FT::QL ? (W::QL + 1) / 2 : FT::QL;
  static_assert(W::PL <= 4 * FT::PL && W::QL <= 2 * QB, "2D windows must fit the sweep buffers");
  __shared__ T xs[4][FT::PL];
  __shared__ T rs[2][QB];
  __shared__ uint8_t fs[2][QB];
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  // register copies, read together with the control word: the sweep never
  // goes back to the table
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  const T* r = C.rv;
  const T* zin = in_sel < 0 ? nullptr : (const T*)C.z[in_sel];
  T* zout = C.z[out_sel];
  const T* xc = add_xc ? (const T*)C.lx[1][0] : nullptr;
  const Dims cd = C.lev[1].d;
  const int fgx = C.fgx, fgy = C.fgy, fzc = C.fzc;
  T* bc = RES ? C.lb[1] : nullptr;
  T* xcz = RES ? C.lx[1][0] : nullptr;
  // The control word, read once for the whole block: block 0 of the case
  // may rewrite it (ending the previous iteration) while other blocks start,
  // and every wave of a block must take the same branch (barriers follow).
  __shared__ CaseCtl sctl;
  __shared__ int sact;
  if (threadIdx.x == 0) sctl = ctl[c];
  __syncthreads();
  const CaseCtl cc = sctl;
  if (settle && cc.pend) {
    // the previous iteration's r.r, reduced by every block in the same
    // fixed order: a case at its stop level skips this V-cycle, and block 0
    // ends the iteration in its control word.  A block that read the word
    // after block 0 rewrote it sees pend = 0 and the new active flag: the
    // same decision.
    double v[3];
    reduce_partials(C.partial + 3 * C.nred, C.nred, 1, false, v);
    if (threadIdx.x == 0) {
      sact = (v[0] <= cc.stop2 || !isfinite(v[0])) ? 0 : 1;
      if (lb == 0) end_iteration(C.sc, ctl + c, cc, v[0]);
    }
    __syncthreads();
    if (!sact) return;
  } else if (!cc.active) {
    return;
  }
  const int lt = xcd_tile(lb, nb);
  const int bx = lt % fgx, by = (lt / fgx) % fgy, bz = lt / (fgx * fgy);
  if constexpr (RES || TY == 4) {
    // dots (last post-smoothing launch): 1 + [defect correction]; the tile
    // partials replace the separate dot kernel for cases with ndot > 0
    int dm = 0;
    if (dots && C.ndot > 0) dm = (dots == 2 || cc.fresh) ? 2 : 1;
    rb_fine2d_body<T, TX, TY, NSW, RES>(op, r, zin, xc, cd, zout, bx, by, &xs[0][0], &rs[0][0], &fs[0][0], bc, xcz,
                                        C.lt == 1, dm, C.q, C.partial, lb, C.ndot, C.r);
  } else {
    if (op.d.dim == 2)
      rb_fine2d_body<T, TX, TY, NSW, 0>(op, r, zin, xc, cd, zout, bx, by, &xs[0][0], &rs[0][0], &fs[0][0], bc, xcz,
                                        0);
    else
      rb_fine_body<T, TX, TY>(op, r, zin, xc, cd, zout, fzc, bx, by, bz, xs, rs, fs);
  }
}

template <typename T, int NSW, int RES>
__global__ __launch_bounds__(RB_THREADS) void kb_rb_coarse(const SolveCase<T>* __restrict__ cs,
                                                           const CaseCtl* __restrict__ ctl, WorkList wl, int l,
                                                           int in_sel, int out_sel, int add_xc) {
  __shared__ T buf[RB_SBUF];
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const SolveCase<T>& C = cs[c];
  const CoarseRows<T> rows{C.lev[l], C.lb[l]};
  const int gx = C.lgx[l], gy = C.lgy[l], zc = C.lzc[l];
  const T* xin = in_sel < 0 ? nullptr : (const T*)C.lx[l][in_sel];
  const T* xc = add_xc ? (const T*)C.lx[l + 1][0] : nullptr;
  const Dims cd = C.lev[l + 1].d;
  T* xout = C.lx[l][out_sel];
  T* bc = RES ? C.lb[l + 1] : nullptr;
  T* xcz = RES ? C.lx[l + 1][0] : nullptr;
  if (!ctl[c].active) return;
  const int lt = xcd_tile(lb, nb);
  if (RES || rows.op.d.dim == 2)
    rb_coarse2d_body<T, NSW, RES>(rows.op, rows.b, xin, xc, cd, xout, lt % gx, (lt / gx) % gy, buf, bc, xcz,
                                  C.lt == l + 1);
  else
    rb_fused_body<T, CoarseRows<T>>(rows, xin, xc, cd, xout, zc, lt % gx, (lt / gx) % gy, lt / (gx * gy),
                                    reinterpret_cast<T(*)[RB_PLANE]>(buf));
}

// Restricted residual (P^T r over the colour-0 children) of every coarse
// cell of level 1; also clears the level-1 iterate.
template <typename T>
__global__ void kb_fine_restrict(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl,
                                 int src_sel) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  const Dims cd = C.lev[1].d;
  const T* x = C.z[src_sel];
  T* bc = C.lb[1];
  T* xc = C.lx[1][0];
  const int nch = op.d.dim == 3 ? 4 : 2;
  CASE_STRIDE(I, cd.N) {
    int ci, cj, ck;
    cell_ijk(cd, I, ci, cj, ck);
    T sum = 0;
    for (int ch = 0; ch < nch; ++ch) {
      int di, dj, dk;
      even_child(ch, di, dj, dk);
      const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
      if (i < op.d.n[0] && j < op.d.n[1] && k < op.d.n[2])
        sum += fine_residual_at<T, T>(op, i, j, k, cell_index(op.d, i, j, k), C.rv, x);
    }
    bc[C.lt == 1 ? tail_el(cd, tail_half(cd), ci, cj, ck) : I] = sum;
    xc[I] = (T)0;
  }
}

// ---------------------------------------------------------------------------
// 3D fine level in the colour-split order (split_index): a red-black sweep
// is two launches, one per colour.  A half-sweep reads the other colour's
// half of the iterate and writes its own: every access is a coalesced
// stream, 13 bytes per cell and full sweep in FP32 (read x of the other
// colour, r and the flag; write x), with the six neighbour reads of a cell
// served from the caches.
// ---------------------------------------------------------------------------

// the other-colour neighbours of cell (i, j, k) (slot s of its colour):
// -x, +x, -y, +y, -z, +z; q < 0 where the neighbour is beyond a wall.  A
// step of one cell wraps by adding or subtracting the axis length.
__device__ inline void split_nbrs(const Dims& d, int hw, int i, int j, int k, long long s, long long (&q)[6],
                                  int (&ni)[6], int (&nj)[6], int (&nk)[6]) {
  const long long row = hw, plane = (long long)hw * d.n[1];
  const long long rs = s - (i >> 1);  // slot of the row's first cell
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    ni[e] = i;
    nj[e] = j;
    nk[e] = k;
    q[e] = s;
  }
  // -x / +x: the other colour's slot in the same row
  int a = i - 1;
  if (a < 0) a = d.per[0] ? a + d.n[0] : -1;
  ni[0] = a;
  q[0] = a >= 0 ? rs + (a >> 1) : -1;
  a = i + 1;
  if (a >= d.n[0]) a = d.per[0] ? a - d.n[0] : -1;
  ni[1] = a;
  q[1] = a >= 0 ? rs + (a >> 1) : -1;
  // -y / +y
  a = j - 1;
  if (a < 0) a = d.per[1] ? a + d.n[1] : -1;
  nj[2] = a;
  q[2] = a >= 0 ? s + row * (a - j) : -1;
  a = j + 1;
  if (a >= d.n[1]) a = d.per[1] ? a - d.n[1] : -1;
  nj[3] = a;
  q[3] = a >= 0 ? s + row * (a - j) : -1;
  // -z / +z
  a = k - 1;
  if (a < 0) a = d.per[2] ? a + d.n[2] : -1;
  nk[4] = a;
  q[4] = a >= 0 ? s + plane * (a - k) : -1;
  a = k + 1;
  if (a >= d.n[2]) a = d.per[2] ? a - d.n[2] : -1;
  nk[5] = a;
  q[5] = a >= 0 ? s + plane * (a - k) : -1;
}

// Tiles of the colour-split kernels: 64 slots of a row x 4 rows (j) of one
// plane (k); a wave takes 64 consecutive slots.  The block -> tile mapping
// needs no per-thread division.
#define SP_TX 64
#define SP_TY 4
__host__ __device__ inline int split_tiles(int nx, int ny, int nz) {
  return ((nx + SP_TX - 1) / SP_TX) * ((ny + SP_TY - 1) / SP_TY) * nz;
}
// A work-group takes SP_TPB consecutive tiles: the per-block set-up (work
// list, control word, operator, constants) is paid once for all of them, and
// the tiles of one XCD's work-groups are contiguous (xcd_tile).
#define SP_TPB 8
#define SP_TPB_R 2  // the restriction: four children per thread, fewer tiles per work-group
__host__ __device__ inline int split_blocks(int tiles, int tpb = SP_TPB) { return (tiles + tpb - 1) / tpb; }
__device__ inline void split_tile(int t, int nx, int ny, int& x, int& y, int& z) {
  const int gx = (nx + SP_TX - 1) / SP_TX, gy = (ny + SP_TY - 1) / SP_TY;
  const int bx = t % gx, r = t / gx;
  x = bx * SP_TX + (int)(threadIdx.x % SP_TX);
  y = (r % gy) * SP_TY + (int)(threadIdx.x / SP_TX);
  z = r / gy;
}

// pointers the compiler may address as global memory (global_load /
// global_store instead of the generic flat forms)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

// Buffer-resource access to the colour-split arrays: a 32-bit byte offset
// per lane (one add per neighbour instead of a 64-bit address), and a load
// past the end of the buffer returns 0.  Every array addressed this way has
// fewer than 2^31 bytes (the plan keeps larger grids on the LDS sweeps).
typedef __amdgpu_buffer_rsrc_t BufRsrc;
__device__ inline BufRsrc buf_rsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline T buf_load(BufRsrc r, int off);
template <>
__device__ inline float buf_load<float>(BufRsrc r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline double buf_load<double>(BufRsrc r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void buf_store(float v, BufRsrc r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline void buf_store(double v, BufRsrc r, int off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// The six other-colour neighbour values of slot sb (bytes) of cell
// (i, j, k) in a colour-split half-sweep: wall sides read past the end of
// the half (0); MODE 1 reads none (a zero start), MODE 2 adds the coarse
// correction of each neighbour's level-1 parent.
template <typename T, int MODE>
__device__ inline void half3_nbrs(BufRsrc bxn, int Hb, int n0, int n1, int n2, int hw, int plane, bool p0, bool p1,
                                  bool p2, int i, int j, int k, int par, int ih, int sb, bool ok,
                                  gptr<const T> xc, int cn0, int cn1, T (&v)[6]) {
  constexpr int TS = (int)sizeof(T);
#pragma unroll
  for (int e = 0; e < 6; ++e) v[e] = (T)0;
  if constexpr (MODE == 1) return;
  const bool xm = i == 0, xp = i == n0 - 1, ym = j == 0, yp = j == n1 - 1, zm = k == 0, zp = k == n2 - 1;
  const int dx0 = xm ? (p0 ? (hw - 1) * TS : Hb) : (par - 1) * TS;
  const int dx1 = xp ? (p0 ? -ih * TS : Hb) : par * TS;
  const int dy0 = ym ? (p1 ? hw * (n1 - 1) * TS : Hb) : -hw * TS;
  const int dy1 = yp ? (p1 ? -hw * (n1 - 1) * TS : Hb) : hw * TS;
  const int dz0 = zm ? (p2 ? plane * (n2 - 1) * TS : Hb) : -plane * TS;
  const int dz1 = zp ? (p2 ? -plane * (n2 - 1) * TS : Hb) : plane * TS;
  v[0] = buf_load<T>(bxn, sb + dx0);
  v[1] = buf_load<T>(bxn, sb + dx1);
  v[2] = buf_load<T>(bxn, sb + dy0);
  v[3] = buf_load<T>(bxn, sb + dy1);
  v[4] = buf_load<T>(bxn, sb + dz0);
  v[5] = buf_load<T>(bxn, sb + dz1);
  if constexpr (MODE == 2) {
    if (ok) {
      // parent cells of the neighbours on level 1 (the wrapped index on a
      // periodic axis; any in-range cell beyond a wall, whose term is
      // dropped)
      const int im = xm ? n0 - 1 : i - 1, ip = xp ? 0 : i + 1;
      const int jm = ym ? n1 - 1 : j - 1, jp = yp ? 0 : j + 1;
      const int km = zm ? n2 - 1 : k - 1, kp = zp ? 0 : k + 1;
      const int pj = (j >> 1) * cn0, pk = (k >> 1) * cn0 * cn1;
      const int pi = i >> 1;
      const int par6[6] = {(im >> 1) + pj + pk,       (ip >> 1) + pj + pk,       pi + (jm >> 1) * cn0 + pk,
                           pi + (jp >> 1) * cn0 + pk, pi + pj + (km >> 1) * cn0 * cn1,
                           pi + pj + (kp >> 1) * cn0 * cn1};
      const bool h[6] = {!xm || p0, !xp || p0, !ym || p1, !yp || p1, !zm || p2, !zp || p2};
      T e6[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) e6[e] = xc[par6[e]];
#pragma unroll
      for (int e = 0; e < 6; ++e) v[e] = h[e] ? v[e] + e6[e] : (T)0;
    }
  }
}

// One colour of a red-black Gauss-Seidel sweep of the 3D fine level: every
// cell of colour `color` takes its new value from the other colour's current
// values.  MODE 1: the other colour is zero (the first half-sweep of a
// V-cycle from a zero guess: no neighbour is read).  MODE 2: the other
// colour's values take the coarse-grid correction of their level-1 parent
// (the first post-smoothing half-sweep; the correction of this colour's own
// values is never needed, a Gauss-Seidel update does not read the old
// value).  Rows and the neighbour sum are formed as in the LDS sweeps, so
// each new value has the same bits as in a whole-grid half-sweep of the
// natural order.
//
// A wave takes 64 consecutive slots of one row (j, k): in the colour-split
// order the x-neighbours of slot s (cell i = 2 ih + par) are the other
// colour's slots s + par - 1 and s + par, the y- and z-neighbours s -+ hw
// and s -+ hw n1.  j, k and par are the same for the whole wave, so the y/z
// offsets and their boundary cases are scalar; only the first and last cell
// of a row wrap (periodic) or lose a neighbour (wall: it reads as 0).  A
// cell with a cut link or a wall side is queued in LDS and updated after
// the work-group's tiles (every cell of a half-sweep reads only the other
// colour, so the order is free): the tile loop then holds the constant-row
// update alone.  Six waves per SIMD leave the compiler 80 VGPRs, enough to
// keep a tile's loads in flight without spilling the row pointers.
template <typename T, int MODE>
__global__ __launch_bounds__(EBIT_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) void kb_half3(
    const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl, int color) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const Dims d = C.op.d;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int hw = (n0 + 1) >> 1;
  const int plane = hw * n1;
  const long long H = split_half(d);
  constexpr int TS = (int)sizeof(T);
  const BufRsrc bxo = buf_rsrc(C.z[0] + color * H, H * TS);
  const BufRsrc bxn = buf_rsrc(C.z[0] + (color ^ 1) * H, H * TS);
  const BufRsrc brv = buf_rsrc(C.rv + color * H, H * TS);
  const BufRsrc bfl = buf_rsrc(C.fs + color * H, H);
  const gptr<const T> xc = (gptr<const T>)(MODE == 2 ? (const T*)C.lx[1][0] : nullptr);
  const int cn0 = C.lev[1].d.n[0], cn1 = C.lev[1].d.n[1];
  // the per-phase constant row, formed once per work-group and read back
  // from LDS (kept out of the per-cell code, where the compiler would
  // otherwise divide again); the queue of cut and wall cells
  __shared__ RegularRow<T> srr;
  __shared__ int nq;
  __shared__ int queue[SP_TPB * SP_TX * SP_TY];
  if (threadIdx.x == 0) {
    srr = regular_row<T>(C.op);
    nq = 0;
  }
  __syncthreads();
  const RegularRow<T> rr = srr;
  const bool p0 = d.per[0], p1 = d.per[1], p2 = d.per[2];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gx = (hw + SP_TX - 1) / SP_TX, gy = (n1 + SP_TY - 1) / SP_TY;
  const int tiles = gx * gy * n2;
  const int t0 = xcd_tile(lb, nb) * SP_TPB, t1 = min(t0 + SP_TPB, tiles);
  // tile coordinates of the first tile, then stepped (the scalar unit is
  // shared by the CU's waves: no division per tile)
  int bx = t0 % gx, by = (t0 / gx) % gy, k = t0 / (gx * gy);
  const int Hb = (int)(H * TS);
  for (int tb = t0; tb < t1; ++tb) {
    if (tb > t0 && ++bx == gx) {
      bx = 0;
      if (++by == gy) {
        by = 0;
        ++k;
      }
    }
    const int j = by * SP_TY + wv;
    const int par = (color + j + k) & 1;
    const int ih = bx * SP_TX + lane;
    const int i = 2 * ih + par;
    const bool ok = j < n1 && ih < hw && i < n0;
    // lanes with no cell load whatever their offset reads (nothing is stored)
    const int s = hw * (j + n1 * k) + ih;
    const int sb = s * TS;
    const uint8_t f = __builtin_amdgcn_raw_buffer_load_b8(bfl, s, 0, 0);
    const T rc = buf_load<T>(brv, sb);
    T v[6];
    half3_nbrs<T, MODE>(bxn, Hb, n0, n1, n2, hw, plane, p0, p1, p2, i, j, k, par, ih, sb, ok, xc, cn0, cn1, v);
    if (!ok) continue;
    const bool wall = (!p0 && (i == 0 || i == n0 - 1)) || (!p1 && (j == 0 || j == n1 - 1)) ||
                      (!p2 && (k == 0 || k == n2 - 1));
    if ((f & F_CUT) || wall) {
      queue[atomicAdd(&nq, 1)] = s;
      continue;
    }
    const bool liq = (f & F_LIQ) != 0;
    T xs = (v[0] + v[1]) + (v[2] + v[3]);
    xs += v[4] + v[5];
    buf_store((rc + (liq ? rr.w1 : rr.w0) * xs) * (liq ? rr.inv1 : rr.inv0), bxo, sb);
  }
  __syncthreads();
  const int nqc = nq;
  if (nqc == 0) return;
  const FineOp& op = C.op;
  for (int q = threadIdx.x; q < nqc; q += blockDim.x) {
    const int s = queue[q];
    const int ih = s % hw, jk = s / hw;
    const int j = jk % n1, kk = jk / n1;
    const int par = (color + j + kk) & 1;
    const int i = 2 * ih + par;
    const int sb = s * TS;
    const uint8_t f = __builtin_amdgcn_raw_buffer_load_b8(bfl, s, 0, 0);
    const T rc = buf_load<T>(brv, sb);
    T v[6];
    half3_nbrs<T, MODE>(bxn, Hb, n0, n1, n2, hw, plane, p0, p1, p2, i, j, kk, par, ih, sb, true, xc, cn0, cn1, v);
    T diag, off[6], mass, rb = 0;
    fine_row<T>(op, i, j, kk, f, diag, off, mass, rb);
    T sum = rc - off[0] * v[0] - off[1] * v[1];
    sum -= off[2] * v[2] + off[3] * v[3];
    sum -= off[4] * v[4] + off[5] * v[5];
    buf_store(sum / diag, bxo, sb);
  }
}

// Residual + restriction of the 3D fine level in the colour-split order:
// after a pre-smoothing that ends with the black half-sweep only the red
// children carry a residual (even_child), r - A x with A's row as
// fine_row forms it; also clears the level-1 iterate.  One thread per
// coarse cell, in tiles of the coarse grid: a red child (i, j, k) of coarse
// cell ci is slot hw (j + n1 k) + ci of colour 0, so a wave's children are
// consecutive slots, and its black neighbours are read as in kb_half3
// (beyond a wall: 0).  The loads of the four children are issued together;
// a regular child (no cut link, no wall side) takes the per-phase constant
// row, the others fine_row in a second pass.
template <typename T>
__global__ __launch_bounds__(EBIT_BLOCK) void kb_fine_restrict_split(const SolveCase<T>* __restrict__ cs,
                                                                     const CaseCtl* __restrict__ ctl,
                                                                     WorkList wl) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const FineOp& op = C.op;
  const Dims d = op.d;
  const Dims cd = C.lev[1].d;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int hw = (n0 + 1) >> 1;
  const int plane = hw * n1;
  const long long H = split_half(d);
  constexpr int TS = (int)sizeof(T);
  const BufRsrc bz0 = buf_rsrc(C.z[0], H * TS);
  const BufRsrc bz1 = buf_rsrc(C.z[0] + H, H * TS);
  const BufRsrc brv = buf_rsrc(C.rv, H * TS);
  const BufRsrc bfl = buf_rsrc(C.fs, H);
  const int Hb = (int)(H * TS);
  const bool p0 = d.per[0], p1 = d.per[1], p2 = d.per[2];
  const RegularRow<T> rr = regular_row<T>(op);
  T* bc = C.lb[1];
  T* xcz = C.lx[1][0];
  const bool tail = C.lt == 1;
  const int tiles = split_tiles(cd.n[0], cd.n[1], cd.n[2]);
  const int t0 = xcd_tile(lb, nb) * SP_TPB_R, t1 = min(t0 + SP_TPB_R, tiles);
  for (int t = t0; t < t1; ++t) {
    int ci, cj, ck;
    split_tile(t, cd.n[0], cd.n[1], ci, cj, ck);
    if (ci >= cd.n[0] || cj >= cd.n[1]) continue;
    T r[4], v[4][6], zc[4];
    uint8_t f[4];
    bool ok[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      int di, dj, dk;
      even_child(ch, di, dj, dk);
      const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
      ok[ch] = i < n0 && j < n1 && k < n2;
      // a child beyond an odd length reads whatever its offset names (the
      // buffer bounds keep it inside) and is dropped
      const int sl = hw * (j + n1 * k) + ci;
      const int sb = sl * TS;
      f[ch] = __builtin_amdgcn_raw_buffer_load_b8(bfl, sl, 0, 0);
      r[ch] = buf_load<T>(brv, sb);
      zc[ch] = buf_load<T>(bz0, sb);
      half3_nbrs<T, 0>(bz1, Hb, n0, n1, n2, hw, plane, p0, p1, p2, i, j, k, (j + k) & 1, ci, sb, ok[ch], nullptr,
                       0, 0, v[ch]);
    }
    int slow = 0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      int di, dj, dk;
      even_child(ch, di, dj, dk);
      const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
      const bool wall = (!p0 && (i == 0 || i == n0 - 1)) || (!p1 && (j == 0 || j == n1 - 1)) ||
                        (!p2 && (k == 0 || k == n2 - 1));
      if (!ok[ch]) {
        r[ch] = (T)0;
      } else if ((f[ch] & F_CUT) || wall) {
        slow |= 1 << ch;
      } else {
        const bool liq = (f[ch] & F_LIQ) != 0;
        T xs = (v[ch][0] + v[ch][1]) + (v[ch][2] + v[ch][3]);
        xs += v[ch][4] + v[ch][5];
        r[ch] = r[ch] - (liq ? rr.dg1 : rr.dg0) * zc[ch] + (liq ? rr.w1 : rr.w0) * xs;
      }
    }
    if (slow) {
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        if (!(slow & (1 << ch))) continue;
        int di, dj, dk;
        even_child(ch, di, dj, dk);
        const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
        T diag, off[6], mass, rb = 0;
        fine_row<T>(op, i, j, k, f[ch], diag, off, mass, rb);
        T x = r[ch] - diag * zc[ch];
#pragma unroll
        for (int e = 0; e < 6; ++e) x -= off[e] * v[ch][e];
        r[ch] = x;
      }
    }
    const int I = ci + cd.n[0] * (cj + cd.n[1] * ck);
    bc[tail ? tail_el(cd, tail_half(cd), ci, cj, ck) : I] = (r[0] + r[1]) + (r[2] + r[3]);
    xcz[I] = (T)0;
  }
}

// the cell flags in the colour-split order (padding slots of odd n0: 0)
template <bool B>
__global__ void k_split_flags(Many<SplitArgs> m) {
  long long lb, nb;
  const SplitArgs& a = many_case<B>(m, lb, nb);
  const Dims& d = a.d;
  const uint8_t* __restrict__ flags = a.flags;
  uint8_t* __restrict__ fs = a.fs;
  const long long H = split_half(d);
  const int hw = (d.n[0] + 1) >> 1;
  for (long long t = lb * blockDim.x + threadIdx.x; t < 2 * H; t += nb * blockDim.x) {
    const int color = t >= H ? 1 : 0;
    const long long s = t - color * H;
    const int ih = (int)(s % hw);
    const long long jk = s / hw;
    const int j = (int)(jk % d.n[1]), k = (int)(jk / d.n[1]);
    const int i = 2 * ih + ((color + j + k) & 1);
    fs[t] = i < d.n[0] ? flags[i + (long long)d.n[0] * jk] : (uint8_t)0;
  }
}

// The six sides -x +x -y +y -z +z of cell (i, j, k) (offset q) of a 3D
// explicit level: the neighbour's coordinate along the side's axis (wrapped;
// across a wall it names a cell whose value is not used), its offset,
// whether the side couples (not across a wall, not along an axis of one
// cell) and the coupling (the lower side's is stored at the neighbour).
template <typename T>
struct CoarseSides {
  int nc[6], nq[6];
  bool has[6];
  T off[6];
};

template <typename T>
__device__ inline void coarse_sides(const CoarseOp<T>& op, const Dims& d, int i, int j, int k, int q,
                                    CoarseSides<T>& S) {
  const int ia[3] = {i, j, k}, ln[3] = {d.n[0], d.n[1], d.n[2]};
  const int st[3] = {1, d.n[0], d.n[0] * d.n[1]};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool one = ln[a] < 2;
    S.nc[2 * a] = ia[a] > 0 ? ia[a] - 1 : ln[a] - 1;
    S.nc[2 * a + 1] = ia[a] + 1 < ln[a] ? ia[a] + 1 : 0;
    S.nq[2 * a] = q + (S.nc[2 * a] - ia[a]) * st[a];
    S.nq[2 * a + 1] = q + (S.nc[2 * a + 1] - ia[a]) * st[a];
    S.has[2 * a] = !one && (ia[a] > 0 || d.per[a]);
    S.has[2 * a + 1] = !one && (ia[a] + 1 < ln[a] || d.per[a]);
  }
#pragma unroll
  for (int e = 0; e < 6; ++e)
    S.off[e] = S.has[e] ? ((e & 1) ? op.off[e >> 1][q] : op.off[e >> 1][S.nq[e]]) : (T)0;
}

// Half-sweep of an explicit 3D coarse level l in the natural order, in
// place on its iterate buffer 0: the cells of one colour ((i + j + k) & 1 ==
// color) take their Gauss-Seidel update from the other colour's values.
// One thread per slot (ih, j, k) of the colour (cell i = 2 ih + parity), so
// a wave covers 64 consecutive cells of the colour and every thread works
// alone: no barrier, all loads of a cell in flight together.  MODE 1: the
// other colour is zero (the first half-sweep from the zero guess: only b and
// the diagonal are read); MODE 2: the other colour's values take their
// level l+1 parent's correction (the first post-smoothing half-sweep; this
// colour's corrected values are never needed); MODE 0: plain.  Every axis
// that is periodic has even length (a same-colour neighbour across the seam
// would be read while it is written): the plan uses the LDS z-march kernel
// on the other levels.
template <typename T, int MODE>
__global__ __launch_bounds__(EBIT_BLOCK) void kb_chalf(const SolveCase<T>* __restrict__ cs,
                                                       const CaseCtl* __restrict__ ctl, WorkList wl, int l,
                                                       int color) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const CoarseOp<T>& op = C.lev[l];
  const Dims d = op.d;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const unsigned hw = (unsigned)(n0 + 1) >> 1;
  const unsigned slots = hw * (unsigned)n1 * (unsigned)n2;
  const T* __restrict__ b = C.lb[l];
  T* __restrict__ x = C.lx[l][0];
  const T* __restrict__ xc = MODE == 2 ? (const T*)C.lx[l + 1][0] : nullptr;
  const Dims cd = C.lev[l + 1].d;
  for (unsigned t = (unsigned)xcd_tile(lb, nb) * blockDim.x + threadIdx.x; t < slots;
       t += (unsigned)nb * blockDim.x) {
    const unsigned ih = t % hw, jk = t / hw;
    const int j = (int)(jk % (unsigned)n1), k = (int)(jk / (unsigned)n1);
    const int i = 2 * (int)ih + ((color + j + k) & 1);
    if (i >= n0) continue;
    const int q = i + n0 * (int)jk;
    CoarseSides<T> S;
    coarse_sides<T>(op, d, i, j, k, q, S);
    T v[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      v[e] = (T)0;
      if (MODE != 1 && S.has[e]) {
        v[e] = x[S.nq[e]];
        if (MODE == 2) {
          const int a = e >> 1;
          const int pi = a == 0 ? S.nc[e] : i, pj = a == 1 ? S.nc[e] : j, pk = a == 2 ? S.nc[e] : k;
          v[e] += xc[cell_index(cd, pi >> 1, pj >> 1, pk >> 1)];
        }
      }
    }
    T sum = b[q] - S.off[0] * v[0] - S.off[1] * v[1];
    sum -= S.off[2] * v[2] + S.off[3] * v[3];
    sum -= S.off[4] * v[4] + S.off[5] * v[5];
    x[q] = sum / op.diag[q];
  }
}

// Restricted residual of a 3D level smoothed by kb_chalf (iterate in buffer
// 0): after the black half-sweep only the red children carry a residual,
// summed in the order of even_child; also clears the level l+1 iterate.
// One thread per cell of level l+1, the loads of its four children issued
// together.
template <typename T>
__global__ __launch_bounds__(EBIT_BLOCK) void kb_chalf_restrict(const SolveCase<T>* __restrict__ cs,
                                                                const CaseCtl* __restrict__ ctl, WorkList wl,
                                                                int l) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const CoarseOp<T>& op = C.lev[l];
  const Dims d = op.d;
  const Dims cd = C.lev[l + 1].d;
  const T* __restrict__ b = C.lb[l];
  const T* __restrict__ x = C.lx[l][0];
  T* bc = C.lb[l + 1];
  T* xcz = C.lx[l + 1][0];
  const bool tail = C.lt == l + 1;
  const unsigned cn0 = (unsigned)cd.n[0], cn1 = (unsigned)cd.n[1];
  const unsigned ncell = cn0 * cn1 * (unsigned)cd.n[2];
  for (unsigned I = (unsigned)xcd_tile(lb, nb) * blockDim.x + threadIdx.x; I < ncell;
       I += (unsigned)nb * blockDim.x) {
    const unsigned cjk = I / cn0;
    const int ci = (int)(I - cjk * cn0), cj = (int)(cjk % cn1), ck = (int)(cjk / cn1);
    T r[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      int di, dj, dk;
      even_child(ch, di, dj, dk);
      const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
      r[ch] = (T)0;
      if (i < d.n[0] && j < d.n[1] && k < d.n[2]) {
        const int q = i + d.n[0] * (j + d.n[1] * k);
        CoarseSides<T> S;
        coarse_sides<T>(op, d, i, j, k, q, S);
        T v[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = S.has[e] ? x[S.nq[e]] : (T)0;
        T sum = b[q] - op.diag[q] * x[q] - S.off[0] * v[0] - S.off[1] * v[1];
        sum -= S.off[2] * v[2] + S.off[3] * v[3];
        sum -= S.off[4] * v[4] + S.off[5] * v[5];
        r[ch] = sum;
      }
    }
    bc[tail ? tail_el(cd, tail_half(cd), ci, cj, ck) : I] = (r[0] + r[1]) + (r[2] + r[3]);
    xcz[I] = (T)0;
  }
}

// the same from explicit level l to level l + 1
template <typename T>
__global__ void kb_coarse_restrict(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl,
                                   int l, int src_sel) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  if (!ctl[c].active) return;
  const SolveCase<T>& C = cs[c];
  const CoarseOp<T> op = C.lev[l];
  const Dims cd = C.lev[l + 1].d;
  const T* b = C.lb[l];
  const T* x = C.lx[l][src_sel];
  T* bc = C.lb[l + 1];
  T* xc = C.lx[l + 1][0];
  const int nch = op.d.dim == 3 ? 4 : 2;
  CASE_STRIDE(I, cd.N) {
    int ci, cj, ck;
    cell_ijk(cd, I, ci, cj, ck);
    T sum = 0;
    for (int ch = 0; ch < nch; ++ch) {
      int di, dj, dk;
      even_child(ch, di, dj, dk);
      const int i = 2 * ci + di, j = 2 * cj + dj, k = 2 * ck + dk;
      if (i < op.d.n[0] && j < op.d.n[1] && k < op.d.n[2]) {
        const long long q = cell_index(op.d, i, j, k);
        sum += b[q] - op.diag[q] * x[q] - coarse_offsum<T>(op, i, j, k, q, x);
      }
    }
    bc[C.lt == l + 1 ? tail_el(cd, tail_half(cd), ci, cj, ck) : I] = sum;
    xc[I] = (T)0;
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(EBIT_TAIL_THREADS) void kb_tail(const SolveCase<T>* __restrict__ cs,
                                                             const CaseCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char tail_smem[];
  const int c = blockIdx.x;
  if (!ctl[c].active) return;
  tail_body<T, DIM>(cs[c].tail, reinterpret_cast<T*>(tail_smem));
}

// z.r and, unless the recurrence restarts, z.q (q = A p of the previous iteration)
template <typename T>
__global__ void kb_dots(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl, int dc) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  if (C.ndot > 0) return;  // formed by the last fine sweep
  const bool first = dc || cc.fresh;
  const T* z = C.z[0];
  const double* r = C.r;
  const double* q = C.q;
  const long long H = C.split ? split_half(C.op.d) : 0;
  double v[2] = {0, 0};
  CASE_STRIDE(i, C.op.d.N) {
    long long zi = i;
    if (C.split) {
      int ci, cj, ck;
      cell_ijk(C.op.d, i, ci, cj, ck);
      zi = split_index(C.op.d, H, ci, cj, ck);
    }
    const double zc = (double)z[zi];
    v[0] += zc * r[i];
    if (!first) v[1] += zc * q[i];
  }
  write_partials<2>(v, C.partial, lb, nb);
}

// End of an outer iteration, given r.r: record it, count the iteration,
// flip the direction slot, clear the restart and pending flags, and stop
// the case once r.r reaches its stop level (or is not finite).
__device__ inline void end_iteration(Scal* sc, CaseCtl* ctl, const CaseCtl& cc, double rr) {
  sc->rr = rr;
  sc->iters += 1;
  CaseCtl n = cc;
  n.fresh = 0;
  n.pend = 0;
  n.pi = cc.pi ^ 1;
  if (rr <= cc.stop2) {
    n.active = 0;
    n.recheck = 1;  // its true residual is formed at the end of the block
  }
  if (!isfinite(rr)) {
    sc->err |= ERR_NAN;
    n.active = 0;
  }
  *ctl = n;
}

// gamma = z.r and beta from the dots' partials, then p_new = z + beta p_old,
// q = A p_new, partial p.q (row 2).  Every block reduces the partials itself,
// in the same fixed order, so no separate reduction launch is needed; block
// 0 records gamma in the slot of this iteration's parity.  Compiled per
// system (SYS) and cell-offset width (I: int below 2^30 cells): the loop is
// bound by the latency of its gathers, and a row that carries one system's
// terms with 32-bit offsets needs fewer registers, so more waves are in
// flight.
template <typename I>
__device__ inline void fine_nbrs_t(const Dims& d, int i, int j, int k, I c, I (&m)[6]) {
  const I s1 = d.n[0], s2 = (I)d.n[0] * d.n[1], N = (I)d.N;
  m[0] = i > 0 ? c - 1 : c - 1 + s1;
  m[1] = i + 1 < d.n[0] ? c + 1 : c + 1 - s1;
  m[2] = j > 0 ? c - s1 : c - s1 + s2;
  m[3] = j + 1 < d.n[1] ? c + s1 : c + s1 - s2;
  m[4] = k > 0 ? c - s2 : c - s2 + N;
  m[5] = k + 1 < d.n[2] ? c + s2 : c + s2 - N;
}

template <typename T, int SYS, typename I>
__global__ void kb_p_update_apply(const SolveCase<T>* __restrict__ cs, const CaseCtl* __restrict__ ctl, WorkList wl,
                                  int dc) {
  __shared__ double sbeta;
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  const bool first = dc || cc.fresh;
  {
    double g[3];
    reduce_partials(C.partial, C.ndot > 0 ? C.ndot : nb, 2, false, g);
    if (threadIdx.x == 0) {
      Scal* sc = C.sc;
      const int so = cc.pi, sn = cc.pi ^ 1;
      const double beta = first ? 0.0 : -sc->sa[so] * g[1] / sc->sg[so];
      sbeta = beta;
      if (lb == 0) {
        sc->sg[sn] = g[0];
        sc->gamma = g[0];
        sc->beta = beta;
        sc->zq = g[1];
      }
    }
    __syncthreads();
  }
  const double beta = sbeta;
  const T* z = C.z[0];
  const double* p_old = C.p[cc.pi];
  double* p_new = C.p[cc.pi ^ 1];
  double* q = C.q;
  const long long HS = C.split ? split_half(op.d) : 0;
  double v[1] = {0};
  const I N = (I)op.d.N, stride = (I)nb * (I)blockDim.x;
  for (I i0 = (I)xcd_tile(lb, nb) * (I)blockDim.x + (I)threadIdx.x; i0 < N; i0 += stride) {
    int i, j, k;
    cell_ijk(op.d, i0, i, j, k);
    // the direction at the cell and its neighbours, loaded before the row
    // is assembled (see fine_nbrs)
    I m[6];
    fine_nbrs_t<I>(op.d, i, j, k, i0, m);
    // z of a cell: natural order, or the colour-split order (3D)
    auto zat = [&](I mm) -> double {
      if (!C.split) return (double)z[mm];
      int ci, cj, ck;
      cell_ijk(op.d, (long long)mm, ci, cj, ck);
      return (double)z[split_index(op.d, HS, ci, cj, ck)];
    };
    double pn[6];
#pragma unroll
    for (int qq = 0; qq < 6; ++qq)
      pn[qq] = qq < 2 * op.d.dim ? (first ? zat(m[qq]) : zat(m[qq]) + beta * p_old[m[qq]]) : 0.0;
    const double pc = first ? zat(i0) : zat(i0) + beta * p_old[i0];
    double diag, off[6], mass, rb = 0, mx;
    fine_row<double, SYS>(op, i, j, k, op.flags[i0], diag, off, mass, rb, &mx);
    double s = mx * pc;
#pragma unroll
    for (int qq = 0; qq < 6; ++qq)
      if (qq < 2 * op.d.dim && off[qq] != 0.0) s -= off[qq] * (pc - pn[qq]);
    p_new[i0] = pc;
    q[i0] = s;
    v[0] += pc * s;
  }
  write_partials<1>(v, C.partial + 2 * nb, lb, nb);
}

// The same p-update + A p on a 3D grid, with the new direction staged in
// LDS: a work-group takes 64 x 4 tiles (one cell per thread) and marches
// each along a chunk of z-planes.  Each plane's direction p = z + beta p_old
// is formed once on its tile and 1-cell ring, in coalesced loads issued one
// plane ahead, and the rows read their six neighbours from the staged planes
// instead of gathering fourteen values per cell; a cell with no cut link and
// no wall side takes its phase's constant row.  p_new, q and every row are
// the same bits as in the strided kernel; only the partial sums of p.q group
// the cells differently (still in a fixed order).  A work-group takes units
// (tile, chunk) lb, lb + nb, ... with the chunk doubled until there are at
// most nb units, so the partial row keeps nb entries.  In-plane offsets are
// 32-bit: grids of 2^30 cells or more take the strided kernel.
#define AP_TX 64
#define AP_TY 4
#define AP_QX (AP_TX + 2)
#define AP_QL (AP_QX * (AP_TY + 2))
#define AP_NQ ((AP_QL + RB_THREADS - 1) / RB_THREADS)
#define AP_NW ((AP_TX * AP_TY + RB_THREADS - 1) / RB_THREADS)

// z is in the colour-split order when H > 0: the window cell of offset
// qo[e] (i + n0 j) sits at slot zo[e] ((i >> 1) + hw j) of its plane, in the
// half of colour (zp[e] + k) & 1
template <typename T>
__device__ inline void ap_load(const Dims& d, const int (&qo)[AP_NQ], const int (&zo)[AP_NQ], const int (&zp)[AP_NQ],
                               long long H, int kk, bool first, double beta, const T* __restrict__ z,
                               const double* __restrict__ p_old, double (&v)[AP_NQ]) {
  int k = kk;
  const bool pz = wrap_axis(d, 2, k);
  const long long base = (long long)k * d.n[0] * d.n[1];
  const long long zbase = (long long)k * ((d.n[0] + 1) / 2) * d.n[1];
#pragma unroll
  for (int e = 0; e < AP_NQ; ++e) {
    v[e] = 0.0;
    if (pz && qo[e] >= 0) {
      const long long m = base + qo[e];
      const long long mz = H ? ((zp[e] + k) & 1) * H + zbase + zo[e] : m;
      v[e] = first ? (double)z[mz] : (double)z[mz] + beta * p_old[m];
    }
  }
}

__device__ inline void ap_store(const double (&v)[AP_NQ], double* ps) {
#pragma unroll
  for (int e = 0; e < AP_NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    if (t < AP_QL) ps[t] = v[e];
  }
}

template <typename T, int SYS>
__global__ __launch_bounds__(RB_THREADS) void kb_apply3d(const SolveCase<T>* __restrict__ cs,
                                                         const CaseCtl* __restrict__ ctl, WorkList wl, int dc) {
  __shared__ double ps[4][AP_QL];
  __shared__ double sbeta;
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  const bool first = dc || cc.fresh;
  {
    double g[3];
    reduce_partials(C.partial, C.ndot > 0 ? C.ndot : nb, 2, false, g);
    if (threadIdx.x == 0) {
      Scal* sc = C.sc;
      const int so = cc.pi, sn = cc.pi ^ 1;
      const double beta = first ? 0.0 : -sc->sa[so] * g[1] / sc->sg[so];
      sbeta = beta;
      if (lb == 0) {
        sc->sg[sn] = g[0];
        sc->gamma = g[0];
        sc->beta = beta;
        sc->zq = g[1];
      }
    }
    __syncthreads();
  }
  const double beta = sbeta;
  const Dims& d = op.d;
  const T* z = C.z[0];
  const long long HS = C.split ? split_half(d) : 0;
  const double* p_old = C.p[cc.pi];
  double* p_new = C.p[cc.pi ^ 1];
  double* q = C.q;
  const int gx = (d.n[0] + AP_TX - 1) / AP_TX, gy = (d.n[1] + AP_TY - 1) / AP_TY;
  int zc = C.fzc;
  while (zc < d.n[2] && (long long)gx * gy * ((d.n[2] + zc - 1) / zc) > nb) zc *= 2;
  const int units = gx * gy * ((d.n[2] + zc - 1) / zc);
  double v[1] = {0};
  for (int ut = xcd_tile(lb, nb); ut < units; ut += nb) {
    const int bx = ut % gx, by = (ut / gx) % gy, bz = ut / (gx * gy);
    const int tx0 = bx * AP_TX, ty0 = by * AP_TY;
    const int z0 = bz * zc, z1 = min(z0 + zc, d.n[2]);
    // plane-invariant offsets: the staged window (tile + 1 ring, -1 outside
    // the domain) and this thread's tile cells (-1 outside the domain)
    int qo[AP_NQ], zo[AP_NQ], zp[AP_NQ], wo[AP_NW], wq[AP_NW], wi[AP_NW], wj[AP_NW];
#pragma unroll
    for (int e = 0; e < AP_NQ; ++e) {
      const int t = threadIdx.x + e * RB_THREADS;
      qo[e] = -1;
      zo[e] = 0;
      zp[e] = 0;
      if (t >= AP_QL) continue;
      int i = tx0 + t % AP_QX - 1, j = ty0 + t / AP_QX - 1;
      if (wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
        qo[e] = i + d.n[0] * j;
        zo[e] = (i >> 1) + ((d.n[0] + 1) / 2) * j;
        zp[e] = (i + j) & 1;
      }
    }
#pragma unroll
    for (int w = 0; w < AP_NW; ++w) {
      const int t = threadIdx.x + w * RB_THREADS;
      const int lx = t % AP_TX, ly = t / AP_TX;
      wi[w] = tx0 + lx;
      wj[w] = ty0 + ly;
      wq[w] = (ly + 1) * AP_QX + (lx + 1);
      wo[w] = (t < AP_TX * AP_TY && wi[w] < d.n[0] && wj[w] < d.n[1]) ? wi[w] + d.n[0] * wj[w] : -1;
    }
    const long long pl = (long long)d.n[0] * d.n[1];
    double pa[AP_NQ];
    // four plane slots: the store of plane k+1 goes to the slot plane k-3
    // had, which no wave reads after the previous plane's barrier, so one
    // barrier per plane suffices (the last plane of a unit ends with a
    // second one before the next unit's stores)
    ap_load<T>(d, qo, zo, zp, HS, z0 - 1, first, beta, z, p_old, pa);
    ap_store(pa, ps[(z0 + 3) & 3]);
    ap_load<T>(d, qo, zo, zp, HS, z0, first, beta, z, p_old, pa);
    ap_store(pa, ps[z0 & 3]);
    ap_load<T>(d, qo, zo, zp, HS, z0 + 1, first, beta, z, p_old, pa);
    for (int k = z0; k < z1; ++k) {
      // plane k+1 joins planes k-1 and k
      ap_store(pa, ps[(k + 1) & 3]);
      __syncthreads();
      if (k + 1 < z1) ap_load<T>(d, qo, zo, zp, HS, k + 2, first, beta, z, p_old, pa);
      const double* pm = ps[(k + 3) & 3];
      const double* p0 = ps[k & 3];
      const double* pp = ps[(k + 1) & 3];
      const long long base = (long long)k * pl;
#pragma unroll
      for (int w = 0; w < AP_NW; ++w) {
        if (wo[w] < 0) continue;
        const int e = wq[w];
        const long long i0 = base + wo[w];
        // neighbours in the order of fine_nbrs: -x, +x, -y, +y, -z, +z
        const double pn[6] = {p0[e - 1], p0[e + 1], p0[e - AP_QX], p0[e + AP_QX], pm[e], pp[e]};
        const double pc = p0[e];
        const uint8_t f = op.flags[i0];
        double s;
        if (!(f & F_CUT) && (d.per[0] || (wi[w] > 0 && wi[w] + 1 < d.n[0])) &&
            (d.per[1] || (wj[w] > 0 && wj[w] + 1 < d.n[1])) && (d.per[2] || (k > 0 && k + 1 < d.n[2]))) {
          // no cut link, no wall side: the phase's constant row, with the
          // mass and couplings fine_row gives, in its order (the same bits)
          const bool liq = (f & F_LIQ) != 0;
          const double cw = -(liq ? op.coef[1] : op.coef[0]) * op.ih2;
          s = (liq ? op.mass[1] : op.mass[0]) * pc;
          if (cw != 0.0) {
#pragma unroll
            for (int qq = 0; qq < 6; ++qq) s -= cw * (pc - pn[qq]);
          }
        } else {
          double diag, off[6], mass, rb = 0, mx;
          fine_row<double, SYS>(op, wi[w], wj[w], k, f, diag, off, mass, rb, &mx);
          s = mx * pc;
#pragma unroll
          for (int qq = 0; qq < 6; ++qq)
            if (off[qq] != 0.0) s -= off[qq] * (pc - pn[qq]);
        }
        p_new[i0] = pc;
        q[i0] = s;
        v[0] += pc * s;
      }
    }
    __syncthreads();
  }
  write_partials<1>(v, C.partial + 2 * nb, lb, nb);
}

// 3D grids whose fine iterate is in the colour-split order: the p-update and
// A p as two streaming passes (they replace kb_apply3d there).
//
// kb_p_update3: gamma = z.r and beta from the dots' partials (every block
// reduces them in the same fixed order; block 0 records gamma), then
// p_new = z + beta p_old over the natural order.  A wave takes 64
// consecutive cells of a row; z is read through the colour-split order.
#define PU_TPB 8
template <typename T>
__global__ __launch_bounds__(EBIT_BLOCK) void kb_p_update3(const SolveCase<T>* __restrict__ cs,
                                                           const CaseCtl* __restrict__ ctl, WorkList wl, int dc) {
  __shared__ double sbeta;
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  const bool first = dc || cc.fresh;
  {
    double g[3];
    reduce_partials(C.partial, C.ndot > 0 ? C.ndot : C.nred, 2, false, g);
    if (threadIdx.x == 0) {
      Scal* sc = C.sc;
      const int so = cc.pi, sn = cc.pi ^ 1;
      const double beta = first ? 0.0 : -sc->sa[so] * g[1] / sc->sg[so];
      sbeta = beta;
      if (lb == 0) {
        sc->sg[sn] = g[0];
        sc->gamma = g[0];
        sc->beta = beta;
        sc->zq = g[1];
      }
    }
    __syncthreads();
  }
  const double beta = sbeta;
  const Dims& d = C.op.d;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int hw = (n0 + 1) >> 1;
  const long long H = split_half(d);
  constexpr int TS = (int)sizeof(T);
  const BufRsrc bz0 = buf_rsrc(C.z[0], H * TS);
  const BufRsrc bz1 = buf_rsrc(C.z[0] + H, H * TS);
  const BufRsrc bpo = buf_rsrc(C.p[cc.pi], d.N * 8);
  const BufRsrc bpn = buf_rsrc(C.p[cc.pi ^ 1], d.N * 8);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gx = (n0 + SP_TX - 1) / SP_TX, gy = (n1 + SP_TY - 1) / SP_TY;
  const int tiles = gx * gy * n2;
  const int t0 = xcd_tile(lb, nb) * PU_TPB, t1 = min(t0 + PU_TPB, tiles);
  int bx = t0 % gx, by = (t0 / gx) % gy, k = t0 / (gx * gy);
  // every tile's loads are issued before the first store (the stores could
  // alias the loads, so the compiler would otherwise wait per tile)
  int cnv[PU_TPB];
  bool okv[PU_TPB];
  T zv[PU_TPB];
  double pov[PU_TPB];
#pragma unroll
  for (int u = 0; u < PU_TPB; ++u) {
    if (u > 0 && ++bx == gx) {
      bx = 0;
      if (++by == gy) {
        by = 0;
        ++k;
      }
    }
    const int j = by * SP_TY + wv;
    const int i = bx * SP_TX + lane;
    okv[u] = t0 + u < t1 && j < n1 && i < n0;
    const int cn = okv[u] ? i + n0 * (j + n1 * k) : 0;
    const int zs = okv[u] ? (i >> 1) + hw * (j + n1 * k) : 0;
    cnv[u] = cn;
    zv[u] = ((i + j + k) & 1) ? buf_load<T>(bz1, zs * TS) : buf_load<T>(bz0, zs * TS);
    pov[u] = first ? 0.0 : buf_load<double>(bpo, cn * 8);
  }
#pragma unroll
  for (int u = 0; u < PU_TPB; ++u)
    if (okv[u]) buf_store(first ? (double)zv[u] : (double)zv[u] + beta * pov[u], bpn, cnv[u] * 8);
}

// kb_apply_q3: q = A p_new with p_new read at the cell and its six
// neighbours (cache hits but the cell's own), and the partial sums of p.q
// (row 2, one per reduction work-group: this kernel runs on the reduction
// work list).  Rows as in kb_apply3d: a cell with no cut link and no wall
// side takes its phase's constant row, the others fine_row; the same bits.
template <typename T, int SYS>
__global__ __launch_bounds__(EBIT_BLOCK) void kb_apply_q3(const SolveCase<T>* __restrict__ cs,
                                                          const CaseCtl* __restrict__ ctl, WorkList wl) {
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  const FineOp op = C.op;
  const Dims& d = op.d;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int pl = n0 * n1;
  const BufRsrc bp = buf_rsrc(C.p[cc.pi ^ 1], d.N * 8);
  const BufRsrc bq = buf_rsrc(C.q, d.N * 8);
  const BufRsrc bf = buf_rsrc(op.flags, d.N);
  const bool p0 = d.per[0], p1 = d.per[1], p2 = d.per[2];
  // the phases' constant rows (kept out of the per-cell code)
  __shared__ double srow[4];
  if (threadIdx.x == 0) {
    srow[0] = op.mass[0];
    srow[1] = op.mass[1];
    srow[2] = -op.coef[0] * op.ih2;
    srow[3] = -op.coef[1] * op.ih2;
  }
  __syncthreads();
  const double m0 = srow[0], m1 = srow[1], cw0 = srow[2], cw1 = srow[3];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gx = (n0 + SP_TX - 1) / SP_TX, gy = (n1 + SP_TY - 1) / SP_TY;
  const int tiles = gx * gy * n2;
  const int tpb = (tiles + nb - 1) / nb;
  const int t0 = xcd_tile(lb, nb) * tpb, t1 = min(t0 + tpb, tiles);
  double v[1] = {0};
  constexpr int U = 2;  // tiles whose loads are issued before any store
  int bx = t0 % gx, by = (t0 / gx) % gy, k = t0 / (gx * gy);
  for (int tb = t0; tb < t1; tb += U) {
    int cnv[U], iv[U], jv[U], kv[U];
    bool okv[U];
    uint8_t fv[U];
    double pcv[U], pnv[U][6];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (tb + u > t0 && ++bx == gx) {
        bx = 0;
        if (++by == gy) {
          by = 0;
          ++k;
        }
      }
      const int j = by * SP_TY + wv;
      const int i = bx * SP_TX + lane;
      const bool ok = tb + u < t1 && j < n1 && i < n0;
      const int cn = ok ? i + n0 * (j + n1 * k) : 0;
      okv[u] = ok;
      cnv[u] = cn;
      iv[u] = i;
      jv[u] = j;
      kv[u] = k;
      const bool xm = i == 0, xp = i == n0 - 1, ym = j == 0, yp = j == n1 - 1, zm = k == 0, zp = k == n2 - 1;
      // neighbours in the order of fine_nbrs: -x, +x, -y, +y, -z, +z (the
      // wrapped cell on a periodic axis; the cell itself beyond a wall, where
      // the row has no coupling)
      int q[6];
      q[0] = xm ? (p0 ? cn + n0 - 1 : cn) : cn - 1;
      q[1] = xp ? (p0 ? cn - n0 + 1 : cn) : cn + 1;
      q[2] = ym ? (p1 ? cn + pl - n0 : cn) : cn - n0;
      q[3] = yp ? (p1 ? cn - pl + n0 : cn) : cn + n0;
      q[4] = zm ? (p2 ? cn + pl * (n2 - 1) : cn) : cn - pl;
      q[5] = zp ? (p2 ? cn - pl * (n2 - 1) : cn) : cn + pl;
      if (!ok) {
#pragma unroll
        for (int e = 0; e < 6; ++e) q[e] = 0;
      }
      fv[u] = __builtin_amdgcn_raw_buffer_load_b8(bf, cn, 0, 0);
      pcv[u] = buf_load<double>(bp, cn * 8);
#pragma unroll
      for (int e = 0; e < 6; ++e) pnv[u][e] = buf_load<double>(bp, q[e] * 8);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!okv[u]) continue;
      const int i = iv[u], j = jv[u], k2 = kv[u];
      const uint8_t f = fv[u];
      const double pc = pcv[u];
      const bool xm = i == 0, xp = i == n0 - 1, ym = j == 0, yp = j == n1 - 1, zm = k2 == 0, zp = k2 == n2 - 1;
      double sq;
      if (!(f & F_CUT) && (p0 || (!xm && !xp)) && (p1 || (!ym && !yp)) && (p2 || (!zm && !zp))) {
        const bool liq = (f & F_LIQ) != 0;
        const double cw = liq ? cw1 : cw0;
        sq = (liq ? m1 : m0) * pc;
        if (cw != 0.0) {
#pragma unroll
          for (int qq = 0; qq < 6; ++qq) sq -= cw * (pc - pnv[u][qq]);
        }
      } else {
        double diag, off[6], mass, rb = 0, mx;
        fine_row<double, SYS>(op, i, j, k2, f, diag, off, mass, rb, &mx);
        sq = mx * pc;
#pragma unroll
        for (int qq = 0; qq < 6; ++qq)
          if (off[qq] != 0.0) sq -= off[qq] * (pc - pnv[u][qq]);
      }
      buf_store(sq, bq, cnv[u] * 8);
      v[0] += pc * sq;
    }
  }
  write_partials<1>(v, C.partial + 2 * nb, lb, nb);
}

// alpha = gamma / (p.q) from the p-update's partials (every block, fixed
// order), then x += alpha p, r -= alpha q, partial r.r (row 3).
template <typename T>
__global__ void kb_update_xr(const SolveCase<T>* __restrict__ cs, CaseCtl* __restrict__ ctl, WorkList wl, int pend) {
  __shared__ double salpha;
  int lb, nb;
  const int c = wl_find(wl, lb, nb);
  const CaseCtl cc = ctl[c];
  if (!cc.active) return;
  const SolveCase<T>& C = cs[c];
  {
    double dlt[3];
    reduce_partials(C.partial + 2 * nb, nb, 1, false, dlt);
    if (threadIdx.x == 0) {
      Scal* sc = C.sc;
      const int sn = cc.pi ^ 1;
      const double alpha = sc->sg[sn] / dlt[0];
      salpha = alpha;
      if (lb == 0) {
        sc->sa[sn] = alpha;
        sc->alpha = alpha;
        sc->delta = dlt[0];
      }
    }
    __syncthreads();
  }
  const double alpha = salpha;
  const double* p = C.p[cc.pi ^ 1];
  const double* q = C.q;
  double* x = C.x;
  double* r = C.r;
  T* rv = C.rv;
  const long long H = C.split ? split_half(C.op.d) : 0;
  double v[1] = {0};
  CASE_STRIDE(i, C.op.d.N) {
    x[i] += alpha * p[i];
    const double rc = r[i] - alpha * q[i];
    r[i] = rc;
    // the V-cycle's copy of r (rounded once to FP32 in mixed precision;
    // in the colour-split order in 3D)
    if (C.split) {
      int ci, cj, ck;
      cell_ijk(C.op.d, i, ci, cj, ck);
      rv[split_index(C.op.d, H, ci, cj, ck)] = (T)rc;
    } else if constexpr (!std::is_same<T, double>::value) {
      rv[i] = (T)rc;
    }
    v[0] += rc * rc;
  }
  write_partials<1>(v, C.partial + 3 * nb, lb, nb);
  // the r.r partials are taken by the next V-cycle's first launch (no
  // other field of the control word changes here)
  if (pend && lb == 0 && threadIdx.x == 0) ctl[c].pend = 1;
}

// One block per case: reduce its partials (nv rows from row `row`).
// FIN_INIT records b.b, r.r and the floor norm; FIN_RR ends an iteration:
// the direction slot flips, the restart flag clears, the iteration count
// advances, and the case stops (active = 0) once r.r <= stop2 or on NaN/Inf.
template <typename T>
__global__ void kb_finalize(const SolveCase<T>* __restrict__ cs, CaseCtl* __restrict__ ctl, int kind, int nv,
                            int row, int mask, double rtol2) {
  const int c = blockIdx.x;
  const CaseCtl cc = ctl[c];
  if (!selected(cc, mask)) return;
  if (kind == FIN_PEND && !cc.pend) return;
  const SolveCase<T>& C = cs[c];
  double v[3];
  reduce_partials(C.partial + row * C.nred, C.nred, nv, false, v);
  if (threadIdx.x != 0) return;
  Scal* sc = C.sc;
  bool bad = false;
  if (kind == FIN_START) {
    // the start of a solve clears the case's scalars
    int* w = reinterpret_cast<int*>(sc);
    for (int t = 0; t < (int)(sizeof(Scal) / sizeof(int)); ++t) w[t] = 0;
  }
  if (kind == FIN_INIT || kind == FIN_START) {
    sc->bb = v[0];
    sc->rr = v[1];
    sc->aa = v[2];
    bad = !isfinite(v[0]) || !isfinite(v[1]);
    if (kind == FIN_START) {
      // the start of a solve: b = 0 gives x = 0; a residual already at
      // rtol |b| stops before the first iteration (and is confirmed like
      // any other stop); otherwise iterate down to rtol^2 |b|^2
      CaseCtl n{0, 1, 0, 0, 0, 0, rtol2 * v[0]};
      if (v[0] == 0.0)
        n.recheck = 2;
      else if (!(v[1] <= n.stop2))
        n.active = 1;
      else
        n.recheck = 1;
      ctl[c] = n;
    }
  } else {
    end_iteration(sc, ctl + c, cc, v[0]);
  }
  if (bad) {
    sc->err |= ERR_NAN;
    ctl[c].active = 0;
  }
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + EBIT_BLOCK - 1) / EBIT_BLOCK); }

}  // namespace ebit

using namespace ebit;

extern "C" {

hipError_t ebit_launch_split_flags(const Dims* d, const uint8_t* flags, uint8_t* fsplit, hipStream_t st) {
  const long long n = 2 * split_half(*d);
  SplitArgs a;
  a.d = *d;
  a.flags = flags;
  a.fs = fsplit;
  hipLaunchKernelGGL(k_split_flags<false>, dim3(nblk(n)), dim3(EBIT_BLOCK), 0, st, many_one(a));
  return hipGetLastError();
}

hipError_t ebit_launch_fill_f64(long long n, double* x, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<double>, dim3(nblk(n)), dim3(EBIT_BLOCK), 0, st, n, x, v);
  return hipGetLastError();
}
hipError_t ebit_launch_fill_f32(long long n, float* x, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<float>, dim3(nblk(n)), dim3(EBIT_BLOCK), 0, st, n, x, v);
  return hipGetLastError();
}

// The build plan of a context: the first level built by the one-work-group
// kernel (>= 2; levels of at most EBIT_BUILD_SMALL cells go there) and the
// per-system tables it reads (host copies; the caller uploads them).
#define EBIT_BUILD_SMALL 1024
void ebit_build_tables(const EbitLevelHost* lv, int nlev, int want32, void* host_tabs) {
  BuildTable* tab = (BuildTable*)host_tabs;
  int ls = nlev;
  for (int l = 2; l < nlev; ++l)
    if (lv[l].d.N <= EBIT_BUILD_SMALL) {
      ls = l;
      break;
    }
  int dl = -1;
  for (int l = 1; l < nlev; ++l)
    if (lv[l].inv64[0]) dl = l;
  for (int sys = 0; sys < 2; ++sys) {
    BuildTable& t = tab[sys];
    memset(&t, 0, sizeof(t));
    t.ls = ls;
    t.nlev = nlev;
    t.dl = dl;
    for (int l = 0; l < nlev; ++l) {
      t.d[l] = lv[l].d;
      if (l == 0) continue;
      t.diag[l] = lv[l].diag64[sys];
      t.mass[l] = lv[l].mass64[sys];
      t.d32[l] = want32 ? lv[l].diag32[sys] : nullptr;
      t.i32[l] = want32 ? lv[l].img32[sys] : nullptr;
      t.i64[l] = lv[l].img64[sys];
      for (int a = 0; a < 3; ++a) {
        const bool on = a < lv[l].d.dim;
        t.off[l][a] = on ? lv[l].off64[sys][a] : nullptr;
        t.o32[l][a] = (on && want32) ? lv[l].off32[sys][a] : nullptr;
      }
    }
    if (dl >= 0) {
      t.inv64 = lv[dl].inv64[sys];
      t.inv32 = want32 ? lv[dl].inv32[sys] : nullptr;
      t.inv_ok = lv[dl].inv_ok + sys;
    }
  }
}

size_t ebit_build_table_bytes(void) { return 2 * sizeof(BuildTable); }

// Build both systems' coarse hierarchies: level 1 from the matrix-free fine
// operators, the larger levels one launch each, the small ones (and the
// dense inverse) in one work-group per system; FP32 copies written with
// the FP64 values when wanted.
// The launched levels of a hierarchy build (levels 1 .. ls-1): level 1 from
// the fine operators, the others each from the level above.  Returns how
// many levels past the first were described.
int ebit_build_args(const FineOp* op, const EbitLevelHost* lv, int nlev, int want32, int ls, BuildFineArgs* fine,
                    BuildCoarseArgs* coarse) {
  int nc = 0;
  for (int l = 1; l < ls && l < nlev; ++l) {
    BuildOut o[2];
    CoarseOp<double> f[2];
    memset(o, 0, sizeof(o));
    memset(f, 0, sizeof(f));
    for (int sys = 0; sys < 2; ++sys) {
      o[sys].cd = lv[l].d;
      o[sys].diag = lv[l].diag64[sys];
      o[sys].mass = lv[l].mass64[sys];
      o[sys].d32 = want32 ? lv[l].diag32[sys] : nullptr;
      o[sys].i32 = want32 ? lv[l].img32[sys] : nullptr;
      o[sys].i64 = lv[l].img64[sys];
      for (int a = 0; a < 3; ++a) {
        const bool on = a < o[sys].cd.dim;
        o[sys].off[a] = on ? lv[l].off64[sys][a] : nullptr;
        o[sys].o32[a] = (on && want32) ? lv[l].off32[sys][a] : nullptr;
      }
      if (l > 1) {
        f[sys].d = lv[l - 1].d;
        f[sys].diag = lv[l - 1].diag64[sys];
        f[sys].mass = lv[l - 1].mass64[sys];
        for (int a = 0; a < 3; ++a) f[sys].off[a] = (a < f[sys].d.dim) ? lv[l - 1].off64[sys][a] : nullptr;
      }
    }
    const unsigned nb = nblk(o[0].cd.N);
    if (l == 1) {
      memset(fine, 0, sizeof(*fine));
      fine->op[0] = op[0];
      fine->op[1] = op[1];
      fine->o[0] = o[0];
      fine->o[1] = o[1];
      fine->nb = nb;
    } else {
      BuildCoarseArgs& a = coarse[nc++];
      memset(&a, 0, sizeof(a));
      a.op[0] = f[0];
      a.op[1] = f[1];
      a.o[0] = o[0];
      a.o[1] = o[1];
      a.nb = nb;
    }
  }
  return nc;
}

hipError_t ebit_build_hierarchy(const FineOp* op, EbitLevelHost* lv, int nlev, int want32, const void* dev_tabs,
                                int ls, hipStream_t st) {
  // one launch per level for both systems
  BuildFineArgs fine;
  BuildCoarseArgs coarse[EBIT_MAX_LEVELS];
  const int nc = ebit_build_args(op, lv, nlev, want32, ls, &fine, coarse);
  if (ls > 1 && nlev > 1)
    hipLaunchKernelGGL(k_build_from_fine2<false>, dim3(2 * fine.nb), dim3(EBIT_BLOCK), 0, st, many_one(fine));
  for (int q = 0; q < nc; ++q) {
    if (lv[0].d.dim == 3)
      hipLaunchKernelGGL((k_build_from_coarse2<3, false>), dim3(2 * coarse[q].nb), dim3(EBIT_BLOCK), 0, st,
                         many_one(coarse[q]));
    else
      hipLaunchKernelGGL((k_build_from_coarse2<2, false>), dim3(2 * coarse[q].nb), dim3(EBIT_BLOCK), 0, st,
                         many_one(coarse[q]));
  }
  BuildSmallArgs a;
  a.tabs = dev_tabs;
  if (lv[0].d.dim == 3)
    hipLaunchKernelGGL((k_build_small<3, false>), dim3(2), dim3(1024), 0, st, many_one(a));
  else
    hipLaunchKernelGGL((k_build_small<2, false>), dim3(2), dim3(1024), 0, st, many_one(a));
  return hipGetLastError();
}

// Batched forms: n cases per launch (tab: device table; start: n + 1 block
// offsets; blocks = start[n]).
hipError_t ebit_launch_build_fine_many(int n, const BuildFineArgs* tab, const int* start, int blocks,
                                       hipStream_t st) {
  hipLaunchKernelGGL(k_build_from_fine2<true>, dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}
hipError_t ebit_launch_build_coarse_many(int n, int dim, const BuildCoarseArgs* tab, const int* start, int blocks,
                                         hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL((k_build_from_coarse2<3, true>), dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st,
                       many_tab(tab, start, n));
  else
    hipLaunchKernelGGL((k_build_from_coarse2<2, true>), dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st,
                       many_tab(tab, start, n));
  return hipGetLastError();
}
// two blocks (one per system) per case
hipError_t ebit_launch_build_small_many(int n, int dim, const BuildSmallArgs* tab, const int* start,
                                        hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL((k_build_small<3, true>), dim3((unsigned)(2 * n)), dim3(1024), 0, st, many_tab(tab, start, n));
  else
    hipLaunchKernelGGL((k_build_small<2, true>), dim3((unsigned)(2 * n)), dim3(1024), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}
hipError_t ebit_launch_heat_rhs_many(int n, const HeatRhsArgs* tab, const int* start, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_heat_rhs<true>, dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}
// one block per case
hipError_t ebit_launch_finalize_many(int n, const FinArgs* tab, const int* start, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize<true>, dim3((unsigned)n), dim3(256), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}
hipError_t ebit_launch_scal_many(int n, const ScalArgs* tab, const int* start, hipStream_t st) {
  hipLaunchKernelGGL(k_scal<true>, dim3((unsigned)n), dim3(64), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}
hipError_t ebit_launch_split_flags_many(int n, const SplitArgs* tab, const int* start, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_split_flags<true>, dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}

hipError_t ebit_launch_apply(const FineOp* op, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_apply, dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, *op, x, y);
  return hipGetLastError();
}

hipError_t ebit_launch_heat_rhs(const FineOp* op, const double* Ts, double* b, hipStream_t st) {
  HeatRhsArgs a;
  a.op = *op;
  a.Ts = Ts;
  a.b = b;
  hipLaunchKernelGGL(k_heat_rhs<false>, dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, many_one(a));
  return hipGetLastError();
}

hipError_t ebit_launch_finalize_max(const double* partial, int nb, Scal* sc, hipStream_t st) {
  FinArgs a;
  a.partial = partial;
  a.nb = nb;
  a.nv = 1;
  a.kind = FIN_MAX;
  a.sc = sc;
  hipLaunchKernelGGL(k_finalize<false>, dim3(1), dim3(256), 0, st, many_one(a));
  return hipGetLastError();
}

// LDS the tail kernel may use: the device's per-work-group maximum (raising
// the kernel's dynamic-LDS limit above 64 KiB where the device allows it).
int ebit_tail_lds_setup(void) {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 64 * 1024;
  if (v > 64 * 1024) {
    if (hipFuncSetAttribute((const void*)kb_tail<float, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)kb_tail<float, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)kb_tail<double, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)kb_tail<double, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess) {
      (void)hipGetLastError();
      return 64 * 1024;
    }
  }
  return v;
}

// ---- profiling ----
hipError_t ebit_prof_flush(EbitProfiler* pr) {
  if (!pr || pr->npend == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(pr->ev1[pr->npend - 1]);
  if (e != hipSuccess) return e;
  for (int i = 0; i < pr->npend; ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr->ev0[i], pr->ev1[i]);
    if (e != hipSuccess) return e;
    pr->ms[pr->kid[i]] += ms;
    pr->launches[pr->kid[i]] += pr->count[i];
  }
  pr->npend = 0;
  return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solve plans: device tables and work lists of a batch of cases, and the
// host side of the outer iteration.
// ---------------------------------------------------------------------------
namespace {

// Bracket one launch, or a run of n consecutive launches of one class, with
// events when profiling is on (a run shares one pair of events, so the
// events' own dispatch is paid once per run).
struct ProfScope {
  EbitProfiler* pr;
  hipStream_t st;
  int slot;
  ProfScope(EbitProfiler* p, int kid, hipStream_t s, int n = 1) : pr(p), st(s), slot(-1) {
    if (!pr || !pr->on) return;
    if (pr->npend == EBIT_PROF_CAP) (void)ebit_prof_flush(pr);
    slot = pr->npend++;
    pr->kid[slot] = kid;
    pr->count[slot] = n;
    (void)hipEventRecord(pr->ev0[slot], st);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(pr->ev1[slot], st);
  }
};

template <typename T>
CoarseOp<T> coarse_op_of(const EbitLevelHost& L, int sys);
template <>
CoarseOp<double> coarse_op_of<double>(const EbitLevelHost& L, int sys) {
  CoarseOp<double> c;
  c.d = L.d;
  c.diag = L.diag64[sys];
  for (int a = 0; a < 3; ++a) c.off[a] = L.off64[sys][a];
  c.mass = L.mass64[sys];
  return c;
}
template <>
CoarseOp<float> coarse_op_of<float>(const EbitLevelHost& L, int sys) {
  CoarseOp<float> c;
  c.d = L.d;
  c.diag = L.diag32[sys];
  for (int a = 0; a < 3; ++a) c.off[a] = L.off32[sys][a];
  c.mass = L.mass64[sys];
  return c;
}
template <typename T>
T* lvx(const EbitLevelHost& L, int s);
template <>
double* lvx<double>(const EbitLevelHost& L, int s) { return s ? L.x64b : L.x64; }
template <>
float* lvx<float>(const EbitLevelHost& L, int s) { return s ? L.x32b : L.x32; }
template <typename T>
T* lvb(const EbitLevelHost& L);
template <>
double* lvb<double>(const EbitLevelHost& L) { return L.b64; }
template <>
float* lvb<float>(const EbitLevelHost& L) { return L.b32; }
template <typename T>
const T* timg(const EbitLevelHost& L, int sys);
template <>
const float* timg<float>(const EbitLevelHost& L, int sys) { return L.img32[sys]; }
template <>
const double* timg<double>(const EbitLevelHost& L, int sys) { return L.img64[sys]; }
template <typename T>
T* zb(const EbitSolveBufs& B, int s);
template <typename T>
T* rvb(const EbitSolveBufs& B, int dim);
template <>
double* rvb<double>(const EbitSolveBufs& B, int dim) { return dim == 3 ? B.r64s : B.r; }
template <>
float* rvb<float>(const EbitSolveBufs& B, int) { return B.r32; }
template <>
double* zb<double>(const EbitSolveBufs& B, int s) { return s ? B.z64b : B.z64; }
template <>
float* zb<float>(const EbitSolveBufs& B, int s) { return s ? B.z32b : B.z32; }

// z-chunk of a tx x ty-tiled sweep (the fine one: 64 x 8): about 16
// work-groups per compute unit, at most 32 planes each.  Work-groups that hold interface cells run
// longer (their rows are assembled from the cut fractions); with several
// rounds of short work-groups the others fill in around them, which more
// than pays for the re-read planes at the chunk ends.
int rb_zchunk(const Dims& d, int tx = 64, int ty = 8) {
  if (d.dim < 3) return 1;
  const long long tiles = (long long)((d.n[0] + tx - 1) / tx) * ((d.n[1] + ty - 1) / ty);
  int zc = 32;
  while (zc > 4 && tiles * ((d.n[2] + zc - 1) / zc) < 4096) zc >>= 1;
  return zc;
}

// z-chunk of an explicit coarse level: as the fine level's, but a level
// that still has 1024 work-groups at 8 planes takes 8 (fewer re-read
// planes), and one that would have fewer than 1024 at 4 planes takes 2
// (its launches are short, and more work-groups in flight pay for the
// re-read planes); measured on the 256^3 film.
int rb_zchunk_coarse(const Dims& d) {
  const int zc = rb_zchunk(d, RB_TX, RB_TY);
  if (d.dim < 3 || zc != 4) return zc;
  const long long tiles = (long long)((d.n[0] + RB_TX - 1) / RB_TX) * ((d.n[1] + RB_TY - 1) / RB_TY);
  if (tiles * ((d.n[2] + 7) / 8) >= 1024) return 8;
  return tiles * ((d.n[2] + 3) / 4) < 1024 ? 2 : 4;
}

// The dense level of a hierarchy (the first of at most EBIT_DENSE_MAX
// cells, whose inverse the build computes), or -1.
int dense_level(const EbitLevelHost* lv, int nlev) {
  for (int l = 1; l < nlev; ++l)
    if (lv[l].inv64[0]) return l;
  return -1;
}

// LDS elements of a tail from level lt down: the copied coefficient image
// (with the dense inverse at its end), x and b of every level, and the
// dense solve's scratch.
long long tail_lds_elems(const EbitLevelHost* lv, int nlev, int lt, long long* coef) {
  const int dl = dense_level(lv, nlev);
  long long c = dl >= 0 ? tail_pad(lv[dl].d.N * lv[dl].d.N) : 0, xb = 0;
  for (int l = lt; l < nlev; ++l) {
    c += tail_img_elems(lv[l].d);
    xb += 4 * tail_half(lv[l].d);
  }
  if (coef) *coef = c;
  return c + xb + EBIT_DENSE_MAX;
}

// First level (>= 1) of the tail: the levels from there down fit lds_bytes
// of LDS and lie in the tail image, and the top one has at most tail_cells
// cells; the coarsest level and the dense level are always in the tail.
template <typename T>
int tail_start(const EbitLevelHost* lv, int nlev, int tail_cells, int lds_bytes) {
  const int dl = dense_level(lv, nlev);
  int lt = nlev - 1;
  for (int l = nlev - 2; l >= 1; --l) {
    // a work-group level: at most tail_kmax cells per thread and colour
    const long long hc = (long long)((lv[l].d.n[0] + 1) / 2) * lv[l].d.n[1] * lv[l].d.n[2];
    const int kmax = lv[l].d.dim == 2 ? tail_kmax<T, 2>() : tail_kmax<T, 3>();
    if (lv[l].d.N > EBIT_TAIL_IMG_CELLS || nlev - l > EBIT_TAIL_MAX || hc > (long long)kmax * EBIT_TAIL_THREADS ||
        tail_lds_elems(lv, nlev, l, nullptr) * (long long)sizeof(T) > lds_bytes)
      break;
    if (lv[l].d.N > tail_cells && (dl < 0 || l < dl)) break;
    lt = l;
  }
  return lt;
}

// reduction blocks of a case: one cell per thread up to EBIT_RED_BLOCKS blocks
int red_blocks(long long N) {
  const long long b = (N + EBIT_BLOCK - 1) / EBIT_BLOCK;
  return (int)(b < 1 ? 1 : (b > EBIT_RED_BLOCKS ? EBIT_RED_BLOCKS : b));
}

const size_t PALIGN = 256;
struct PCarver {
  char* base;
  size_t off;
  template <typename X>
  X* take(size_t n) {
    off = (off + PALIGN - 1) / PALIGN * PALIGN;
    X* p = base ? (X*)(base + off) : nullptr;
    off += n * sizeof(X);
    return p;
  }
};

constexpr int PLAN_MAX_K = 16;                     // outer iterations per graph block
constexpr int PLAN_LISTS = 6 + 3 * EBIT_MAX_LEVELS;  // work lists of a plan

struct HostList {
  WorkList w;
  int blocks;
};

template <typename T>
struct PlanT {
  int n = 0, dim = 0, Lmax = 0;
  ebit_opts o;
  std::vector<EbitPlanCase> cases;
  SolveCase<T>* d_cs[2] = {nullptr, nullptr};
  SolveCase<T>* h_cs[2] = {nullptr, nullptr};
  // control words and scalars of every case, one contiguous block on the
  // device and its pinned host mirror (one copy each way)
  CaseCtl* d_ctl = nullptr;
  CaseCtl* h_ctl = nullptr;
  Scal* d_sc = nullptr;
  Scal* h_sc = nullptr;
  void* h_blk = nullptr;
  HostList fine, frestrict, red;
  HostList half;       // 3D: the colour-split half-sweeps (tiles of one colour's slots)
  HostList hrestrict;  // 3D: their restriction (tiles of level 1)
  HostList pupd;       // 3D split: the p-update (tiles of the natural order)
  HostList coarse[EBIT_MAX_LEVELS], crestrict[EBIT_MAX_LEVELS];
  // 3D split: coarse levels smoothed by natural-order half-sweeps (every
  // periodic axis of even length in every case), and their work lists
  bool chalf_on[EBIT_MAX_LEVELS] = {};
  HostList chalf[EBIT_MAX_LEVELS];
  size_t tail_bytes = 0;
  hipStream_t ist = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t graph[2][PLAN_MAX_K + 1] = {};
  bool no_graph = false;
  // outer iterations of the last solve of each system (most over the
  // cases): the first block of the next solve runs that many
  int last_iters[2] = {0, 0};
  // 2D: some / all cases take their dot products from the last fine sweep
  bool anydot = false, alldot = true;
  // some case has 2^30 cells or more: 64-bit cell offsets in the p-update
  bool wide = false;
  // 3D: the fine level is smoothed in the colour-split order
  bool split = false;
  // test switch: report the cases still running after the first block as
  // stalled (EBIT_TEST_FP32_STALL)
  bool force_stall = false;
};

template <typename T>
size_t plan_carve(int n, PCarver& cv, PlanT<T>* P, int** wl) {
  SolveCase<T>* cs0 = cv.take<SolveCase<T>>(n);
  SolveCase<T>* cs1 = cv.take<SolveCase<T>>(n);
  char* blk = cv.take<char>(n * (sizeof(CaseCtl) + sizeof(Scal)));
  CaseCtl* ctl = (CaseCtl*)blk;
  Scal* sc = blk ? (Scal*)(blk + n * sizeof(CaseCtl)) : nullptr;
  int* w = cv.take<int>((size_t)PLAN_LISTS * (2 * n + 1));
  if (P) {
    P->d_cs[0] = cs0;
    P->d_cs[1] = cs1;
    P->d_ctl = ctl;
    P->d_sc = sc;
    *wl = w;
  }
  return (cv.off + PALIGN - 1) / PALIGN * PALIGN;
}

// append a work list of (case, blocks) entries with at least one block
HostList make_list(const std::vector<std::pair<int, int>>& ent, std::vector<int>& host, const int* dev) {
  HostList L;
  const size_t o = host.size();
  int tot = 0;
  int m = 0;
  for (const auto& e : ent)
    if (e.second > 0) ++m;
  for (const auto& e : ent)
    if (e.second > 0) {
      host.push_back(tot);
      tot += e.second;
    }
  host.push_back(tot);
  for (const auto& e : ent)
    if (e.second > 0) host.push_back(e.first);
  L.w.start = dev + o;
  L.w.cid = dev + o + m + 1;
  L.w.n = m;
  L.w.c0 = 0;
  for (const auto& e : ent)
    if (e.second > 0) {
      L.w.c0 = e.first;
      break;
    }
  L.w.total = tot;
  L.blocks = tot;
  return L;
}

// res: also restrict the residual to the next level (2D only)
// dots: the outer loop's dot products in this launch (2D; 1 + [defect
// correction], 0 none)
template <typename T>
void launch_fine(const PlanT<T>& P, const SolveCase<T>* cs, int in, int out, int add, int nsw, int res, int dots,
                 hipStream_t st) {
  CaseCtl* ctl = P.d_ctl;
  // the first pre-smoothing launch takes the pending r.r (2D)
  const int settle = (P.dim == 2 && in < 0) ? 1 : 0;
  const dim3 g(P.fine.blocks), b(RB_THREADS);
  if (P.dim == 3)
    hipLaunchKernelGGL((kb_rb_fine<T, 64, 8, 1, 0>), g, b, 0, st, cs, ctl, P.fine.w, in, out, add, 0, 0);
  else if (nsw == 2 && res)
    hipLaunchKernelGGL((kb_rb_fine<T, 64, 4, 2, 1>), g, b, 0, st, cs, ctl, P.fine.w, in, out, add, dots, settle);
  else if (nsw == 2)
    hipLaunchKernelGGL((kb_rb_fine<T, 64, 4, 2, 0>), g, b, 0, st, cs, ctl, P.fine.w, in, out, add, dots, settle);
  else if (res)
    hipLaunchKernelGGL((kb_rb_fine<T, 64, 4, 1, 1>), g, b, 0, st, cs, ctl, P.fine.w, in, out, add, dots, settle);
  else
    hipLaunchKernelGGL((kb_rb_fine<T, 64, 4, 1, 0>), g, b, 0, st, cs, ctl, P.fine.w, in, out, add, dots, settle);
}

template <typename T>
void launch_coarse(const PlanT<T>& P, const SolveCase<T>* cs, int l, int in, int out, int add, int nsw, int res,
                   hipStream_t st) {
  const CaseCtl* ctl = P.d_ctl;
  const dim3 g(P.coarse[l].blocks), b(RB_THREADS);
  if (nsw == 2 && res)
    hipLaunchKernelGGL((kb_rb_coarse<T, 2, 1>), g, b, 0, st, cs, ctl, P.coarse[l].w, l, in, out, add);
  else if (nsw == 2)
    hipLaunchKernelGGL((kb_rb_coarse<T, 2, 0>), g, b, 0, st, cs, ctl, P.coarse[l].w, l, in, out, add);
  else if (res)
    hipLaunchKernelGGL((kb_rb_coarse<T, 1, 1>), g, b, 0, st, cs, ctl, P.coarse[l].w, l, in, out, add);
  else
    hipLaunchKernelGGL((kb_rb_coarse<T, 1, 0>), g, b, 0, st, cs, ctl, P.coarse[l].w, l, in, out, add);
}

// A run of ns sweeps on a level, as launches t0, t0 + 1, ... of the
// level's m launches (1-based): launch t writes buffer 0 when m - t is even,
// else buffer 1, so consecutive launches alternate (no launch reads the
// buffer it writes: the tiles' halos come from the input) and the level's
// last launch lands in buffer 0.  In 2D two sweeps go in one launch where
// the run allows it.  launch(in, out, add, nsw, res), res set on the run's
// last launch when res_last.  Returns the buffer the run's last launch
// wrote.
template <typename L>
int sweep_run(int ns, int t0, int m, int in, int add_first, bool pairs, int res_last, const L& launch) {
  int t = t0;
  for (int s = 0; s < ns; ++t) {
    const int nsw = (pairs && s + 1 < ns) ? 2 : 1;
    const int out = ((m - t) % 2 == 0) ? 0 : 1;
    launch(in, out, s == 0 ? add_first : 0, nsw, (res_last && s + nsw == ns) ? 1 : 0);
    in = out;
    s += nsw;
  }
  return in;
}

// One V(nu1, nu2) cycle on A z = r (zero initial guess) for every active
// case.  The launches of a level alternate between its two iterate buffers
// (sweep_run), the last one landing in buffer 0.
template <typename T>
void vcycle_b(const PlanT<T>& P, const SolveCase<T>* cs, hipStream_t st, EbitProfiler* pf) {
  const int nu1 = P.o.nu1, nu2 = P.o.nu2;
  const CaseCtl* ctl = P.d_ctl;
  const bool pairs = P.dim == 2;
  // launches per level before and after the correction
  const int npre = pairs ? (nu1 + 1) / 2 : nu1, npost = pairs ? (nu2 + 1) / 2 : nu2, m = npre + npost;
  const int preb = ((m - npre) % 2 == 0) ? 0 : 1;  // buffer of the pre-smoothed iterate
  // in 2D the last pre-smoothing launch of a level also restricts
  const int fuse = pairs ? 1 : 0;
  auto fine = [&](int in, int out, int add, int nsw, int res) { launch_fine(P, cs, in, out, add, nsw, res, 0, st); };
  // the last post-smoothing launch also forms the dot products (2D)
  const int dots = P.anydot ? 1 + (P.o.outer == EBIT_OUTER_DC ? 1 : 0) : 0;
  auto fine_post = [&](int in, int out, int add, int nsw, int last) {
    launch_fine(P, cs, in, out, add, nsw, 0, last ? dots : 0, st);
  };
  // 3D: a sweep is two colour-split half-sweeps (red, then black)
  auto half = [&](int color, int first, int add) {
    if (first)
      hipLaunchKernelGGL((kb_half3<T, 1>), dim3(P.half.blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl, P.half.w, color);
    else if (add)
      hipLaunchKernelGGL((kb_half3<T, 2>), dim3(P.half.blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl, P.half.w, color);
    else
      hipLaunchKernelGGL((kb_half3<T, 0>), dim3(P.half.blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl, P.half.w, color);
  };
  if (P.split) {
    {
      ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st, 2 * nu1);
      for (int sw = 0; sw < nu1; ++sw) {
        half(0, sw == 0 ? 1 : 0, 0);
        half(1, 0, 0);
      }
    }
    ProfScope ps(pf, EBIT_KC_FINE_RESTRICT, st);
    hipLaunchKernelGGL(kb_fine_restrict_split<T>, dim3(P.hrestrict.blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl,
                       P.hrestrict.w);
  } else {
    {
      ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st, npre);
      sweep_run(nu1, 1, m, -1, 0, pairs, fuse, fine);
    }
    if (!fuse) {
      ProfScope ps(pf, EBIT_KC_FINE_RESTRICT, st);
      hipLaunchKernelGGL(kb_fine_restrict<T>, dim3(P.frestrict.blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl,
                         P.frestrict.w, preb);
    }
  }
  // 3D coarse levels of even periodic lengths: half-sweeps in place on
  // buffer 0 (red, then black), like the fine level
  auto chalf = [&](int l, int color, int mode) {
    const dim3 g(P.chalf[l].blocks), b(EBIT_BLOCK);
    if (mode == 1)
      hipLaunchKernelGGL((kb_chalf<T, 1>), g, b, 0, st, cs, ctl, P.chalf[l].w, l, color);
    else if (mode == 2)
      hipLaunchKernelGGL((kb_chalf<T, 2>), g, b, 0, st, cs, ctl, P.chalf[l].w, l, color);
    else
      hipLaunchKernelGGL((kb_chalf<T, 0>), g, b, 0, st, cs, ctl, P.chalf[l].w, l, color);
  };
  for (int l = 1; l < P.Lmax; ++l) {
    auto coarse = [&](int in, int out, int add, int nsw, int res) {
      launch_coarse(P, cs, l, in, out, add, nsw, res, st);
    };
    if (P.chalf_on[l]) {
      ProfScope ps(pf, EBIT_KC_COARSE, st, 2 * nu1 + 1);
      for (int sw = 0; sw < nu1; ++sw) {
        chalf(l, 0, sw == 0 ? 1 : 0);
        chalf(l, 1, 0);
      }
      hipLaunchKernelGGL(kb_chalf_restrict<T>, dim3(P.crestrict[l].blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl,
                         P.crestrict[l].w, l);
      continue;
    }
    {
      ProfScope ps(pf, EBIT_KC_COARSE, st, npre);
      sweep_run(nu1, 1, m, -1, 0, pairs, fuse, coarse);
    }
    if (!fuse) {
      ProfScope ps(pf, EBIT_KC_COARSE, st);
      hipLaunchKernelGGL(kb_coarse_restrict<T>, dim3(P.crestrict[l].blocks), dim3(EBIT_BLOCK), 0, st, cs, ctl,
                         P.crestrict[l].w, l, preb);
    }
  }
  {
    ProfScope ps(pf, EBIT_KC_TAIL, st);
    if (P.dim == 3)
      hipLaunchKernelGGL((kb_tail<T, 3>), dim3(P.n), dim3(EBIT_TAIL_THREADS), P.tail_bytes, st, cs, ctl);
    else
      hipLaunchKernelGGL((kb_tail<T, 2>), dim3(P.n), dim3(EBIT_TAIL_THREADS), P.tail_bytes, st, cs, ctl);
  }
  for (int l = P.Lmax - 1; l >= 1; --l) {
    auto coarse = [&](int in, int out, int add, int nsw, int res) {
      launch_coarse(P, cs, l, in, out, add, nsw, res, st);
    };
    if (P.chalf_on[l]) {
      ProfScope ps(pf, EBIT_KC_COARSE, st, 2 * nu2);
      for (int sw = 0; sw < nu2; ++sw) {
        chalf(l, 0, sw == 0 ? 2 : 0);
        chalf(l, 1, 0);
      }
      continue;
    }
    ProfScope ps(pf, EBIT_KC_COARSE, st, npost);
    sweep_run(nu2, npre + 1, m, preb, 1, pairs, 0, coarse);
  }
  if (P.split) {
    ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st, 2 * nu2);
    for (int sw = 0; sw < nu2; ++sw) {
      half(0, 0, sw == 0 ? 1 : 0);
      half(1, 0, 0);
    }
  } else {
    ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st, npost);
    sweep_run(nu2, npre + 1, m, preb, 1, pairs, 1, fine_post);
  }
}

// K outer iterations: flexible CG preconditioned by one V-cycle; defect
// correction is the same loop with beta = 0 (x += alpha V(r) with the
// energy-optimal step alpha = (r.z)/(z.Az), which contracts for any SPD A).
template <typename T>
void launch_p_update(const PlanT<T>& P, const SolveCase<T>* cs, int sys, int dc, hipStream_t st) {
  const dim3 g(P.red.blocks), b(EBIT_BLOCK);
  const CaseCtl* ctl = P.d_ctl;
  // 3D: the LDS-staged kernel; from 2^30 cells on (or with the test
  // switch), the strided kernel with 64-bit offsets
  if (P.wide) {
    if (sys == EBIT_SYS_HEAT)
      hipLaunchKernelGGL((kb_p_update_apply<T, EBIT_SYS_HEAT, long long>), g, b, 0, st, cs, ctl, P.red.w, dc);
    else
      hipLaunchKernelGGL((kb_p_update_apply<T, EBIT_SYS_PRESSURE, long long>), g, b, 0, st, cs, ctl, P.red.w, dc);
  } else if (P.split) {
    // p-update, then q = A p with the p.q partials on the reduction work list
    hipLaunchKernelGGL(kb_p_update3<T>, dim3(P.pupd.blocks), b, 0, st, cs, ctl, P.pupd.w, dc);
    if (sys == EBIT_SYS_HEAT)
      hipLaunchKernelGGL((kb_apply_q3<T, EBIT_SYS_HEAT>), g, b, 0, st, cs, ctl, P.red.w);
    else
      hipLaunchKernelGGL((kb_apply_q3<T, EBIT_SYS_PRESSURE>), g, b, 0, st, cs, ctl, P.red.w);
  } else if (P.dim == 3) {
    if (sys == EBIT_SYS_HEAT)
      hipLaunchKernelGGL((kb_apply3d<T, EBIT_SYS_HEAT>), g, b, 0, st, cs, ctl, P.red.w, dc);
    else
      hipLaunchKernelGGL((kb_apply3d<T, EBIT_SYS_PRESSURE>), g, b, 0, st, cs, ctl, P.red.w, dc);
  } else {
    if (sys == EBIT_SYS_HEAT)
      hipLaunchKernelGGL((kb_p_update_apply<T, EBIT_SYS_HEAT, int>), g, b, 0, st, cs, ctl, P.red.w, dc);
    else
      hipLaunchKernelGGL((kb_p_update_apply<T, EBIT_SYS_PRESSURE, int>), g, b, 0, st, cs, ctl, P.red.w, dc);
  }
}

template <typename T>
void iterations(const PlanT<T>& P, const SolveCase<T>* cs, int sys, int K, hipStream_t st, EbitProfiler* pf) {
  const int dc = P.o.outer == EBIT_OUTER_DC;
  for (int k = 0; k < K; ++k) {
    vcycle_b(P, cs, st, pf);
    if (!P.alldot)
      hipLaunchKernelGGL(kb_dots<T>, dim3(P.red.blocks), dim3(EBIT_BLOCK), 0, st, cs, (const CaseCtl*)P.d_ctl,
                         P.red.w, dc);
    {
      ProfScope ps(pf, EBIT_KC_OUTER_APPLY, st);
      launch_p_update(P, cs, sys, dc, st);
    }
    {
      ProfScope ps(pf, EBIT_KC_OUTER_UPDATE, st);
      hipLaunchKernelGGL(kb_update_xr<T>, dim3(P.red.blocks), dim3(EBIT_BLOCK), 0, st, cs, P.d_ctl, P.red.w,
                         P.dim == 2 ? 1 : 0);
    }
    // 3D: end the iteration here; 2D: the next V-cycle's first launch does
    if (P.dim != 2)
      hipLaunchKernelGGL(kb_finalize<T>, dim3(P.n), dim3(256), 0, st, cs, P.d_ctl, (int)FIN_RR, 1, 3,
                         (int)MASK_ACTIVE, 0.0);
  }
  // the last iteration of the block is ended before the host reads it
  if (P.dim == 2)
    hipLaunchKernelGGL(kb_finalize<T>, dim3(P.n), dim3(256), 0, st, cs, P.d_ctl, (int)FIN_PEND, 1, 3, (int)MASK_ALL,
                       0.0);
  // cases whose recurrence reached its stop level in this block: the true
  // residual b - A x, its norm and the floor norm, for the host to judge
  // from the same read-back
  launch_resid_init(P.red.blocks, cs, P.d_ctl, P.red.w, sys, (int)MASK_STOPPED, 1, 0, st);
  hipLaunchKernelGGL(kb_finalize<T>, dim3(P.n), dim3(256), 0, st, cs, P.d_ctl, (int)FIN_INIT, 3, 0,
                     (int)MASK_STOPPED, 0.0);
}

// Run K iterations: replay the captured graph of the block (captured on
// first use), or launch eagerly while per-launch profiling is on.
template <typename T>
hipError_t run_block(PlanT<T>& P, int sys, int K, EbitProfiler* pf) {
  const SolveCase<T>* cs = P.d_cs[sys];
  if ((pf && pf->on) || P.no_graph || K > PLAN_MAX_K) {
    iterations(P, cs, sys, K, P.ist, pf);
    return hipGetLastError();
  }
  hipGraphExec_t& ge = P.graph[sys][K];
  if (!ge) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(P.ist, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      iterations(P, cs, sys, K, P.ist, nullptr);
      e = hipStreamEndCapture(P.ist, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      // no graph on this stream or runtime: launch eagerly from now on
      (void)hipGetLastError();
      ge = nullptr;
      P.no_graph = true;
      iterations(P, cs, sys, K, P.ist, nullptr);
      return hipGetLastError();
    }
  }
  return hipGraphLaunch(ge, P.ist);
}

// EBIT_WIDE_OFFSETS=1 in the environment selects the 64-bit-offset kernels
// at any size (a test of the form the large grids take; same results).
bool wide_offsets_env() {
  const char* e = std::getenv("EBIT_WIDE_OFFSETS");
  return e && e[0] == '1';
}

// EBIT_TEST_FP32_STALL=1 makes a mixed-precision plan report every case
// that is still iterating after its first block as stalled (a test of the
// FP64 fallback from the host side; the kernels run as always).
bool force_stall_env() {
  const char* e = std::getenv("EBIT_TEST_FP32_STALL");
  return e && e[0] == '1';
}

template <typename T>
hipError_t plan_create_t(PlanT<T>* P, int n, const EbitPlanCase* cases, const ebit_opts* o, int tail_lds, void* mem,
                         size_t bytes) {
  P->n = n;
  const bool wide_env = wide_offsets_env();
  P->force_stall = std::is_same<T, float>::value && force_stall_env();
  P->o = *o;
  P->cases.assign(cases, cases + n);
  P->dim = cases[0].lv[0].d.dim;
  PCarver cv{(char*)mem, 0};
  int* d_wl = nullptr;
  if (plan_carve<T>(n, cv, P, &d_wl) > bytes) return hipErrorInvalidValue;
  hipError_t e;
  for (int s = 0; s < 2; ++s)
    if ((e = hipHostMalloc((void**)&P->h_cs[s], n * sizeof(SolveCase<T>), 0)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&P->h_blk, n * (sizeof(CaseCtl) + sizeof(Scal)), 0)) != hipSuccess) return e;
  P->h_ctl = (CaseCtl*)P->h_blk;
  P->h_sc = (Scal*)((char*)P->h_blk + n * sizeof(CaseCtl));
  if ((e = hipStreamCreateWithFlags(&P->ist, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming)) != hipSuccess) return e;
  std::vector<int> lt(n);
  size_t tail_elems = 0;
  P->Lmax = 1;
  for (int c = 0; c < n; ++c) {
    const EbitPlanCase& pc = cases[c];
    lt[c] = tail_start<T>(pc.lv, pc.nlev, o->tail_cells, tail_lds);
    const size_t el = (size_t)tail_lds_elems(pc.lv, pc.nlev, lt[c], nullptr);
    if (el > tail_elems) tail_elems = el;
    if (lt[c] > P->Lmax) P->Lmax = lt[c];
  }
  P->tail_bytes = tail_elems * sizeof(T);
  std::vector<std::pair<int, int>> efine, efr, ered, ehalf, ehres, epu;
  // 3D grids smooth the fine level in the colour-split order and run the
  // p-update and A p as streaming passes, addressed by 32-bit buffer
  // offsets: every FP64 fine array must stay below 2^31 bytes (fewer than
  // 2^28 cells), else the grids keep the LDS z-march kernels
  P->split = P->dim == 3;
  for (int c = 0; c < n; ++c)
    if (cases[c].lv[0].d.N * (long long)sizeof(double) >= (1LL << 31)) P->split = false;
  std::vector<std::pair<int, int>> ecs[EBIT_MAX_LEVELS], ecr[EBIT_MAX_LEVELS], ech[EBIT_MAX_LEVELS];
  for (int l = 1; l < P->Lmax; ++l) {
    P->chalf_on[l] = P->split;
    for (int c = 0; c < n; ++c) {
      if (l >= lt[c]) continue;
      const Dims& d = cases[c].lv[l].d;
      for (int a = 0; a < 3; ++a)
        if (d.per[a] && d.n[a] > 1 && (d.n[a] & 1)) P->chalf_on[l] = false;
    }
  }
  for (int sys = 0; sys < 2; ++sys)
    for (int c = 0; c < n; ++c) {
      const EbitPlanCase& pc = cases[c];
      SolveCase<T>& C = P->h_cs[sys][c];
      memset(&C, 0, sizeof(C));
      C.op = pc.op[sys];
      C.b = pc.b;
      C.x = nullptr;
      C.r = pc.B.r;
      C.rv = rvb<T>(pc.B, P->split ? 3 : 2);
      C.split = P->split ? 1 : 0;
      C.fs = pc.B.fsplit;
      C.z[0] = zb<T>(pc.B, 0);
      C.z[1] = zb<T>(pc.B, 1);
      C.p[0] = pc.B.p[0];
      C.p[1] = pc.B.p[1];
      C.q = pc.B.q;
      C.partial = pc.B.partial;
      C.sc = P->d_sc + c;
      const Dims& fd = pc.lv[0].d;
      C.nred = red_blocks(fd.N);
      if (fd.N >= (1LL << 30) || wide_env) P->wide = true;
      C.nlev = pc.nlev;
      C.lt = lt[c];
      const int fty = P->dim == 3 ? 8 : 4;
      C.fzc = rb_zchunk(fd);
      C.fgx = (fd.n[0] + 63) / 64;
      C.fgy = (fd.n[1] + fty - 1) / fty;
      // one dot partial per fine tile, while they fit the rows the
      // reduction blocks leave (2D sweeps hold r and z of a tile in LDS)
      const int tiles = C.fgx * C.fgy;
      C.ndot = (P->dim == 2 && tiles <= C.nred) ? tiles : 0;
      if (sys == 0) {
        P->anydot = P->anydot || C.ndot > 0;
        P->alldot = P->alldot && C.ndot > 0;
      }
      for (int l = 1; l < pc.nlev; ++l) {
        const EbitLevelHost& L = pc.lv[l];
        C.lev[l] = coarse_op_of<T>(L, sys);
        C.lb[l] = lvb<T>(L);
        C.lx[l][0] = lvx<T>(L, 0);
        C.lx[l][1] = lvx<T>(L, 1);
        C.lzc[l] = rb_zchunk_coarse(L.d);
        const int ctx = L.d.dim == 2 ? RB_CTX : RB_TX;
        C.lgx[l] = (L.d.n[0] + ctx - 1) / ctx;
        const int cty = L.d.dim == 2 ? RB_CTY : RB_TY;
        C.lgy[l] = (L.d.n[1] + cty - 1) / cty;
      }
      TailArgs<T>& ta = C.tail;
      ta.nl = pc.nlev - lt[c];
      ta.nu1 = o->nu1;
      ta.nu2 = o->nu2;
      long long coef = 0;
      tail_lds_elems(pc.lv, pc.nlev, lt[c], &coef);
      long long cb = 0, xr = 0;
      for (int m = 0; m < ta.nl; ++m) xr += 2 * tail_half(pc.lv[lt[c] + m].d);
      long long xb = coef, bb = coef + xr;
      for (int m = 0; m < ta.nl; ++m) {
        const EbitLevelHost& L = pc.lv[lt[c] + m];
        ta.L[m].d = L.d;
        ta.L[m].hs = (int)tail_half(L.d);
        ta.L[m].cb = (int)cb;
        ta.L[m].xb = (int)xb;
        ta.L[m].bb = (int)bb;
        cb += tail_img_elems(L.d);
        xb += 2 * tail_half(L.d);
        bb += 2 * tail_half(L.d);
      }
      ta.tmp = (int)bb;
      const int dl = dense_level(pc.lv, pc.nlev);
      ta.dl = dl >= lt[c] ? dl - lt[c] : -1;
      ta.inv = (int)cb;
      ta.inv_ok = dl >= 0 ? pc.lv[dl].inv_ok + sys : nullptr;
      ta.img = timg<T>(pc.lv[lt[c]], sys);
      ta.cvec = (int)(coef * (long long)sizeof(T) / 16);
      ta.bg = lvb<T>(pc.lv[lt[c]]);
      ta.xg = lvx<T>(pc.lv[lt[c]], 0);
      if (sys == 0) {
        const int fgz = (fd.n[2] + C.fzc - 1) / C.fzc;
        efine.push_back({c, C.fgx * C.fgy * fgz});
        ehalf.push_back({c, P->split ? split_blocks(split_tiles((fd.n[0] + 1) / 2, fd.n[1], fd.n[2])) : 0});
        const Dims& d1 = pc.lv[1].d;
        ehres.push_back({c, P->split ? split_blocks(split_tiles(d1.n[0], d1.n[1], d1.n[2]), SP_TPB_R) : 0});
        epu.push_back({c, P->split ? split_blocks(split_tiles(fd.n[0], fd.n[1], fd.n[2]), PU_TPB) : 0});
        efr.push_back({c, (int)nblk(pc.lv[1].d.N)});
        ered.push_back({c, C.nred});
        for (int l = 1; l < lt[c]; ++l) {
          const Dims& d = pc.lv[l].d;
          ecs[l].push_back({c, C.lgx[l] * C.lgy[l] * ((d.n[2] + C.lzc[l] - 1) / C.lzc[l])});
          ecr[l].push_back({c, (int)nblk(pc.lv[l + 1].d.N)});
          ech[l].push_back({c, P->chalf_on[l] ? (int)nblk((long long)((d.n[0] + 1) / 2) * d.n[1] * d.n[2]) : 0});
        }
      }
    }
  std::vector<int> host;
  P->fine = make_list(efine, host, d_wl);
  P->frestrict = make_list(efr, host, d_wl);
  P->red = make_list(ered, host, d_wl);
  P->half = make_list(ehalf, host, d_wl);
  P->hrestrict = make_list(ehres, host, d_wl);
  P->pupd = make_list(epu, host, d_wl);
  for (int l = 1; l < P->Lmax; ++l) {
    P->coarse[l] = make_list(ecs[l], host, d_wl);
    P->crestrict[l] = make_list(ecr[l], host, d_wl);
    P->chalf[l] = make_list(ech[l], host, d_wl);
  }
  if ((e = hipMemcpyAsync(d_wl, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice, P->ist)) != hipSuccess)
    return e;
  return hipStreamSynchronize(P->ist);
}

template <typename T>
void plan_destroy_t(PlanT<T>* P) {
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k <= PLAN_MAX_K; ++k)
      if (P->graph[s][k]) (void)hipGraphExecDestroy(P->graph[s][k]);
  if (P->ist) {
    (void)hipStreamSynchronize(P->ist);
    (void)hipStreamDestroy(P->ist);
  }
  if (P->ev_in) (void)hipEventDestroy(P->ev_in);
  if (P->ev_out) (void)hipEventDestroy(P->ev_out);
  for (int s = 0; s < 2; ++s)
    if (P->h_cs[s]) (void)hipHostFree(P->h_cs[s]);
  if (P->h_blk) (void)hipHostFree(P->h_blk);
  delete P;
}

// The outer loop of every case of the plan, to rel. residual rtol.  Status
// per case: 0 converged, 1 max_iters or stagnation above the rounding floor,
// 2 NaN/Inf.  Returns a HIP error, if any.
template <typename T>
hipError_t plan_solve_t(PlanT<T>& P, int sys, double* const* x, int use_guess, hipStream_t ust, EbitProfiler* pf,
                        EbitSolveOut* out) {
  const int n = P.n;
  const ebit_opts& o = P.o;
  const int dc = o.outer == EBIT_OUTER_DC;
  hipStream_t st = P.ist;
  hipError_t e;
#define PK(expr)                          \
  do {                                    \
    if ((e = (expr)) != hipSuccess) return e; \
  } while (0)
  for (int c = 0; c < n; ++c) {
    P.h_cs[sys][c].op = P.cases[c].op[sys];
    P.h_cs[sys][c].x = x[c];
  }
  const SolveCase<T>* cs = P.d_cs[sys];
  const size_t blk = n * (sizeof(CaseCtl) + sizeof(Scal));
  PK(hipEventRecord(P.ev_in, ust));
  PK(hipStreamWaitEvent(st, P.ev_in, 0));
  PK(hipMemcpyAsync(P.d_cs[sys], P.h_cs[sys], n * sizeof(SolveCase<T>), hipMemcpyHostToDevice, st));
  // start: the device forms r = b - A x (a cold start clears x in the same
  // pass), then clears the scalars and decides per case (b = 0: x = 0;
  // already converged: stopped; else iterate to rtol |b|); no host round
  // trip before the first block of iterations
  launch_resid_init(P.red.blocks, cs, P.d_ctl, P.red.w, sys, (int)MASK_ALL, use_guess ? 1 : 0, use_guess ? 0 : 1,
                    st);
  hipLaunchKernelGGL(kb_finalize<T>, dim3(n), dim3(256), 0, st, cs, P.d_ctl, (int)FIN_START, 3, 0, (int)MASK_ALL,
                     o.rtol * o.rtol);
  if (use_guess)
    hipLaunchKernelGGL(kb_zero_x<T>, dim3(P.red.blocks), dim3(EBIT_BLOCK), 0, st, cs, (const CaseCtl*)P.d_ctl,
                       P.red.w, (int)MASK_ZERO);
  PK(hipGetLastError());
  const double fc = 2.220446049250313e-16;
  std::vector<int> status(n, -1), restarts(n, 0), at_floor(n, 0), stalled(n, 0);
  std::vector<double> tol2(n, 0.0), floor2(n, 0.0), last_true(n, 0.0), bb(n, 0.0);
  const int check = o.check_every > 0 ? o.check_every : 1;
  for (bool first = true;; first = false) {
    // the first block runs as many iterations as the last solve of this
    // system took (time steps change the systems little), later ones
    // check_every
    int K = first && P.last_iters[sys] > 0 ? std::min(P.last_iters[sys], PLAN_MAX_K) : check;
    int running = 0;
    for (int c = 0; c < n; ++c)
      if (status[c] < 0) {
        ++running;
        const int left = o.max_iters - (first ? 0 : P.h_sc[c].iters);
        if (left < K) K = left;
      }
    if (running == 0) break;
    if (K < 1) K = 1;
    // the host's decisions of the last round (only needed before a block)
    if (!first) PK(hipMemcpyAsync(P.d_ctl, P.h_ctl, n * sizeof(CaseCtl), hipMemcpyHostToDevice, st));
    PK(run_block(P, sys, K, pf));
    PK(hipMemcpyAsync(P.h_blk, P.d_ctl, blk, hipMemcpyDeviceToHost, st));
    PK(hipStreamSynchronize(st));
    for (int c = 0; c < n; ++c) {
      if (status[c] >= 0) continue;
      const Scal& S = P.h_sc[c];
      CaseCtl& cc = P.h_ctl[c];
      if (first) {
        bb[c] = S.bb;
        tol2[c] = o.rtol * o.rtol * S.bb;
        floor2[c] = fc * fc * S.aa;
      }
      if (S.err & ERR_NAN) {
        status[c] = 2;
        cc.active = 0;
      } else if (P.force_stall && S.bb != 0.0 && !(S.rr <= tol2[c])) {
        status[c] = 1;
        stalled[c] = 1;
        cc.active = 0;
        cc.recheck = 0;
      } else if (S.bb == 0.0) {
        status[c] = 0;  // b = 0: x = 0 (cleared on the device)
        cc.active = 0;
        cc.recheck = 0;
      } else if (cc.recheck == 1) {
        // the recurrence stopped and the block's end formed the true
        // residual (S.rr, S.aa)
        cc.recheck = 0;
        const double rr = S.rr;
        floor2[c] = fc * fc * S.aa;
        // At the representability floor the residual no longer tracks the
        // error, but the compensated residual still carries it: take two more
        // restart cycles there before stopping.
        const bool stagnant = restarts[c] > 0 && rr > 0.25 * last_true[c];
        if (stagnant && rr <= floor2[c]) ++at_floor[c];
        if (rr <= tol2[c] || at_floor[c] >= 2) {
          status[c] = 0;
        } else if (restarts[c] >= 8 || (stagnant && rr > floor2[c]) || S.iters >= o.max_iters) {
          status[c] = 1;
          // the inner cycle stopped contracting (not the iteration limit)
          stalled[c] = S.iters < o.max_iters ? 1 : 0;
        } else {
          // restart the recurrence from the recomputed residual
          ++restarts[c];
          last_true[c] = rr;
          cc.active = 1;
          cc.fresh = 1;
          cc.stop2 = fmax(tol2[c], 1e-12 * rr);
        }
      } else if (!cc.active || S.iters >= o.max_iters) {
        status[c] = 1;
        cc.active = 0;
      }
    }
  }
  {
    int most = 0;
    for (int c = 0; c < n; ++c) most = std::max(most, P.h_sc[c].iters);
    P.last_iters[sys] = most;
  }
  PK(hipEventRecord(P.ev_out, st));
  PK(hipStreamWaitEvent(ust, P.ev_out, 0));
  for (int c = 0; c < n; ++c) {
    const Scal& S = P.h_sc[c];
    EbitSolveOut& r = out[c];
    r.status = status[c] < 0 ? 1 : status[c];
    r.stalled = stalled[c];
    r.iters = S.iters;
    r.bnorm = sqrt(bb[c]);
    r.rel_res = bb[c] > 0 ? sqrt(S.rr / bb[c]) : 0.0;
    r.res_floor = bb[c] > 0 ? sqrt(floor2[c] / bb[c]) : 0.0;
  }
  return hipSuccess;
#undef PK
}

}  // namespace

struct EbitPlan {
  int precision;
  PlanT<float>* f;
  PlanT<double>* d;
};

extern "C" {

size_t ebit_plan_device_bytes(int ncases, int precision) {
  PCarver cv{nullptr, 0};
  if (precision == EBIT_MIXED) return plan_carve<float>(ncases, cv, nullptr, nullptr);
  return plan_carve<double>(ncases, cv, nullptr, nullptr);
}

hipError_t ebit_plan_create(EbitPlan** out, int ncases, const EbitPlanCase* cases, const ebit_opts* o, int tail_lds,
                            void* mem, size_t bytes) {
  *out = nullptr;
  EbitPlan* p = new (std::nothrow) EbitPlan{o->precision, nullptr, nullptr};
  if (!p) return hipErrorOutOfMemory;
  hipError_t e;
  if (o->precision == EBIT_MIXED) {
    p->f = new (std::nothrow) PlanT<float>;
    e = p->f ? plan_create_t<float>(p->f, ncases, cases, o, tail_lds, mem, bytes) : hipErrorOutOfMemory;
  } else {
    p->d = new (std::nothrow) PlanT<double>;
    e = p->d ? plan_create_t<double>(p->d, ncases, cases, o, tail_lds, mem, bytes) : hipErrorOutOfMemory;
  }
  if (e != hipSuccess) {
    ebit_plan_destroy(p);
    return e;
  }
  *out = p;
  return hipSuccess;
}

void ebit_plan_destroy(EbitPlan* p) {
  if (!p) return;
  if (p->f) plan_destroy_t(p->f);
  if (p->d) plan_destroy_t(p->d);
  delete p;
}

hipError_t ebit_plan_solve(EbitPlan* p, int sys, double* const* x, int use_guess, hipStream_t ust, EbitProfiler* pf,
                           EbitSolveOut* out) {
  if (p->f) return plan_solve_t<float>(*p->f, sys, x, use_guess, ust, pf, out);
  return plan_solve_t<double>(*p->d, sys, x, use_guess, ust, pf, out);
}

}  // extern "C"
