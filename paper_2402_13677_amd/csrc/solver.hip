// Geometric multigrid for the two interface-aware elliptic operators, and the
// FP64 outer loop (flexible preconditioned CG, or defect correction).
//
// Fine level: matrix-free (flags + sparse theta reads give every row).
// Coarse levels: 2^d box aggregation; the coarse operator keeps the summed
// mass part and half of the aggregated flux part (couplings, interface and
// wall terms), i.e. A_c = P^T M P + 1/2 P^T (A - M) P, which stays 5/7-point,
// symmetric and scales like a re-discretisation on the coarse grid.
// Smoother: red-black Gauss-Seidel (red then black before the correction,
// black then red after, so the V-cycle is a symmetric preconditioner).
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
template <typename T, typename TB>
__device__ inline T fine_residual_at(const FineOp& op, int i, int j, int k, long long c, const TB* b,
                                     const T* x) {
  T diag, off[6], mass, rb = 0;
  fine_row<T>(op, i, j, k, op.flags[c], diag, off, mass, rb);
  T s = (T)b[c] - diag * x[c];
  for (int q = 0; q < 2 * op.d.dim; ++q) {
    if (off[q] == (T)0) continue;
    int ni, nj, nk;
    neighbour(op.d, i, j, k, q, ni, nj, nk);
    s -= off[q] * x[cell_index(op.d, ni, nj, nk)];
  }
  return s;
}

// Residual of the 2^d children of every coarse cell, summed (= P^T r); also
// clears the coarse iterate.
template <typename T, typename TB>
__global__ void k_fine_resid_restrict(FineOp op, const TB* __restrict__ b, const T* __restrict__ x,
                                      Dims cd, T* __restrict__ bc, T* __restrict__ xc) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= cd.N) return;
  int ci, cj, ck;
  cell_ijk(cd, I, ci, cj, ck);
  T sum = 0;
  for (int dk = 0; dk < 2; ++dk) {
    const int k = 2 * ck + dk;
    if (k >= op.d.n[2]) break;
    for (int dj = 0; dj < 2; ++dj) {
      const int j = 2 * cj + dj;
      if (j >= op.d.n[1]) break;
      for (int di = 0; di < 2; ++di) {
        const int i = 2 * ci + di;
        if (i >= op.d.n[0]) break;
        sum += fine_residual_at<T, TB>(op, i, j, k, cell_index(op.d, i, j, k), b, x);
      }
    }
  }
  bc[I] = sum;
  xc[I] = (T)0;
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

template <typename T>
__global__ void k_coarse_resid_restrict(CoarseOp<T> op, const T* __restrict__ b, const T* __restrict__ x,
                                        Dims cd, T* __restrict__ bc, T* __restrict__ xc) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= cd.N) return;
  int ci, cj, ck;
  cell_ijk(cd, I, ci, cj, ck);
  T sum = 0;
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
        sum += b[c] - op.diag[c] * x[c] - coarse_offsum<T>(op, i, j, k, c, x);
      }
    }
  }
  bc[I] = sum;
  xc[I] = (T)0;
}

// Coarsest level: at most a few cells; a fixed number of symmetric
// Gauss-Seidel sweeps by one thread (exact for one cell).
template <typename T>
__global__ void k_coarsest(CoarseOp<T> op, const T* __restrict__ b, T* __restrict__ x, int sweeps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (long long c = 0; c < op.d.N; ++c) x[c] = (T)0;
  for (int s = 0; s < sweeps; ++s) {
    for (int dir = 0; dir < 2; ++dir)
      for (long long q = 0; q < op.d.N; ++q) {
        const long long c = dir ? (op.d.N - 1 - q) : q;
        int i, j, k;
        cell_ijk(op.d, c, i, j, k);
        x[c] = (b[c] - coarse_offsum<T>(op, i, j, k, c, x)) / op.diag[c];
      }
  }
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
#define RB_TY 8
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
  __device__ inline void row(int i, int j, int k, long long c, T& diag, T off[6], T& rhs) const {
    diag = op.diag[c];
    rhs = b[c];
    for (int a = 0; a < 3; ++a) {
      off[2 * a] = off[2 * a + 1] = (T)0;
      if (a >= op.d.dim) continue;
      int ni, nj, nk;
      if (neighbour(op.d, i, j, k, 2 * a + 1, ni, nj, nk) && op.d.n[a] > 1) off[2 * a + 1] = op.off[a][c];
      if (neighbour(op.d, i, j, k, 2 * a, ni, nj, nk) && op.d.n[a] > 1)
        off[2 * a] = op.off[a][cell_index(op.d, ni, nj, nk)];
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
__global__ __launch_bounds__(RB_THREADS) void k_rb_fused(R rows, const T* __restrict__ xin,
                                                         const T* __restrict__ xc, Dims cd, T* __restrict__ xout,
                                                         int zchunk) {
  __shared__ T buf[4][RB_PLANE];
  const Dims& d = rows.dims();
  const int tx0 = blockIdx.x * RB_TX, ty0 = blockIdx.y * RB_TY;
  const int z0 = blockIdx.z * zchunk;
  const int z1 = min(z0 + zchunk, d.n[2]);
  const bool zdim = d.dim == 3;
  auto slot = [&](int k) { return buf[((k % 4) + 4) % 4]; };
  if (zdim) {
    for (int k = z0 - 2; k <= z0 + 1; ++k) rb_load_plane<T>(rows, k, tx0, ty0, xin, xc, cd, slot(k));
    __syncthreads();
    // red on the tile + 1 ring of the two planes before the first black one
    rb_update_plane<T, 1>(rows, z0 - 1, tx0, ty0, 0, slot(z0 - 2), slot(z0 - 1),
                       slot(z0));
    __syncthreads();
    rb_update_plane<T, 1>(rows, z0, tx0, ty0, 0, slot(z0 - 1), slot(z0), slot(z0 + 1));
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
      rb_load_plane<T>(rows, k + 2, tx0, ty0, xin, xc, cd, slot(k + 2));
      __syncthreads();
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

// wrap index v along axis a; false if it lies outside a non-periodic domain
__device__ inline bool wrap_axis(const Dims& d, int a, int& v) {
  if (v >= 0 && v < d.n[a]) return true;
  if (!d.per[a]) return false;
  v = (v % d.n[a] + d.n[a]) % d.n[a];
  return true;
}

template <typename T, int TX, int TY>
__device__ inline void fine_load_x(const Dims& d, int kk, int tx0, int ty0, const T* __restrict__ xin,
                                   const T* __restrict__ xc, const Dims& cd, T (&v)[FineTile<TX, TY>::NX]) {
  using FT = FineTile<TX, TY>;
  int k = kk;
  const bool pz = wrap_axis(d, 2, k);
#pragma unroll
  for (int e = 0; e < FT::NX; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    T s = (T)0;
    if (pz && t < FT::PL && (xin || xc)) {
      int i = tx0 + t % FT::PX - 2, j = ty0 + t / FT::PX - 2;
      if (wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
        if (xin) s = xin[cell_index(d, i, j, k)];
        if (xc) s += xc[cell_index(cd, i >> 1, j >> 1, k >> 1)];
      }
    }
    v[e] = s;
  }
}

template <int TX, int TY>
__device__ inline void fine_load_rf(const Dims& d, int kk, int tx0, int ty0, const double* __restrict__ rhs,
                                    const uint8_t* __restrict__ flags, double (&r)[FineTile<TX, TY>::NQ],
                                    uint8_t (&f)[FineTile<TX, TY>::NQ]) {
  using FT = FineTile<TX, TY>;
  int k = kk;
  const bool pz = wrap_axis(d, 2, k);
#pragma unroll
  for (int e = 0; e < FT::NQ; ++e) {
    const int t = threadIdx.x + e * RB_THREADS;
    r[e] = 0.0;
    f[e] = 0;
    if (pz && t < FT::QL) {
      int i = tx0 + t % FT::QX - 1, j = ty0 + t / FT::QX - 1;
      if (wrap_axis(d, 0, i) && wrap_axis(d, 1, j)) {
        const long long c = cell_index(d, i, j, k);
        r[e] = rhs[c];
        f[e] = flags[c];
      }
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

template <int TX, int TY>
__device__ inline void fine_store_rf(const double (&r)[FineTile<TX, TY>::NQ], const uint8_t (&f)[FineTile<TX, TY>::NQ],
                                     double* rs, uint8_t* fs) {
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
};

template <typename T>
__device__ inline RegularRow<T> regular_row(const FineOp& op) {
  const T ih2 = (T)op.ih2;
  T w[2], inv[2];
  for (int ph = 0; ph < 2; ++ph) {
    w[ph] = (T)op.coef[ph] * ih2;
    T dg = (op.sys == EBIT_SYS_HEAT) ? (T)op.mass[ph] : (T)0;
    for (int s = 0; s < 2 * op.d.dim; ++s) dg += w[ph];
    inv[ph] = (T)1 / dg;
  }
  return RegularRow<T>{w[0], w[1], inv[0], inv[1]};
}

// Update the cells of one colour of plane k on the tile (RING = 0) or on the
// tile + 1 ring (RING = 1) from LDS.  Threads walk only the cells of the
// colour; regular cells take the per-phase constant row, cells with a cut
// link or a wall face the full row of fine_row.
template <typename T, int TX, int TY, int RING>
__device__ inline void fine_update(const FineOp& op, const RegularRow<T>& rr, int k, int tx0, int ty0, int color,
                                   const T* pm, T* p0, const T* pp, const double* rq, const uint8_t* fq) {
  using FT = FineTile<TX, TY>;
  constexpr int WX = TX + 2 * RING, WY = TY + 2 * RING, HX = WX / 2;
  static_assert(WX % 2 == 0, "tile width must be even");
  const Dims& d = op.d;
  int kw = k;
  if (!wrap_axis(d, 2, kw)) return;
  const bool zwall = d.dim == 3 && !d.per[2] && (kw == 0 || kw == d.n[2] - 1);
  for (int t = threadIdx.x; t < HX * WY; t += RB_THREADS) {
    const int ly = t / HX - RING;
    const int j = ty0 + ly;
    const int lx = 2 * (t % HX) - RING + ((color + tx0 - RING + j + k) & 1);
    const int i = tx0 + lx;
    int iw = i, jw = j;
    if (!wrap_axis(d, 0, iw) || !wrap_axis(d, 1, jw)) continue;
    const int qq = (ly + 1) * FT::QX + (lx + 1);
    const int q = (ly + 2) * FT::PX + (lx + 2);
    const uint8_t f = fq[qq];
    const bool wall = zwall || (!d.per[0] && (iw == 0 || iw == d.n[0] - 1)) ||
                      (!d.per[1] && (jw == 0 || jw == d.n[1] - 1));
    if (!(f & F_CUT) && !wall) {
      const bool liq = (f & F_LIQ) != 0;
      T xn = (p0[q - 1] + p0[q + 1]) + (p0[q - FT::PX] + p0[q + FT::PX]);
      if (d.dim == 3) xn += pm[q] + pp[q];
      p0[q] = ((T)rq[qq] + (liq ? rr.w1 : rr.w0) * xn) * (liq ? rr.inv1 : rr.inv0);
    } else {
      T diag, off[6], mass, rb = 0;
      fine_row<T>(op, iw, jw, kw, f, diag, off, mass, rb);
      T sum = (T)rq[qq] - off[0] * p0[q - 1] - off[1] * p0[q + 1];
      sum -= off[2] * p0[q - FT::PX] + off[3] * p0[q + FT::PX];
      if (d.dim == 3) sum -= off[4] * pm[q] + off[5] * pp[q];
      p0[q] = sum / diag;
    }
  }
}

template <typename T, int TX, int TY>
__device__ inline void fine_write(const Dims& d, int k, int tx0, int ty0, const T* p0, T* __restrict__ xout) {
  using FT = FineTile<TX, TY>;
  for (int t = threadIdx.x; t < TX * TY; t += RB_THREADS) {
    const int lx = t % TX, ly = t / TX;
    const int i = tx0 + lx, j = ty0 + ly;
    if (i < d.n[0] && j < d.n[1]) xout[cell_index(d, i, j, k)] = p0[(ly + 2) * FT::PX + (lx + 2)];
  }
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(RB_THREADS) void k_rb_fine(FineOp op, const double* __restrict__ rhs,
                                                        const T* __restrict__ xin, const T* __restrict__ xc, Dims cd,
                                                        T* __restrict__ xout, int zchunk) {
  using FT = FineTile<TX, TY>;
  __shared__ T xs[4][FT::PL];
  __shared__ double rs[2][FT::QL];
  __shared__ uint8_t fs[2][FT::QL];
  const Dims& d = op.d;
  const RegularRow<T> rr = regular_row<T>(op);
  const int tx0 = blockIdx.x * TX, ty0 = blockIdx.y * TY;
  T xv[FT::NX];
  double rv[FT::NQ];
  uint8_t fv[FT::NQ];
  if (d.dim < 3) {
    fine_load_x<T, TX, TY>(d, 0, tx0, ty0, xin, xc, cd, xv);
    fine_load_rf<TX, TY>(d, 0, tx0, ty0, rhs, op.flags, rv, fv);
    fine_store<T, TX, TY>(xv, xs[0]);
    fine_store_rf<TX, TY>(rv, fv, rs[0], fs[0]);
    __syncthreads();
    fine_update<T, TX, TY, 1>(op, rr, 0, tx0, ty0, 0, xs[0], xs[0], xs[0], rs[0], fs[0]);
    __syncthreads();
    fine_update<T, TX, TY, 0>(op, rr, 0, tx0, ty0, 1, xs[0], xs[0], xs[0], rs[0], fs[0]);
    __syncthreads();
    fine_write<T, TX, TY>(d, 0, tx0, ty0, xs[0], xout);
    return;
  }
  // slots: x plane p in xs[p & 3], r / flags of plane p in rs[p & 1] (p may be negative)
  const int z0 = blockIdx.z * zchunk;
  const int z1 = min(z0 + zchunk, d.n[2]);
  {
    T xa[FT::NX], xb[FT::NX];
    double ra[FT::NQ];
    uint8_t fa[FT::NQ];
    fine_load_x<T, TX, TY>(d, z0 - 2, tx0, ty0, xin, xc, cd, xv);
    fine_load_x<T, TX, TY>(d, z0 - 1, tx0, ty0, xin, xc, cd, xa);
    fine_load_x<T, TX, TY>(d, z0, tx0, ty0, xin, xc, cd, xb);
    fine_load_rf<TX, TY>(d, z0 - 1, tx0, ty0, rhs, op.flags, rv, fv);
    fine_load_rf<TX, TY>(d, z0, tx0, ty0, rhs, op.flags, ra, fa);
    fine_store<T, TX, TY>(xv, xs[(z0 - 2) & 3]);
    fine_store<T, TX, TY>(xa, xs[(z0 - 1) & 3]);
    fine_store<T, TX, TY>(xb, xs[z0 & 3]);
    fine_store_rf<TX, TY>(rv, fv, rs[(z0 - 1) & 1], fs[(z0 - 1) & 1]);
    fine_store_rf<TX, TY>(ra, fa, rs[z0 & 1], fs[z0 & 1]);
    fine_load_x<T, TX, TY>(d, z0 + 1, tx0, ty0, xin, xc, cd, xv);
    fine_store<T, TX, TY>(xv, xs[(z0 + 1) & 3]);
  }
  __syncthreads();
  fine_update<T, TX, TY, 1>(op, rr, z0 - 1, tx0, ty0, 0, xs[(z0 - 2) & 3], xs[(z0 - 1) & 3], xs[z0 & 3],
                         rs[(z0 - 1) & 1], fs[(z0 - 1) & 1]);
  __syncthreads();
  fine_update<T, TX, TY, 1>(op, rr, z0, tx0, ty0, 0, xs[(z0 - 1) & 3], xs[z0 & 3], xs[(z0 + 1) & 3], rs[z0 & 1],
                         fs[z0 & 1]);
  fine_load_x<T, TX, TY>(d, z0 + 2, tx0, ty0, xin, xc, cd, xv);
  fine_load_rf<TX, TY>(d, z0 + 1, tx0, ty0, rhs, op.flags, rv, fv);
  __syncthreads();
  for (int k = z0; k < z1; ++k) {
    // plane k+2's iterate replaces plane k-2's, plane k+1's r / flags replace plane k-1's
    fine_store<T, TX, TY>(xv, xs[(k + 2) & 3]);
    fine_store_rf<TX, TY>(rv, fv, rs[(k + 1) & 1], fs[(k + 1) & 1]);
    __syncthreads();
    if (k + 1 < z1) {
      fine_load_x<T, TX, TY>(d, k + 3, tx0, ty0, xin, xc, cd, xv);
      fine_load_rf<TX, TY>(d, k + 2, tx0, ty0, rhs, op.flags, rv, fv);
    }
    fine_update<T, TX, TY, 1>(op, rr, k + 1, tx0, ty0, 0, xs[k & 3], xs[(k + 1) & 3], xs[(k + 2) & 3], rs[(k + 1) & 1],
                           fs[(k + 1) & 1]);
    __syncthreads();
    fine_update<T, TX, TY, 0>(op, rr, k, tx0, ty0, 1, xs[(k - 1) & 3], xs[k & 3], xs[(k + 1) & 3], rs[k & 1],
                           fs[k & 1]);
    __syncthreads();
    fine_write<T, TX, TY>(d, k, tx0, ty0, xs[k & 3], xout);
  }
}

// ---------------------------------------------------------------------------
// tail of the V-cycle: every level small enough to sit in LDS, in one
// work-group (no launch per smoothing sweep on the coarse levels).  The
// coefficients of all tail levels are staged into LDS once, at the start.
// ---------------------------------------------------------------------------
#define EBIT_TAIL_MAX 16
#define EBIT_TAIL_THREADS 1024

// LDS block of one tail level: x, b, diag, off[0 .. dim-1], N elements each.
struct TailLevel {
  Dims d;
  int base;  // element offset of x
};

__host__ __device__ inline long long tail_level_elems(const Dims& d) { return (3 + d.dim) * d.N; }

template <typename T>
struct TailArgs {
  int nl;  // levels in the tail; the last one is the coarsest
  int nu1, nu2;
  TailLevel L[EBIT_TAIL_MAX];
  const T* diag[EBIT_TAIL_MAX];
  const T* off[EBIT_TAIL_MAX][3];
  const T* bg;  // right-hand side of the top tail level
  T* xg;        // its correction (output)
};

// The 1024 threads of the tail form 32 rows of 32: thread row ty takes grid
// rows (j, k) = ty, ty + 32, ... and lane tx the cells i = 2 tx + parity,
// + 64, ... of one colour (or every cell for the grid transfers).
struct TailRow {
  int j, k;
  __device__ TailRow(const Dims& d, int r) : j(r % d.n[1]), k(r / d.n[1]) {}
  __device__ void next(const Dims& d) {
    j += 32;
    while (j >= d.n[1]) {
      j -= d.n[1];
      ++k;
    }
  }
};

// sum over the neighbours of cell q = (i, j, k) of coupling x neighbour; the
// same neighbour set as neighbour() (periodic wrap, none across a wall)
template <typename T>
__device__ inline T tail_offsum(const T* x, const Dims& d, int i, int j, int k, int q) {
  const int N = (int)d.N;
  T s = 0;
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const int s1 = n0, s2 = n0 * n1;
  {
    const T* o = x + 3 * N;
    if (i + 1 < n0) s += o[q] * x[q + 1];
    else if (d.per[0]) s += o[q] * x[q + 1 - n0];
    if (i > 0) s += o[q - 1] * x[q - 1];
    else if (d.per[0]) s += o[q + n0 - 1] * x[q + n0 - 1];
  }
  if (d.dim >= 2) {
    const T* o = x + 4 * N;
    if (j + 1 < n1) s += o[q] * x[q + s1];
    else if (d.per[1]) s += o[q] * x[q + s1 - s2];
    if (j > 0) s += o[q - s1] * x[q - s1];
    else if (d.per[1]) s += o[q + s2 - s1] * x[q + s2 - s1];
  }
  if (d.dim == 3) {
    const T* o = x + 5 * N;
    if (k + 1 < n2) s += o[q] * x[q + s2];
    else if (d.per[2]) s += o[q] * x[q + s2 - N];
    if (k > 0) s += o[q - s2] * x[q - s2];
    else if (d.per[2]) s += o[q + N - s2] * x[q + N - s2];
  }
  return s;
}

template <typename T>
__device__ inline void tail_sweep(T* sm, const TailLevel& L, int color) {
  const Dims& d = L.d;
  const int N = (int)d.N;
  T* x = sm + L.base;
  const T* b = x + N;
  const T* dg = x + 2 * N;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int rows = d.n[1] * d.n[2];
  TailRow r(d, ty);
  for (int row = ty; row < rows; row += 32, r.next(d)) {
    const int base = row * d.n[0];
    for (int i = 2 * tx + ((r.j + r.k + color) & 1); i < d.n[0]; i += 64) {
      const int q = base + i;
      x[q] = (b[q] - tail_offsum<T>(x, d, i, r.j, r.k, q)) / dg[q];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(EBIT_TAIL_THREADS) void k_tail(TailArgs<T> a) {
  extern __shared__ __align__(16) unsigned char tail_smem[];
  T* sm = reinterpret_cast<T*>(tail_smem);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5;
  for (int l = 0; l < a.nl; ++l) {
    const TailLevel& L = a.L[l];
    const int N = (int)L.d.N;
    T* x = sm + L.base;
    const T* dg = a.diag[l];
    const T* o0 = a.off[l][0];
    const T* o1 = a.off[l][1];
    const T* o2 = a.off[l][2];
    for (int q = tid; q < N; q += nth) {
      x[2 * N + q] = dg[q];
      x[3 * N + q] = o0[q];
      if (L.d.dim >= 2) x[4 * N + q] = o1[q];
      if (L.d.dim == 3) x[5 * N + q] = o2[q];
      if (l == 0) {
        x[N + q] = a.bg[q];
        x[q] = (T)0;
      }
    }
  }
  __syncthreads();
  for (int l = 0; l < a.nl - 1; ++l) {
    const TailLevel& L = a.L[l];
    const Dims& d = L.d;
    const int N = (int)d.N;
    T* x = sm + L.base;
    const T* b = x + N;
    const T* dg = x + 2 * N;
    for (int s = 0; s < a.nu1; ++s)
      for (int col = 0; col < 2; ++col) {
        tail_sweep(sm, L, col);
        __syncthreads();
      }
    // residual of the 2^d children, summed into the coarse right-hand side
    const TailLevel& C = a.L[l + 1];
    const Dims& cd = C.d;
    T* xc = sm + C.base;
    T* bc = xc + cd.N;
    const int crows = cd.n[1] * cd.n[2];
    TailRow r(cd, ty);
    for (int row = ty; row < crows; row += 32, r.next(cd)) {
      for (int ci = tx; ci < cd.n[0]; ci += 32) {
        T sum = 0;
        for (int dk = 0; dk < 2; ++dk) {
          const int k = 2 * r.k + dk;
          if (k >= d.n[2]) break;
          for (int dj = 0; dj < 2; ++dj) {
            const int j = 2 * r.j + dj;
            if (j >= d.n[1]) break;
            for (int di = 0; di < 2; ++di) {
              const int i = 2 * ci + di;
              if (i >= d.n[0]) break;
              const int q = i + d.n[0] * (j + d.n[1] * k);
              sum += b[q] - dg[q] * x[q] - tail_offsum<T>(x, d, i, j, k, q);
            }
          }
        }
        const int I = row * cd.n[0] + ci;
        bc[I] = sum;
        xc[I] = (T)0;
      }
    }
    __syncthreads();
  }
  {
    // coarsest level: symmetric Gauss-Seidel by one thread (exact for one cell)
    const TailLevel& L = a.L[a.nl - 1];
    const Dims& d = L.d;
    const int N = (int)d.N;
    T* x = sm + L.base;
    const T* b = x + N;
    const T* dg = x + 2 * N;
    if (tid == 0) {
      const int sweeps = N == 1 ? 1 : 50;
      for (int s = 0; s < sweeps; ++s)
        for (int dir = 0; dir < 2; ++dir)
          for (int qq = 0; qq < N; ++qq) {
            const int q = dir ? (N - 1 - qq) : qq;
            const int i = q % d.n[0], j = (q / d.n[0]) % d.n[1], k = q / (d.n[0] * d.n[1]);
            x[q] = (b[q] - tail_offsum<T>(x, d, i, j, k, q)) / dg[q];
          }
    }
    __syncthreads();
  }
  for (int l = a.nl - 2; l >= 0; --l) {
    const TailLevel& L = a.L[l];
    const Dims& d = L.d;
    T* x = sm + L.base;
    const TailLevel& C = a.L[l + 1];
    const T* xc = sm + C.base;
    const int rows = d.n[1] * d.n[2];
    TailRow r(d, ty);
    for (int row = ty; row < rows; row += 32, r.next(d)) {
      const int cb = C.d.n[0] * ((r.j >> 1) + C.d.n[1] * (r.k >> 1));
      for (int i = tx; i < d.n[0]; i += 32) x[row * d.n[0] + i] += xc[cb + (i >> 1)];
    }
    __syncthreads();
    for (int s = 0; s < a.nu2; ++s)
      for (int col = 1; col >= 0; --col) {
        tail_sweep(sm, L, col);
        __syncthreads();
      }
  }
  {
    const int N = (int)a.L[0].d.N;
    const T* x = sm + a.L[0].base;
    for (int q = tid; q < N; q += nth) a.xg[q] = x[q];
  }
}

// ---------------------------------------------------------------------------
// hierarchy construction
// ---------------------------------------------------------------------------
struct BuildOut {
  Dims cd;
  double* diag;
  double* mass;
  double* off[3];
};

// aggregate index of a (wrapped) fine cell along each axis: q >> 1
__global__ void k_build_from_fine(FineOp op, BuildOut o) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= o.cd.N) return;
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
        for (int s = 0; s < 2 * op.d.dim; ++s) {
          if (off[s] == 0.0) continue;
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
  o.diag[I] = M + 0.5 * F;
  o.mass[I] = M;
  for (int a = 0; a < 3; ++a)
    if (o.off[a]) o.off[a][I] = 0.5 * cross[a];
}

__global__ void k_build_from_coarse(CoarseOp<double> op, BuildOut o) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= o.cd.N) return;
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
        M += op.mass[c];
        F += op.diag[c] - op.mass[c];
        for (int s = 0; s < 2 * op.d.dim; ++s) {
          int ni, nj, nk;
          if (!neighbour(op.d, i, j, k, s, ni, nj, nk)) continue;
          const long long m = cell_index(op.d, ni, nj, nk);
          const double off = (s & 1) ? op.off[s >> 1][c] : op.off[s >> 1][m];
          if (off == 0.0) continue;
          const bool same = (ni >> 1) == ci && (nj >> 1) == cj && (nk >> 1) == ck;
          if (same)
            F += off;
          else if (s & 1)
            cross[s >> 1] += off;
        }
      }
    }
  }
  o.diag[I] = M + 0.5 * F;
  o.mass[I] = M;
  for (int a = 0; a < 3; ++a)
    if (o.off[a]) o.off[a][I] = 0.5 * cross[a];
}

__global__ void k_cast_level(long long n, int dim, const double* d64, const double* o0, const double* o1,
                             const double* o2, float* d32, float* p0, float* p1, float* p2) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  d32[t] = (float)d64[t];
  p0[t] = (float)o0[t];
  if (dim > 1) p1[t] = (float)o1[t];
  if (dim > 2) p2[t] = (float)o2[t];
}

// ---------------------------------------------------------------------------
// outer loop kernels (FP64) with deterministic two-stage reductions
// ---------------------------------------------------------------------------
#define GRID_STRIDE(c, N) \
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < (N); c += (long long)gridDim.x * blockDim.x)

template <int NV>
__device__ inline void write_partials(double (&v)[NV], double* partial) {
  __shared__ double sh[NV * 4];
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < NV; ++q) partial[q * gridDim.x + blockIdx.x] = v[q];
}

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
__global__ void k_resid_init(FineOp op, const double* __restrict__ b, const double* __restrict__ x,
                             double* __restrict__ r, double* partial) {
  double v[3] = {0, 0, 0};
  GRID_STRIDE(c, op.d.N) {
    const double bc = b[c];
    double rc = bc, ac = fabs(bc);
    if (x) {
      int i, j, k;
      cell_ijk(op.d, c, i, j, k);
      double diag, off[6], mass, rb = 0, mx;
      fine_row<double>(op, i, j, k, op.flags[c], diag, off, mass, rb, &mx);
      const double xc = x[c];
      double hi = bc, lo = 0.0;
      {
        const double p = mx * xc;
        dd_add(hi, lo, -p, -fma(mx, xc, -p));
      }
      ac += fabs(diag * xc);
      for (int q = 0; q < 2 * op.d.dim; ++q) {
        if (off[q] == 0.0) continue;
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
    v[0] += bc * bc;
    v[1] += rc * rc;
    v[2] += ac * ac;
  }
  write_partials<3>(v, partial);
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
    for (int q = 0; q < 2 * op.d.dim; ++q) {
      if (off[q] == 0.0) continue;
      int ni, nj, nk;
      neighbour(op.d, i, j, k, q, ni, nj, nk);
      s -= off[q] * (xc - x[cell_index(op.d, ni, nj, nk)]);
    }
    y[c] = s;
  }
}

// heat right-hand side: b = rho cp/dt T* + interface and wall terms
__global__ void k_heat_rhs(FineOp op, const double* __restrict__ Ts, double* __restrict__ b) {
  GRID_STRIDE(c, op.d.N) {
    int i, j, k;
    cell_ijk(op.d, c, i, j, k);
    const uint8_t f = op.flags[c];
    double diag, off[6], mass;
    double rb = op.mass[(f & F_LIQ) ? 1 : 0] * Ts[c];
    fine_row<double>(op, i, j, k, f, diag, off, mass, rb);
    b[c] = rb;
  }
}

// z.r and z.q (q = A p of the previous iteration)
template <typename TZ>
__global__ void k_dots_zr_zq(long long N, const TZ* __restrict__ z, const double* __restrict__ r,
                             const double* __restrict__ q, double* partial) {
  double v[2] = {0, 0};
  GRID_STRIDE(c, N) {
    const double zc = (double)z[c];
    v[0] += zc * r[c];
    if (q) v[1] += zc * q[c];
  }
  write_partials<2>(v, partial);
}

// p_new = z + beta p_old; q = A p_new; partial p.q
template <typename TZ>
__global__ void k_p_update_apply(FineOp op, const TZ* __restrict__ z, const double* __restrict__ p_old,
                                 double* __restrict__ p_new, double* __restrict__ q, const Scal* sc,
                                 int first, double* partial) {
  const double beta = first ? 0.0 : sc->beta;
  double v[1] = {0};
  GRID_STRIDE(c, op.d.N) {
    int i, j, k;
    cell_ijk(op.d, c, i, j, k);
    double diag, off[6], mass, rb = 0, mx;
    fine_row<double>(op, i, j, k, op.flags[c], diag, off, mass, rb, &mx);
    const double pc = first ? (double)z[c] : (double)z[c] + beta * p_old[c];
    double s = mx * pc;
    for (int qq = 0; qq < 2 * op.d.dim; ++qq) {
      if (off[qq] == 0.0) continue;
      int ni, nj, nk;
      neighbour(op.d, i, j, k, qq, ni, nj, nk);
      const long long m = cell_index(op.d, ni, nj, nk);
      const double pm = first ? (double)z[m] : (double)z[m] + beta * p_old[m];
      s -= off[qq] * (pc - pm);
    }
    p_new[c] = pc;
    q[c] = s;
    v[0] += pc * s;
  }
  write_partials<1>(v, partial);
}

// x += alpha p; r -= alpha q; partial r.r
__global__ void k_update_xr(long long N, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q, const Scal* sc,
                            double* partial) {
  const double alpha = sc->alpha;
  double v[1] = {0};
  GRID_STRIDE(c, N) {
    x[c] += alpha * p[c];
    const double rc = r[c] - alpha * q[c];
    r[c] = rc;
    v[0] += rc * rc;
  }
  write_partials<1>(v, partial);
}

// finalize kinds
enum { FIN_INIT = 0, FIN_GAMMA = 1, FIN_DELTA = 2, FIN_RR = 3, FIN_MAX = 4, FIN_SUM1 = 5 };

__global__ void k_finalize(const double* __restrict__ partial, int nb, int nv, Scal* sc, int kind, int first) {
  __shared__ double sh[4 * 4];
  double v[3] = {0, 0, 0};
  for (int q = 0; q < nv; ++q) {
    double s = 0;
    if (kind == FIN_MAX) {
      for (int t = threadIdx.x; t < nb; t += blockDim.x) s = fmax(s, partial[q * nb + t]);
    } else {
      for (int t = threadIdx.x; t < nb; t += blockDim.x) s += partial[q * nb + t];
    }
    v[q] = s;
  }
  if (kind == FIN_MAX) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double m = wave_max(v[0]);
    if (lane == 0) sh[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) v[0] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  } else {
    block_sum<3>(v, sh);
  }
  if (threadIdx.x != 0) return;
  bool bad = false;
  switch (kind) {
    case FIN_INIT:
      sc->bb = v[0];
      sc->rr = v[1];
      sc->aa = v[2];
      bad = !isfinite(v[0]) || !isfinite(v[1]);
      break;
    case FIN_GAMMA: {
      const double gnew = v[0];
      sc->beta = first ? 0.0 : -sc->alpha * v[1] / sc->gamma;
      sc->gamma = gnew;
      sc->zq = v[1];
      bad = !isfinite(gnew);
      break;
    }
    case FIN_DELTA:
      sc->delta = v[0];
      sc->alpha = sc->gamma / v[0];
      bad = !isfinite(sc->alpha);
      break;
    case FIN_RR:
      sc->rr = v[0];
      bad = !isfinite(v[0]);
      break;
    case FIN_MAX:
      sc->divmax = v[0];
      break;
    case FIN_SUM1:
      sc->red[0] = v[0];
      break;
  }
  if (bad) sc->err |= ERR_NAN;
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + EBIT_BLOCK - 1) / EBIT_BLOCK); }

}  // namespace ebit

using namespace ebit;

extern "C" {

hipError_t ebit_launch_fill_f64(long long n, double* x, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<double>, dim3(nblk(n)), dim3(EBIT_BLOCK), 0, st, n, x, v);
  return hipGetLastError();
}
hipError_t ebit_launch_fill_f32(long long n, float* x, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<float>, dim3(nblk(n)), dim3(EBIT_BLOCK), 0, st, n, x, v);
  return hipGetLastError();
}

// Build the coarse hierarchy of one system: level 1 from the matrix-free fine
// operator, then each level from the one above; FP32 copies if wanted.
hipError_t ebit_build_hierarchy(const FineOp* op, EbitLevelHost* lv, int nlev, int sys, int want32,
                                hipStream_t st) {
  for (int l = 1; l < nlev; ++l) {
    BuildOut o;
    o.cd = lv[l].d;
    o.diag = lv[l].diag64[sys];
    o.mass = lv[l].mass64[sys];
    for (int a = 0; a < 3; ++a) o.off[a] = (a < o.cd.dim) ? lv[l].off64[sys][a] : nullptr;
    if (l == 1) {
      hipLaunchKernelGGL(k_build_from_fine, dim3(nblk(o.cd.N)), dim3(EBIT_BLOCK), 0, st, *op, o);
    } else {
      CoarseOp<double> f;
      f.d = lv[l - 1].d;
      f.diag = lv[l - 1].diag64[sys];
      f.mass = lv[l - 1].mass64[sys];
      for (int a = 0; a < 3; ++a) f.off[a] = (a < f.d.dim) ? lv[l - 1].off64[sys][a] : nullptr;
      hipLaunchKernelGGL(k_build_from_coarse, dim3(nblk(o.cd.N)), dim3(EBIT_BLOCK), 0, st, f, o);
    }
    if (want32) {
      const int dim = o.cd.dim;
      hipLaunchKernelGGL(k_cast_level, dim3(nblk(o.cd.N)), dim3(EBIT_BLOCK), 0, st, o.cd.N, dim,
                         o.diag, o.off[0], o.off[1], o.off[2], lv[l].diag32[sys], lv[l].off32[sys][0],
                         dim > 1 ? lv[l].off32[sys][1] : nullptr, dim > 2 ? lv[l].off32[sys][2] : nullptr);
    }
  }
  return hipGetLastError();
}

}  // extern "C"

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
    pr->launches[pr->kid[i]] += 1;
  }
  pr->npend = 0;
  return hipSuccess;
}

// Bracket one launch with events when profiling is on.
struct ProfScope {
  EbitProfiler* pr;
  hipStream_t st;
  int slot;
  ProfScope(EbitProfiler* p, int kid, hipStream_t s) : pr(p), st(s), slot(-1) {
    if (!pr || !pr->on) return;
    if (pr->npend == EBIT_PROF_CAP) (void)ebit_prof_flush(pr);
    slot = pr->npend++;
    pr->kid[slot] = kid;
    (void)hipEventRecord(pr->ev0[slot], st);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(pr->ev1[slot], st);
  }
};

// ---- V-cycle driver (templated on the inner precision) ----
template <typename T>
static CoarseOp<T> coarse_op(const EbitLevelHost& L, int sys);
template <>
CoarseOp<double> coarse_op<double>(const EbitLevelHost& L, int sys) {
  CoarseOp<double> c;
  c.d = L.d;
  c.diag = L.diag64[sys];
  for (int a = 0; a < 3; ++a) c.off[a] = (a < L.d.dim) ? L.off64[sys][a] : nullptr;
  c.mass = L.mass64[sys];
  return c;
}
template <>
CoarseOp<float> coarse_op<float>(const EbitLevelHost& L, int sys) {
  CoarseOp<float> c;
  c.d = L.d;
  c.diag = L.diag32[sys];
  for (int a = 0; a < 3; ++a) c.off[a] = (a < L.d.dim) ? L.off32[sys][a] : nullptr;
  c.mass = L.mass64[sys];
  return c;
}
template <typename T>
static T* lvx(const EbitLevelHost& L);
template <>
double* lvx<double>(const EbitLevelHost& L) { return L.x64; }
template <>
float* lvx<float>(const EbitLevelHost& L) { return L.x32; }
template <typename T>
static T* lvb(const EbitLevelHost& L);
template <>
double* lvb<double>(const EbitLevelHost& L) { return L.b64; }
template <>
float* lvb<float>(const EbitLevelHost& L) { return L.b32; }

// First coarse level (>= 1) from which the tail kernel takes over: the
// remaining levels (x, b and coefficients) must fit lds_bytes of LDS and the
// top one hold at most tail_cells cells.
template <typename T>
static int tail_start(const EbitLevelHost* lv, int nlev, int tail_cells, int lds_bytes) {
  if (tail_cells <= 0) return nlev;
  long long tot = 0;
  int lt = nlev;
  for (int l = nlev - 1; l >= 1; --l) {
    tot += tail_level_elems(lv[l].d);
    if (tot * (long long)sizeof(T) > lds_bytes || lv[l].d.N > tail_cells || nlev - l > EBIT_TAIL_MAX) break;
    lt = l;
  }
  return lt;
}

template <typename T>
static T* lvxb(const EbitLevelHost& L);
template <>
double* lvxb<double>(const EbitLevelHost& L) { return L.x64b; }
template <>
float* lvxb<float>(const EbitLevelHost& L) { return L.x32b; }

static inline dim3 rb_grid(const Dims& d, int zchunk) {
  return dim3((unsigned)((d.n[0] + RB_TX - 1) / RB_TX), (unsigned)((d.n[1] + RB_TY - 1) / RB_TY),
              (unsigned)((d.n[2] + zchunk - 1) / zchunk));
}

// z-chunk: enough work-groups to fill the chip, at most 32 planes each
static inline int rb_zchunk(const Dims& d) {
  if (d.dim < 3) return 1;
  const long long tiles = (long long)((d.n[0] + RB_TX - 1) / RB_TX) * ((d.n[1] + RB_TY - 1) / RB_TY);
  int zc = 32;
  while (zc > 4 && tiles * ((d.n[2] + zc - 1) / zc) < 1024) zc >>= 1;
  return zc;
}

// S = nu1 + nu2 fused sweeps on one level; sweep s (1-based) writes X when
// S - s is even and Xb otherwise, so the last one lands in X.  The first
// pre-smoothing sweep starts from zero; the first post-smoothing sweep adds
// the coarse correction xc on load.  launch(in, xc, out) issues one sweep.
template <typename T, typename L>
static void smooth_pre(const L& launch, int nu1, int S, T* X, T* Xb, hipStream_t st, EbitProfiler* pf, int kc) {
  const T* in = nullptr;
  for (int s = 1; s <= nu1; ++s) {
    T* out = ((S - s) % 2 == 0) ? X : Xb;
    ProfScope ps(pf, kc, st);
    launch(in, (const T*)nullptr, out);
    in = out;
  }
}
template <typename T, typename L>
static void smooth_post(const L& launch, int nu1, int S, T* X, T* Xb, const T* xc, hipStream_t st, EbitProfiler* pf,
                        int kc) {
  const T* in = ((S - nu1) % 2 == 0) ? X : Xb;
  for (int s = nu1 + 1; s <= S; ++s) {
    T* out = ((S - s) % 2 == 0) ? X : Xb;
    ProfScope ps(pf, kc, st);
    launch(in, s == nu1 + 1 ? xc : (const T*)nullptr, out);
    in = out;
  }
}

// fine-level sweep launcher: 64 x 8 tiles marching along z in 3D, 64 x 4
// tiles in 2D (twice the work-groups for the single plane)
template <typename T>
struct FineSweep {
  FineOp op;
  const double* r;
  Dims cd;
  hipStream_t st;
  void operator()(const T* in, const T* xc, T* out) const {
    const Dims& d = op.d;
    if (d.dim == 3) {
      const int zc = rb_zchunk(d);
      const dim3 g((unsigned)((d.n[0] + 63) / 64), (unsigned)((d.n[1] + 7) / 8), (unsigned)((d.n[2] + zc - 1) / zc));
      hipLaunchKernelGGL((k_rb_fine<T, 64, 8>), g, dim3(RB_THREADS), 0, st, op, r, in, xc, cd, out, zc);
    } else {
      const dim3 g((unsigned)((d.n[0] + 63) / 64), (unsigned)((d.n[1] + 3) / 4), 1);
      hipLaunchKernelGGL((k_rb_fine<T, 64, 4>), g, dim3(RB_THREADS), 0, st, op, r, in, xc, cd, out, 1);
    }
  }
};

// explicit coarse-level sweep launcher
template <typename T>
struct CoarseSweep {
  CoarseRows<T> rows;
  Dims cd;
  hipStream_t st;
  void operator()(const T* in, const T* xc, T* out) const {
    const Dims& d = rows.op.d;
    const int zc = rb_zchunk(d);
    hipLaunchKernelGGL((k_rb_fused<T, CoarseRows<T>>), rb_grid(d, zc), dim3(RB_THREADS), 0, st, rows, in, xc, cd,
                       out, zc);
  }
};

// One V(nu1, nu2) cycle on A z = r (zero initial guess); the fine level is
// matrix-free, levels 1 .. lt-1 explicit, levels lt .. in the tail kernel.
template <typename T>
static hipError_t vcycle(const FineOp& op, const EbitLevelHost* lv, int nlev, const double* r, T* z, T* zb,
                         int nu1, int nu2, int tail_cells, int tail_lds, hipStream_t st, EbitProfiler* pf) {
  const int sys = op.sys;
  const int S = nu1 + nu2;
  const FineSweep<T> fine{op, r, nlev > 1 ? lv[1].d : op.d, st};
  if (nlev == 1) {
    smooth_pre<T>(fine, S, S, z, zb, st, pf, EBIT_KC_FINE_SMOOTH);
    return hipGetLastError();
  }
  // descend
  smooth_pre<T>(fine, nu1, S, z, zb, st, pf, EBIT_KC_FINE_SMOOTH);
  const T* zpre = ((S - nu1) % 2 == 0) ? z : zb;
  {
    ProfScope ps(pf, EBIT_KC_FINE_RESTRICT, st);
    hipLaunchKernelGGL((k_fine_resid_restrict<T, double>), dim3(nblk(lv[1].d.N)), dim3(EBIT_BLOCK), 0, st, op, r,
                       zpre, lv[1].d, lvb<T>(lv[1]), lvx<T>(lv[1]));
  }
  // first level whose whole remaining hierarchy fits the tail kernel's LDS
  const int lt = tail_start<T>(lv, nlev, tail_cells, tail_lds);
  for (int l = 1; l < lt; ++l) {
    const CoarseRows<T> rows{coarse_op<T>(lv[l], sys), lvb<T>(lv[l])};
    const CoarseSweep<T> sw{rows, lv[l + 1].d, st};
    smooth_pre<T>(sw, nu1, S, lvx<T>(lv[l]), lvxb<T>(lv[l]), st, pf, EBIT_KC_COARSE);
    const T* xpre = ((S - nu1) % 2 == 0) ? lvx<T>(lv[l]) : lvxb<T>(lv[l]);
    ProfScope ps(pf, EBIT_KC_COARSE, st);
    hipLaunchKernelGGL(k_coarse_resid_restrict<T>, dim3(nblk(lv[l + 1].d.N)), dim3(EBIT_BLOCK), 0, st, rows.op,
                       (const T*)lvb<T>(lv[l]), xpre, lv[l + 1].d, lvb<T>(lv[l + 1]), lvx<T>(lv[l + 1]));
  }
  if (lt < nlev) {
    TailArgs<T> ta;
    ta.nl = nlev - lt;
    ta.nu1 = nu1;
    ta.nu2 = nu2;
    long long off = 0;
    for (int m = 0; m < ta.nl; ++m) {
      const EbitLevelHost& L = lv[lt + m];
      ta.L[m].d = L.d;
      ta.L[m].base = (int)off;
      const CoarseOp<T> c = coarse_op<T>(L, sys);
      ta.diag[m] = c.diag;
      for (int q = 0; q < 3; ++q) ta.off[m][q] = c.off[q];
      off += tail_level_elems(L.d);
    }
    ta.bg = lvb<T>(lv[lt]);
    ta.xg = lvx<T>(lv[lt]);
    ProfScope ps(pf, EBIT_KC_TAIL, st);
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(EBIT_TAIL_THREADS), (size_t)off * sizeof(T), st, ta);
  } else {
    CoarseOp<T> c = coarse_op<T>(lv[nlev - 1], sys);
    hipLaunchKernelGGL(k_coarsest<T>, dim3(1), dim3(64), 0, st, c, (const T*)lvb<T>(lv[nlev - 1]),
                       lvx<T>(lv[nlev - 1]), c.d.N == 1 ? 1 : 50);
  }
  // ascend: the first post-smoothing sweep of each level adds the correction
  for (int l = lt - 1; l >= 1; --l) {
    const CoarseSweep<T> sw{CoarseRows<T>{coarse_op<T>(lv[l], sys), lvb<T>(lv[l])}, lv[l + 1].d, st};
    smooth_post<T>(sw, nu1, S, lvx<T>(lv[l]), lvxb<T>(lv[l]), (const T*)lvx<T>(lv[l + 1]), st, pf, EBIT_KC_COARSE);
  }
  smooth_post<T>(fine, nu1, S, z, zb, (const T*)lvx<T>(lv[1]), st, pf, EBIT_KC_FINE_SMOOTH);
  return hipGetLastError();
}

extern "C" {

hipError_t ebit_launch_apply(const FineOp* op, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_apply, dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, *op, x, y);
  return hipGetLastError();
}

hipError_t ebit_launch_heat_rhs(const FineOp* op, const double* Ts, double* b, hipStream_t st) {
  hipLaunchKernelGGL(k_heat_rhs, dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, *op, Ts, b);
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
    if (hipFuncSetAttribute((const void*)ebit::k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)ebit::k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
            hipSuccess) {
      (void)hipGetLastError();
      return 64 * 1024;
    }
  }
  return v;
}

hipError_t ebit_launch_finalize_max(const double* partial, int nb, Scal* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partial, nb, 1, sc, (int)FIN_MAX, 0);
  return hipGetLastError();
}

}  // extern "C"

namespace ebit {

static hipError_t read_scal(Scal* d, Scal* h, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(h, d, sizeof(Scal), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

template <typename T>
static T* zbuf2(const EbitSolveBufs* B);
template <>
double* zbuf2<double>(const EbitSolveBufs* B) { return B->z64b; }
template <>
float* zbuf2<float>(const EbitSolveBufs* B) { return B->z32b; }
template <typename T>
static T* zbuf(const EbitSolveBufs* B);
template <>
double* zbuf<double>(const EbitSolveBufs* B) { return B->z64; }
template <>
float* zbuf<float>(const EbitSolveBufs* B) { return B->z32; }

template <typename T>
static int solve_t(const FineOp& op, const EbitLevelHost* lv, int nlev, const EbitSolveBufs* B, const double* b,
                   double* x, int use_guess, const ebit_opts* o, hipStream_t st, int* iters, int* vcyc,
                   double* relres, double* bnorm, double* floor, hipError_t* herr) {
  const long long N = op.d.N;
  const int RB = EBIT_RED_BLOCKS;
  Scal hs;
  T* z = zbuf<T>(B);
  *iters = 0;
  *vcyc = 0;
  *herr = hipSuccess;
#define CK(e)                 \
  do {                        \
    hipError_t _e = (e);      \
    if (_e != hipSuccess) {   \
      *herr = _e;             \
      return -1;              \
    }                         \
  } while (0)
  // reset device scalars (a fill kernel, so the sequence stays graph-capturable)
  hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st, (long long)(sizeof(Scal) / sizeof(double)),
                     (double*)B->scal, 0.0);
  if (!use_guess) hipLaunchKernelGGL(k_fill<double>, dim3(nblk(N)), dim3(EBIT_BLOCK), 0, st, N, x, 0.0);
  hipLaunchKernelGGL(k_resid_init, dim3(RB), dim3(EBIT_BLOCK), 0, st, op, b, use_guess ? (const double*)x : nullptr,
                     B->r, B->partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, (const double*)B->partial, RB, 3, B->scal,
                     (int)FIN_INIT, 1);
  CK(hipGetLastError());
  CK(read_scal(B->scal, &hs, st));
  if (hs.err & ERR_NAN) return 2;
  const double bb = hs.bb;
  *bnorm = sqrt(bb);
  if (bb == 0.0) {
    hipLaunchKernelGGL(k_fill<double>, dim3(nblk(N)), dim3(EBIT_BLOCK), 0, st, N, x, 0.0);
    *relres = 0.0;
    *floor = 0.0;
    CK(hipGetLastError());
    return 0;
  }
  const double tol2 = o->rtol * o->rtol * bb;
  // representability floor of the residual: eps || |b| + |A||x| ||
  const double fc = 2.220446049250313e-16;
  double floor2 = fc * fc * hs.aa;
  double rr = hs.rr;
  if (rr <= tol2) {
    *relres = sqrt(rr / bb);
    *floor = sqrt(floor2 / bb);
    return 0;
  }
  const int check = o->check_every > 0 ? o->check_every : 1;
  int it = 0;
  int restarts = 0;
  int first = 1;
  int pi = 0;
  bool conv = false;
  double last_true = rr;  // last recomputed residual (squared)
  int at_floor = 0;
  while (it < o->max_iters) {
    CK(vcycle<T>(op, lv, nlev, B->r, z, zbuf2<T>(B), o->nu1, o->nu2, o->tail_cells, B->tail_lds, st, B->prof));
    ++*vcyc;
    // defect correction = the same loop with beta = 0: x += alpha V(r) with the
    // energy-optimal step alpha = (r.z)/(z.Az), so it contracts for any SPD A
    const int fresh = (o->outer == EBIT_OUTER_DC) ? 1 : first;
    hipLaunchKernelGGL(k_dots_zr_zq<T>, dim3(RB), dim3(EBIT_BLOCK), 0, st, N, (const T*)z,
                       (const double*)B->r, fresh ? nullptr : (const double*)B->q, B->partial);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, (const double*)B->partial, RB, 2, B->scal,
                       (int)FIN_GAMMA, fresh);
    {
      ProfScope ps(B->prof, EBIT_KC_OUTER_APPLY, st);
      hipLaunchKernelGGL(k_p_update_apply<T>, dim3(RB), dim3(EBIT_BLOCK), 0, st, op, (const T*)z,
                         (const double*)B->p[pi], B->p[1 - pi], B->q, (const Scal*)B->scal, fresh, B->partial);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, (const double*)B->partial, RB, 1, B->scal,
                       (int)FIN_DELTA, 0);
    pi = 1 - pi;
    {
      ProfScope ps(B->prof, EBIT_KC_OUTER_UPDATE, st);
      hipLaunchKernelGGL(k_update_xr, dim3(RB), dim3(EBIT_BLOCK), 0, st, N, x, B->r, (const double*)B->p[pi],
                         (const double*)B->q, (const Scal*)B->scal, B->partial);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, (const double*)B->partial, RB, 1, B->scal,
                       (int)FIN_RR, 0);
    first = 0;
    CK(hipGetLastError());
    ++it;
    if (it % check == 0 || it == o->max_iters) {
      CK(read_scal(B->scal, &hs, st));
      if (hs.err & ERR_NAN) {
        *iters = it;
        return 2;
      }
      rr = hs.rr;
      if (rr <= tol2 || (restarts > 0 && rr <= 1e-12 * last_true)) {
        // recompute the true residual (the CG recurrence drifts from it)
        hipLaunchKernelGGL(k_resid_init, dim3(RB), dim3(EBIT_BLOCK), 0, st, op, b, (const double*)x, B->r,
                           B->partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, (const double*)B->partial, RB, 3, B->scal,
                           (int)FIN_INIT, 0);
        CK(hipGetLastError());
        CK(read_scal(B->scal, &hs, st));
        rr = hs.rr;
        floor2 = fc * fc * hs.aa;
        // At the representability floor the residual no longer tracks the
        // error, but the compensated residual still carries it: take two more
        // restart cycles there before stopping.
        const bool stagnant = restarts > 0 && rr > 0.25 * last_true;
        if (stagnant && rr <= floor2) ++at_floor;
        if (rr <= tol2 || at_floor >= 2) {
          conv = true;
          break;
        }
        if (restarts >= 8 || (stagnant && rr > floor2)) break;
        ++restarts;
        last_true = rr;
        first = 1;  // restart the recurrence from the recomputed residual
      }
    }
  }
  *floor = sqrt(floor2 / bb);
  *iters = it;
  *relres = sqrt(rr / bb);
  return conv ? 0 : 1;
#undef CK
}

}  // namespace ebit

extern "C" int ebit_solve_stream(const FineOp* op, const EbitLevelHost* lv, int nlev, const EbitSolveBufs* B,
                                 const double* b, double* x, int use_guess, const ebit_opts* o, hipStream_t st,
                                 int* iters, int* vcyc, double* relres, double* bnorm, double* floor,
                                 hipError_t* herr) {
  if (o->precision == EBIT_MIXED)
    return ebit::solve_t<float>(*op, lv, nlev, B, b, x, use_guess, o, st, iters, vcyc, relres, bnorm, floor, herr);
  return ebit::solve_t<double>(*op, lv, nlev, B, b, x, use_guess, o, st, iters, vcyc, relres, bnorm, floor, herr);
}
