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

template <typename T, typename TB>
__global__ void k_fine_smooth(FineOp op, const TB* __restrict__ b, T* __restrict__ x, int color) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!red_black_cell(op.d, t, color, i, j, k)) return;
  const long long c = cell_index(op.d, i, j, k);
  T diag, off[6], mass, rb = 0;
  fine_row<T>(op, i, j, k, op.flags[c], diag, off, mass, rb);
  T s = (T)b[c];
  for (int q = 0; q < 2 * op.d.dim; ++q) {
    if (off[q] == (T)0) continue;
    int ni, nj, nk;
    neighbour(op.d, i, j, k, q, ni, nj, nk);
    s -= off[q] * x[cell_index(op.d, ni, nj, nk)];
  }
  x[c] = s / diag;
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

template <typename T>
__global__ void k_prolong(Dims fd, Dims cd, T* __restrict__ x, const T* __restrict__ xc) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= fd.N) return;
  int i, j, k;
  cell_ijk(fd, c, i, j, k);
  x[c] += xc[cell_index(cd, i >> 1, j >> 1, k >> 1)];
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
__global__ void k_coarse_smooth(CoarseOp<T> op, const T* __restrict__ b, T* __restrict__ x, int color) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!red_black_cell(op.d, t, color, i, j, k)) return;
  const long long c = cell_index(op.d, i, j, k);
  x[c] = (b[c] - coarse_offsum<T>(op, i, j, k, c, x)) / op.diag[c];
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

// One V(nu1, nu2) cycle on A z = r with z = 0 initially; fine level matrix-free.
template <typename T>
static hipError_t vcycle(const FineOp& op, const EbitLevelHost* lv, int nlev, const double* r, T* z,
                         int nu1, int nu2, hipStream_t st, EbitProfiler* pf) {
  const Dims& fd = op.d;
  const int sys = op.sys;
  hipLaunchKernelGGL(k_fill<T>, dim3(nblk(fd.N)), dim3(EBIT_BLOCK), 0, st, fd.N, z, (T)0);
  if (nlev == 1) {
    // no coarse level: smoothing only
    for (int s = 0; s < nu1 + nu2; ++s)
      for (int col = 0; col < 2; ++col)
        hipLaunchKernelGGL((k_fine_smooth<T, double>), dim3(nblk(half_count(fd))), dim3(EBIT_BLOCK), 0, st, op,
                           r, z, col);
    return hipGetLastError();
  }
  // descend
  for (int s = 0; s < nu1; ++s)
    for (int col = 0; col < 2; ++col) {
      ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st);
      hipLaunchKernelGGL((k_fine_smooth<T, double>), dim3(nblk(half_count(fd))), dim3(EBIT_BLOCK), 0, st, op, r,
                         z, col);
    }
  {
    ProfScope ps(pf, EBIT_KC_FINE_RESTRICT, st);
    hipLaunchKernelGGL((k_fine_resid_restrict<T, double>), dim3(nblk(lv[1].d.N)), dim3(EBIT_BLOCK), 0, st, op, r,
                       (const T*)z, lv[1].d, lvb<T>(lv[1]), lvx<T>(lv[1]));
  }
  for (int l = 1; l < nlev - 1; ++l) {
    CoarseOp<T> c = coarse_op<T>(lv[l], sys);
    for (int s = 0; s < nu1; ++s)
      for (int col = 0; col < 2; ++col)
        hipLaunchKernelGGL(k_coarse_smooth<T>, dim3(nblk(half_count(c.d))), dim3(EBIT_BLOCK), 0, st, c,
                           (const T*)lvb<T>(lv[l]), lvx<T>(lv[l]), col);
    hipLaunchKernelGGL(k_coarse_resid_restrict<T>, dim3(nblk(lv[l + 1].d.N)), dim3(EBIT_BLOCK), 0, st, c,
                       (const T*)lvb<T>(lv[l]), (const T*)lvx<T>(lv[l]), lv[l + 1].d, lvb<T>(lv[l + 1]),
                       lvx<T>(lv[l + 1]));
  }
  {
    CoarseOp<T> c = coarse_op<T>(lv[nlev - 1], sys);
    hipLaunchKernelGGL(k_coarsest<T>, dim3(1), dim3(64), 0, st, c, (const T*)lvb<T>(lv[nlev - 1]),
                       lvx<T>(lv[nlev - 1]), c.d.N == 1 ? 1 : 50);
  }
  // ascend
  for (int l = nlev - 2; l >= 1; --l) {
    CoarseOp<T> c = coarse_op<T>(lv[l], sys);
    hipLaunchKernelGGL(k_prolong<T>, dim3(nblk(c.d.N)), dim3(EBIT_BLOCK), 0, st, c.d, lv[l + 1].d, lvx<T>(lv[l]),
                       (const T*)lvx<T>(lv[l + 1]));
    for (int s = 0; s < nu2; ++s)
      for (int col = 1; col >= 0; --col)
        hipLaunchKernelGGL(k_coarse_smooth<T>, dim3(nblk(half_count(c.d))), dim3(EBIT_BLOCK), 0, st, c,
                           (const T*)lvb<T>(lv[l]), lvx<T>(lv[l]), col);
  }
  {
    ProfScope ps(pf, EBIT_KC_FINE_PROLONG, st);
    hipLaunchKernelGGL(k_prolong<T>, dim3(nblk(fd.N)), dim3(EBIT_BLOCK), 0, st, fd, lv[1].d, z,
                       (const T*)lvx<T>(lv[1]));
  }
  for (int s = 0; s < nu2; ++s)
    for (int col = 1; col >= 0; --col) {
      ProfScope ps(pf, EBIT_KC_FINE_SMOOTH, st);
      hipLaunchKernelGGL((k_fine_smooth<T, double>), dim3(nblk(half_count(fd))), dim3(EBIT_BLOCK), 0, st, op, r,
                         z, col);
    }
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
    CK(vcycle<T>(op, lv, nlev, B->r, z, o->nu1, o->nu2, st, B->prof));
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
