/*
 * Plain FP64 geometric multigrid solve for the oracle's link-flux operators.
 *
 * TEST INFRASTRUCTURE ONLY: called from oracle/mg.py, which only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use.  It shares no
 * code with the HIP library.
 *
 * It solves A x = b for the symmetric positive definite systems the oracle
 * assembles for the implicit heat step (Eqs. energy_diffusion, Txx_ghost)
 * and for the variable-density Poisson problem (Eq. poisson_ghost_fluid) on
 * grids too large for a sparse direct factorisation.  The operator is given
 * in flux form on the grid (x fastest, c = i + nx (j + ny k)):
 *
 *   (A x)_c = m_c x_c + sum_a [ w_a(c) (x_c - x_{c+e_a}) + w_a(c-e_a) (x_c - x_{c-e_a}) ]
 *
 * with w_a(c) the weight of the link from c to its +a neighbour (wrapping on
 * a periodic axis; 0 where no link exists).
 *
 * Method (textbook, nothing fused or reordered for speed):
 *   - coarse grids by 2^d aggregation (ceil(n/2) cells per axis), and the
 *     Galerkin coarse operator P^T A P for the piecewise-constant
 *     prolongation P: the coarse mass is the sum of the children's masses,
 *     a coarse link weight is the sum of the fine link weights that cross
 *     between the two aggregates, and fine links inside an aggregate drop;
 *   - restriction P^T (sum over the children), prolongation P (each child
 *     takes its aggregate's value);
 *   - red-black Gauss-Seidel smoothing, red (i+j+k even) then black before
 *     the coarse correction and black then red after it, so the cycle is a
 *     symmetric preconditioner; within one colour every new value is formed
 *     from the current iterate before any is stored, which is exact
 *     Gauss-Seidel for a proper two-colouring and stays a valid symmetric
 *     smoother on a periodic axis of odd length;
 *   - the coarsest grid (at most DENSE_MAX cells) is solved exactly by a
 *     dense Cholesky factorisation;
 *   - preconditioned conjugate gradients with one cycle (gamma = 1: V,
 *     gamma = 2: W) as the preconditioner;
 *   - iterative refinement around it: the residual b - A x is formed in
 *     long double in the flux form above, the correction is solved in
 *     double, and x is accumulated in long double, until the correction no
 *     longer changes x.
 * Every reduction runs over fixed blocks of cells, summed in block order, so
 * the result does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAX_LEVELS 32
#define DENSE_MAX 512
#define RED_BLOCK 4096

typedef struct {
  int n[3];
  int per[3];
  long N;
  double* m;      /* mass (diagonal excess) per cell          */
  double* w[3];   /* link weight to the +a neighbour per cell */
  double* dg;     /* diagonal of A                            */
  double* x;      /* iterate                                  */
  double* b;      /* right-hand side                          */
  double* r;      /* residual                                 */
  double* t;      /* new values of one colour                 */
  double* e;      /* second W-cycle pass                      */
} level_t;

typedef struct {
  int nlev;
  int dim;
  int nu;
  int gamma;
  level_t L[MAX_LEVELS];
  double* chol;   /* dense Cholesky factor of the coarsest level (row major, lower) */
  double* part;   /* block partial sums */
} mg_t;

static inline long cidx(const level_t* L, long i, long j, long k) {
  return i + (long)L->n[0] * (j + (long)L->n[1] * k);
}

/* neighbour of c along axis a, direction s = +1/-1; -1 when off a wall */
static inline long nbr(const level_t* L, long i, long j, long k, int a, int s) {
  long q[3] = {i, j, k};
  q[a] += s;
  if (q[a] < 0 || q[a] >= L->n[a]) {
    if (!L->per[a] || L->n[a] == 1) return -1;
    q[a] = (q[a] + L->n[a]) % L->n[a];
  }
  return cidx(L, q[0], q[1], q[2]);
}

/* weight of the link on side (a, s) of cell (i, j, k) */
static inline double side_w(const level_t* L, long i, long j, long k, int a, int s) {
  if (s > 0) {
    if (nbr(L, i, j, k, a, +1) < 0) return 0.0;
    return L->w[a][cidx(L, i, j, k)];
  }
  long q = nbr(L, i, j, k, a, -1);
  if (q < 0) return 0.0;
  return L->w[a][q];
}

static void* xalloc(size_t bytes) {
  void* p = calloc(bytes ? bytes : 1, 1);
  return p;
}

static void level_free(level_t* L) {
  free(L->m);
  for (int a = 0; a < 3; ++a) free(L->w[a]);
  free(L->dg);
  free(L->x);
  free(L->b);
  free(L->r);
  free(L->t);
  free(L->e);
  memset(L, 0, sizeof(*L));
}

static int level_alloc(level_t* L) {
  size_t s = (size_t)L->N * sizeof(double);
  L->m = xalloc(s);
  for (int a = 0; a < 3; ++a) L->w[a] = xalloc(s);
  L->dg = xalloc(s);
  L->x = xalloc(s);
  L->b = xalloc(s);
  L->r = xalloc(s);
  L->t = xalloc(s);
  L->e = xalloc(s);
  if (!L->m || !L->w[0] || !L->w[1] || !L->w[2] || !L->dg || !L->x || !L->b || !L->r || !L->t || !L->e)
    return -1;
  return 0;
}

static void compute_diag(level_t* L) {
  long nx = L->n[0], ny = L->n[1], nz = L->n[2];
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        long c = cidx(L, i, j, k);
        double d = L->m[c];
        for (int a = 0; a < 3; ++a) d += side_w(L, i, j, k, a, +1) + side_w(L, i, j, k, a, -1);
        L->dg[c] = d;
      }
}

/* Galerkin coarse operator for the piecewise-constant prolongation */
static void coarsen(const level_t* F, level_t* C) {
  long nx = F->n[0], ny = F->n[1], nz = F->n[2];
  /* serial: several children add into one coarse entry */
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        long f = cidx(F, i, j, k);
        long I[3] = {i / 2, j / 2, k / 2};
        if (F->n[0] == 1) I[0] = 0;
        if (F->n[1] == 1) I[1] = 0;
        if (F->n[2] == 1) I[2] = 0;
        long cc = cidx(C, I[0], I[1], I[2]);
        C->m[cc] += F->m[f];
        long fi[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
          long q = nbr(F, i, j, k, a, +1);
          if (q < 0) continue;
          long nb[3] = {fi[0], fi[1], fi[2]};
          nb[a] = (nb[a] + 1) % F->n[a];
          long J = (F->n[a] == 1) ? 0 : nb[a] / 2;
          if (J == I[a]) continue; /* link inside the aggregate */
          C->w[a][cc] += F->w[a][f];
        }
      }
}

/* y = A x */
static void apply(const level_t* L, const double* x, double* y) {
  long nx = L->n[0], ny = L->n[1], nz = L->n[2];
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        long c = cidx(L, i, j, k);
        double s = L->m[c] * x[c];
        for (int a = 0; a < 3; ++a)
          for (int sg = -1; sg <= 1; sg += 2) {
            long q = nbr(L, i, j, k, a, sg);
            if (q < 0) continue;
            double wl = sg > 0 ? L->w[a][c] : L->w[a][q];
            s += wl * (x[c] - x[q]);
          }
        y[c] = s;
      }
}

static void residual(const level_t* L, const double* x, const double* b, double* r) {
  apply(L, x, r);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < L->N; ++c) r[c] = b[c] - r[c];
}

/* one colour of Gauss-Seidel: new values of that colour from the current x */
static void smooth_colour(level_t* L, double* x, const double* b, int colour) {
  long nx = L->n[0], ny = L->n[1], nz = L->n[2];
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        if (((i + j + k) & 1) != colour) continue;
        long c = cidx(L, i, j, k);
        double s = b[c];
        for (int a = 0; a < 3; ++a)
          for (int sg = -1; sg <= 1; sg += 2) {
            long q = nbr(L, i, j, k, a, sg);
            if (q < 0) continue;
            double wl = sg > 0 ? L->w[a][c] : L->w[a][q];
            s += wl * x[q];
          }
        L->t[c] = s / L->dg[c];
      }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        if (((i + j + k) & 1) != colour) continue;
        long c = cidx(L, i, j, k);
        x[c] = L->t[c];
      }
}

static void restrict_sum(const level_t* F, const double* r, level_t* C, double* bc) {
  memset(bc, 0, (size_t)C->N * sizeof(double));
  long nx = F->n[0], ny = F->n[1], nz = F->n[2];
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        long I = F->n[0] == 1 ? 0 : i / 2, J = F->n[1] == 1 ? 0 : j / 2, K = F->n[2] == 1 ? 0 : k / 2;
        bc[cidx(C, I, J, K)] += r[cidx(F, i, j, k)];
      }
}

static void prolong_add(const level_t* F, double* x, const level_t* C, const double* ec) {
  long nx = F->n[0], ny = F->n[1], nz = F->n[2];
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
      for (long i = 0; i < nx; ++i) {
        long I = F->n[0] == 1 ? 0 : i / 2, J = F->n[1] == 1 ? 0 : j / 2, K = F->n[2] == 1 ? 0 : k / 2;
        x[cidx(F, i, j, k)] += ec[cidx(C, I, J, K)];
      }
}

/* dense Cholesky of the coarsest level; -1 if it is not positive definite */
static int dense_setup(mg_t* g) {
  level_t* L = &g->L[g->nlev - 1];
  long N = L->N;
  double* A = xalloc((size_t)N * N * sizeof(double));
  if (!A) return -2;
  double* e = xalloc((size_t)N * sizeof(double));
  double* y = xalloc((size_t)N * sizeof(double));
  for (long c = 0; c < N; ++c) {
    memset(e, 0, (size_t)N * sizeof(double));
    e[c] = 1.0;
    apply(L, e, y);
    for (long r = 0; r < N; ++r) A[r * N + c] = y[r];
  }
  free(e);
  free(y);
  for (long j = 0; j < N; ++j) {
    double d = A[j * N + j];
    for (long k = 0; k < j; ++k) d -= A[j * N + k] * A[j * N + k];
    if (!(d > 0.0)) {
      free(A);
      return -1;
    }
    d = sqrt(d);
    A[j * N + j] = d;
    for (long i = j + 1; i < N; ++i) {
      double s = A[i * N + j];
      for (long k = 0; k < j; ++k) s -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = s / d;
    }
  }
  g->chol = A;
  return 0;
}

static void dense_solve(const mg_t* g, const double* b, double* x) {
  const level_t* L = &g->L[g->nlev - 1];
  long N = L->N;
  const double* A = g->chol;
  for (long i = 0; i < N; ++i) {
    double s = b[i];
    for (long k = 0; k < i; ++k) s -= A[i * N + k] * x[k];
    x[i] = s / A[i * N + i];
  }
  for (long i = N - 1; i >= 0; --i) {
    double s = x[i];
    for (long k = i + 1; k < N; ++k) s -= A[k * N + i] * x[k];
    x[i] = s / A[i * N + i];
  }
}

/* x = B b for level l (zero start): one V (gamma 1) or W (gamma 2) cycle */
static void cycle(mg_t* g, int l, const double* b, double* x) {
  level_t* L = &g->L[l];
  if (l == g->nlev - 1) {
    dense_solve(g, b, x);
    return;
  }
  level_t* C = &g->L[l + 1];
  memset(x, 0, (size_t)L->N * sizeof(double));
  for (int s = 0; s < g->nu; ++s) {
    smooth_colour(L, x, b, 0);
    smooth_colour(L, x, b, 1);
  }
  residual(L, x, b, L->r);
  restrict_sum(L, L->r, C, C->b);
  cycle(g, l + 1, C->b, C->x);
  if (g->gamma > 1 && l + 1 < g->nlev - 1) {
    /* second pass: e = x_c + B (b_c - A_c x_c) */
    residual(C, C->x, C->b, C->r);
    double* rc = xalloc((size_t)C->N * sizeof(double));
    memcpy(rc, C->r, (size_t)C->N * sizeof(double));
    cycle(g, l + 1, rc, C->e);
    for (long c = 0; c < C->N; ++c) C->x[c] += C->e[c];
    free(rc);
  }
  prolong_add(L, x, C, C->x);
  for (int s = 0; s < g->nu; ++s) {
    smooth_colour(L, x, b, 1);
    smooth_colour(L, x, b, 0);
  }
}

static double dot(mg_t* g, long N, const double* a, const double* b) {
  long nb = (N + RED_BLOCK - 1) / RED_BLOCK;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nb; ++k) {
    long lo = k * RED_BLOCK, hi = lo + RED_BLOCK < N ? lo + RED_BLOCK : N;
    double s = 0.0;
    for (long c = lo; c < hi; ++c) s += a[c] * b[c];
    g->part[k] = s;
  }
  double s = 0.0;
  for (long k = 0; k < nb; ++k) s += g->part[k];
  return s;
}

/* preconditioned CG on the finest level: solves A d = r to rtol; returns iterations */
static int pcg(mg_t* g, const double* r0, double* d, double rtol, int maxit, double* relres) {
  level_t* L = &g->L[0];
  long N = L->N;
  double* r = xalloc((size_t)N * sizeof(double));
  double* z = xalloc((size_t)N * sizeof(double));
  double* p = xalloc((size_t)N * sizeof(double));
  double* q = xalloc((size_t)N * sizeof(double));
  memcpy(r, r0, (size_t)N * sizeof(double));
  memset(d, 0, (size_t)N * sizeof(double));
  double bn = sqrt(dot(g, N, r, r));
  int it = 0;
  *relres = 0.0;
  if (bn > 0.0) {
    cycle(g, 0, r, z);
    memcpy(p, z, (size_t)N * sizeof(double));
    double rz = dot(g, N, r, z);
    for (it = 1; it <= maxit; ++it) {
      apply(L, p, q);
      double alpha = rz / dot(g, N, p, q);
#pragma omp parallel for schedule(static)
      for (long c = 0; c < N; ++c) {
        d[c] += alpha * p[c];
        r[c] -= alpha * q[c];
      }
      double rn = sqrt(dot(g, N, r, r));
      *relres = rn / bn;
      if (!(rn > rtol * bn)) break;
      cycle(g, 0, r, z);
      double rz1 = dot(g, N, r, z);
      double beta = rz1 / rz;
      rz = rz1;
#pragma omp parallel for schedule(static)
      for (long c = 0; c < N; ++c) p[c] = z[c] + beta * p[c];
    }
  }
  free(r);
  free(z);
  free(p);
  free(q);
  return it;
}

static void mg_free(mg_t* g) {
  for (int l = 0; l < g->nlev; ++l) level_free(&g->L[l]);
  free(g->chol);
  free(g->part);
  free(g);
}

/*
 * Solve A x = b.  n[3]: cells per axis (n[2] = 1 in 2D), per[3]: periodic
 * axes, m: mass per cell, w[a]: +a link weights (NULL for a >= dim), b: the
 * right-hand side; x receives the solution.  nu: smoothing sweeps before and
 * after the coarse correction, gamma: 1 for V-, 2 for W-cycles, nthreads:
 * OpenMP threads (0 = the runtime default).  info (8 doubles) receives:
 * [0] relative residual ||b - A x|| / ||b|| of the returned (double) x,
 * evaluated in long double in the flux form, [1] refinement rounds,
 * [2] total PCG iterations, [3] levels, [4] first-round PCG iterations,
 * [5] last correction size max|d|/max|x|, [6] the residual of the
 * long-double iterate before rounding.
 * Returns 0, -1 if the coarsest level is not positive definite, -2 if out of
 * memory, -3 if the refinement stalled above the target, -4 on bad sizes.
 */
int oracle_mg_solve(int dim, const int* n, const int* per, const double* m, const double* const* w,
                    const double* b, double* x, double rtol, int max_rounds, double inner_rtol,
                    int max_iters, int nu, int gamma, int nthreads, double* info) {
#ifdef _OPENMP
  int saved = omp_get_max_threads();
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int rc = 0;
  for (int i = 0; i < 8; ++i) info[i] = 0.0;
  if (dim < 2 || dim > 3 || n[0] < 1 || n[1] < 1 || n[2] < 1) return -4;
  mg_t* g = xalloc(sizeof(mg_t));
  if (!g) return -2;
  g->dim = dim;
  g->nu = nu;
  g->gamma = gamma;
  /* level 0 */
  level_t* F = &g->L[0];
  for (int a = 0; a < 3; ++a) {
    F->n[a] = a < dim ? n[a] : 1;
    F->per[a] = a < dim ? per[a] : 0;
  }
  F->N = (long)F->n[0] * F->n[1] * F->n[2];
  if (level_alloc(F)) {
    mg_free(g);
    return -2;
  }
  memcpy(F->m, m, (size_t)F->N * sizeof(double));
  for (int a = 0; a < dim; ++a) memcpy(F->w[a], w[a], (size_t)F->N * sizeof(double));
  compute_diag(F);
  g->nlev = 1;
  while (g->L[g->nlev - 1].N > DENSE_MAX && g->nlev < MAX_LEVELS) {
    level_t* P = &g->L[g->nlev - 1];
    level_t* C = &g->L[g->nlev];
    for (int a = 0; a < 3; ++a) {
      C->n[a] = (P->n[a] + 1) / 2;
      C->per[a] = P->per[a];
    }
    C->N = (long)C->n[0] * C->n[1] * C->n[2];
    if (level_alloc(C)) {
      mg_free(g);
      return -2;
    }
    coarsen(P, C);
    compute_diag(C);
    g->nlev++;
  }
  long N = F->N;
  g->part = xalloc((size_t)((N + RED_BLOCK - 1) / RED_BLOCK + 1) * sizeof(double));
  rc = dense_setup(g);
  if (rc) {
    mg_free(g);
    return rc;
  }
  info[3] = g->nlev;
  /* iterative refinement: x in long double, residual in long double */
  long double* xl = xalloc((size_t)N * sizeof(long double));
  double* r = xalloc((size_t)N * sizeof(double));
  double* d = xalloc((size_t)N * sizeof(double));
  long double* pl = xalloc((size_t)((N + RED_BLOCK - 1) / RED_BLOCK + 1) * sizeof(long double));
  if (!xl || !r || !d || !pl) {
    free(xl);
    free(r);
    free(d);
    free(pl);
    mg_free(g);
    return -2;
  }
  long nbk = (N + RED_BLOCK - 1) / RED_BLOCK;
  long double bn2 = 0.0L;
  for (long c = 0; c < N; ++c) bn2 += (long double)b[c] * b[c];
  double bnorm = sqrtl(bn2);
  int total = 0;
  double relres = 0.0;
  for (int round = 0; round <= max_rounds; ++round) {
    /* r = b - A x in long double, flux form */
    long nx = F->n[0], ny = F->n[1];
#pragma omp parallel for schedule(static)
    for (long kb = 0; kb < nbk; ++kb) {
      long lo = kb * RED_BLOCK, hi = lo + RED_BLOCK < N ? lo + RED_BLOCK : N;
      long double acc = 0.0L;
      for (long c = lo; c < hi; ++c) {
        long i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        long double s = (long double)F->m[c] * xl[c];
        for (int a = 0; a < 3; ++a)
          for (int sg = -1; sg <= 1; sg += 2) {
            long q = nbr(F, i, j, k, a, sg);
            if (q < 0) continue;
            double wl = sg > 0 ? F->w[a][c] : F->w[a][q];
            s += (long double)wl * (xl[c] - xl[q]);
          }
        long double rr = (long double)b[c] - s;
        r[c] = (double)rr;
        acc += rr * rr;
      }
      pl[kb] = acc;
    }
    long double rn2 = 0.0L;
    for (long kb = 0; kb < nbk; ++kb) rn2 += pl[kb];
    relres = bnorm > 0 ? (double)(sqrtl(rn2) / bnorm) : (double)sqrtl(rn2);
    info[0] = relres;
    info[1] = round;
    if (bnorm == 0.0 || relres <= rtol || round == max_rounds) break;
    double rr_in;
    int it = pcg(g, r, d, inner_rtol, max_iters, &rr_in);
    if (round == 0) info[4] = it;
    total += it;
    double dmax = 0.0, xmax = 0.0;
    for (long c = 0; c < N; ++c) {
      xl[c] += (long double)d[c];
      if (fabs(d[c]) > dmax) dmax = fabs(d[c]);
      if (fabsl(xl[c]) > xmax) xmax = (double)fabsl(xl[c]);
    }
    info[5] = xmax > 0 ? dmax / xmax : 0.0;
    /* the correction no longer changes x in double */
    if (round > 0 && dmax <= 1e-17 * xmax) {
      /* recompute the residual of the final x before leaving */
      max_rounds = round + 1;
    }
  }
  info[2] = total;
  info[6] = relres;
  if (bnorm > 0 && relres > rtol && info[5] > 1e-15) rc = -3;
  /* the returned x is xl rounded to double: report the residual of that x */
  for (long c = 0; c < N; ++c) {
    x[c] = (double)xl[c];
    xl[c] = (long double)x[c];
  }
  {
    long nx = F->n[0], ny = F->n[1];
#pragma omp parallel for schedule(static)
    for (long kb = 0; kb < nbk; ++kb) {
      long lo = kb * RED_BLOCK, hi = lo + RED_BLOCK < N ? lo + RED_BLOCK : N;
      long double acc = 0.0L;
      for (long c = lo; c < hi; ++c) {
        long i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        long double s = (long double)F->m[c] * xl[c];
        for (int a = 0; a < 3; ++a)
          for (int sg = -1; sg <= 1; sg += 2) {
            long q = nbr(F, i, j, k, a, sg);
            if (q < 0) continue;
            double wl = sg > 0 ? F->w[a][c] : F->w[a][q];
            s += (long double)wl * (xl[c] - xl[q]);
          }
        long double rr = (long double)b[c] - s;
        acc += rr * rr;
      }
      pl[kb] = acc;
    }
    long double rn2 = 0.0L;
    for (long kb = 0; kb < nbk; ++kb) rn2 += pl[kb];
    info[0] = bnorm > 0 ? (double)(sqrtl(rn2) / bnorm) : (double)sqrtl(rn2);
  }
  free(xl);
  free(r);
  free(d);
  free(pl);
  mg_free(g);
#ifdef _OPENMP
  omp_set_num_threads(saved);
#endif
  return rc;
}
