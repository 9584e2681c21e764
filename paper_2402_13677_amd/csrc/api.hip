// C ABI of the EBIT elliptic-path library: context, workspace carving,
// argument checks and the entry points declared in include/ebit.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ebit_internal.h"
#include "ghost.h"

using namespace ebit;

struct ebit_ctx {
  char solve_log[512];  // EBIT_SOLVE_LOG at creation ("" = no log)
  ebit_grid grid;
  ebit_props props;
  ebit_opts opts;
  hipStream_t st;
  char* ws;
  size_t ws_bytes;
  Dims fd;
  int nlev;
  EbitLevelHost lv[EBIT_MAX_LEVELS];
  uint8_t* flags;
  double* th[3];
  double* cF;
  double* nF;
  double* bvec;
  EbitSolveBufs B;
  double dt;
  int built;
  FineOp op[2];
  hipEvent_t ev0, ev1;
  EbitProfiler* prof;
  EbitPlan* plan;      // solve plan of this one case
  char* plan_mem;
  size_t plan_bytes;
  char* build_tabs;    // device tables of the hierarchy build
  void* adv;           // 2D: marker-motion scratch (edge coordinates and lists)
  int* adv_err;        // 2D: marker-motion error bits
  int adv_ready;       // its coordinate arrays have been set to NaN
  int build_ls;        // first level built by one work-group
  hipError_t herr;
  char msg[512];
};

// A batch of contexts whose solves share one plan: every kernel of a solve
// is one launch over all cases.
// A device table of a batched per-case launch and its host image: the table
// is uploaded only when its content changed since the last upload.
struct Tab {
  char* dev;
  char* host;
  size_t cap, len;
  int valid;
};

// The tables of one batch (carved after the plan's part of the batch
// workspace).  Block offsets depend on the grids only and are uploaded at
// creation; argument tables follow the callers' pointers.
struct BatchTabs {
  Tab geo, fine, small, split, heat, flux, proj, projfu, fin, scal0, scalg;
  Tab coarse[EBIT_MAX_LEVELS];
  int* geo_start[5];
  int* cell_start;
  int* red_start;
  int* fine_start;
  int* coarse_start[EBIT_MAX_LEVELS];
  int* small_start;
  int* unit_start;
  int* split_start;
  int geo_blocks[5], cell_blocks, red_blocks, fine_blocks, split_blocks;
  int fine_n;
  int coarse_n[EBIT_MAX_LEVELS], coarse_blocks[EBIT_MAX_LEVELS];
  int ncoarse;
  Scal* gather;  // the cases' status scalars side by side
};

struct ebit_batch {
  int n;
  ebit_ctx** ctx;
  ebit_opts opts;
  hipStream_t st;
  EbitPlan* plan;
  void* ws;
  size_t ws_bytes;
  hipEvent_t ev0, ev1;
  Scal* hsc;  // host copies of the contexts' status scalars
  BatchTabs t;
  hipError_t herr;
  char msg[512];
};

namespace {

const size_t ALIGN = 256;

struct Carver {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool valid_grid(const ebit_grid* g, char* msg, size_t ml) {
  if (!g) {
    snprintf(msg, ml, "grid is NULL");
    return false;
  }
  if (g->dim != 2 && g->dim != 3) {
    snprintf(msg, ml, "dim must be 2 or 3");
    return false;
  }
  for (int a = 0; a < 3; ++a) {
    if (a < g->dim && g->n[a] < 3) {
      snprintf(msg, ml, "n[%d] must be >= 3", a);
      return false;
    }
    if (a >= g->dim && g->n[a] != 1) {
      snprintf(msg, ml, "n[2] must be 1 in 2D");
      return false;
    }
    if (g->n[a] > (1 << 20)) {
      snprintf(msg, ml, "n[%d] too large", a);
      return false;
    }
  }
  const long long N = (long long)g->n[0] * g->n[1] * g->n[2];
  if (N >= (1LL << 31)) {
    snprintf(msg, ml, "grid has too many cells");
    return false;
  }
  if (!(g->h > 0) || !isfinite(g->h)) {
    snprintf(msg, ml, "h must be positive");
    return false;
  }
  for (int s = 0; s < 2 * g->dim; ++s) {
    for (int w = 0; w < 2; ++w) {
      const int b = w ? g->p_bc[s] : g->T_bc[s];
      if (b < 0 || b > 2) {
        snprintf(msg, ml, "bad boundary kind on side %d", s);
        return false;
      }
    }
    if (!isfinite(g->T_val[s]) || !isfinite(g->p_val[s])) {
      snprintf(msg, ml, "boundary value on side %d not finite", s);
      return false;
    }
  }
  for (int a = 0; a < g->dim; ++a) {
    const int kinds[4] = {g->T_bc[2 * a], g->T_bc[2 * a + 1], g->p_bc[2 * a], g->p_bc[2 * a + 1]};
    int nper = 0;
    for (int q = 0; q < 4; ++q) nper += kinds[q] == EBIT_BC_PERIODIC;
    if (nper != 0 && nper != 4) {
      snprintf(msg, ml, "axis %d: periodic must be set on both sides for T and p", a);
      return false;
    }
    if (nper == 4 && !is_pow2(g->n[a])) {
      snprintf(msg, ml, "axis %d: a periodic axis needs a power-of-two size", a);
      return false;
    }
  }
  // The pressure operator has no mass term: with no outflow (Dirichlet) side
  // it is singular (constants are its null space), and phase change in a
  // closed domain has no compatible right-hand side.  Such a grid is refused.
  bool p_dirichlet = false;
  for (int s = 0; s < 2 * g->dim; ++s) p_dirichlet = p_dirichlet || g->p_bc[s] == EBIT_BC_DIRICHLET;
  if (!p_dirichlet) {
    snprintf(msg, ml, "the pressure needs at least one outflow (Dirichlet) side");
    return false;
  }
  return true;
}

bool valid_props(const ebit_props* p, char* msg, size_t ml) {
  if (!p) {
    snprintf(msg, ml, "props is NULL");
    return false;
  }
  const double v[7] = {p->rho_l, p->rho_v, p->lam_l, p->lam_v, p->cp_l, p->cp_v, p->h_lg};
  for (int q = 0; q < 7; ++q)
    if (!(v[q] > 0) || !isfinite(v[q])) {
      snprintf(msg, ml, "properties must be positive and finite");
      return false;
    }
  if (!isfinite(p->T_sat)) {
    snprintf(msg, ml, "T_sat not finite");
    return false;
  }
  return true;
}

bool valid_opts(const ebit_opts* o, char* msg, size_t ml) {
  if (!o) return true;
  if (o->precision != EBIT_FP64 && o->precision != EBIT_MIXED) {
    snprintf(msg, ml, "bad precision");
    return false;
  }
  if (o->outer != EBIT_OUTER_PCG && o->outer != EBIT_OUTER_DC) {
    snprintf(msg, ml, "bad outer loop");
    return false;
  }
  if (!(o->rtol > 0) || o->max_iters < 1 || o->nu1 < 1 || o->nu2 < 1 || o->nu1 > 8 || o->nu2 > 8 ||
      !(o->theta_min > 0 && o->theta_min <= 0.5)) {
    snprintf(msg, ml, "bad solver options");
    return false;
  }
  return true;
}

Dims dims_of(const ebit_grid* g) {
  Dims d;
  d.dim = g->dim;
  long long N = 1;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = g->n[a];
    d.per[a] = (a < g->dim) && g->T_bc[2 * a] == EBIT_BC_PERIODIC;
    N *= g->n[a];
  }
  d.N = N;
  return d;
}

long long faces(const Dims& d, int a) {
  long long f = 1;
  for (int b = 0; b < 3; ++b) f *= d.n[b] + (b == a ? 1 : 0);
  return f;
}

// Carve the workspace; base == nullptr only measures.  Fills ctx pointers
// when ctx != nullptr.
size_t layout(const ebit_grid* g, const ebit_opts* o, char* base, ebit_ctx* ctx) {
  Carver cv{base, 0};
  const Dims fd = dims_of(g);
  const long long N = fd.N;
  uint8_t* flags = cv.take<uint8_t>(N);
  double* th[3] = {nullptr, nullptr, nullptr};
  for (int a = 0; a < fd.dim; ++a) th[a] = cv.take<double>(faces(fd, a));
  double* cF = cv.take<double>(3 * N);
  double* nF = cv.take<double>(3 * N);
  double* bvec = cv.take<double>(N);
  EbitSolveBufs B;
  // 3D: the fine smoother's iterate, right-hand side and flags are kept in
  // the colour-split order, 2 H entries (N, plus one row per (j, k) when n0
  // is odd)
  const long long NS = fd.dim == 3 ? 2 * split_half(fd) : N;
  B.r = cv.take<double>(N);
  B.r32 = cv.take<float>(NS);
  B.r64s = cv.take<double>(fd.dim == 3 ? NS : 0);
  B.fsplit = cv.take<uint8_t>(fd.dim == 3 ? NS : 0);
  B.z64 = cv.take<double>(NS);
  B.z64b = cv.take<double>(N);
  B.z32 = cv.take<float>(NS);
  B.z32b = cv.take<float>(N);
  B.p[0] = cv.take<double>(N);
  B.p[1] = cv.take<double>(N);
  B.q = cv.take<double>(N);
  B.partial = cv.take<double>(4 * EBIT_RED_BLOCKS);
  B.scal = cv.take<Scal>(1);
  // levels
  EbitLevelHost lv[EBIT_MAX_LEVELS];
  memset(lv, 0, sizeof(lv));
  lv[0].d = fd;
  int nlev = 1;
  while (lv[nlev - 1].d.N > 1 && nlev < EBIT_MAX_LEVELS) {
    Dims c = lv[nlev - 1].d;
    long long NN = 1;
    for (int a = 0; a < 3; ++a) {
      c.n[a] = (c.n[a] + 1) / 2;
      NN *= c.n[a];
    }
    c.N = NN;
    lv[nlev].d = c;
    ++nlev;
  }
  for (int l = 1; l < nlev; ++l) {
    const long long n = lv[l].d.N;
    for (int s = 0; s < 2; ++s) {
      lv[l].diag64[s] = cv.take<double>(n);
      lv[l].mass64[s] = cv.take<double>(n);
      for (int a = 0; a < fd.dim; ++a) lv[l].off64[s][a] = cv.take<double>(n);
      lv[l].diag32[s] = cv.take<float>(n);
      for (int a = 0; a < fd.dim; ++a) lv[l].off32[s][a] = cv.take<float>(n);
    }
    // b holds, on the tail's top level, the colour-split order the tail
    // copies straight into LDS (2 hs >= n elements)
    const long long nb = 2 * ebit::tail_half(lv[l].d);
    lv[l].x64 = cv.take<double>(n);
    lv[l].x64b = cv.take<double>(n);
    lv[l].b64 = cv.take<double>(nb > n ? nb : n);
    lv[l].x32 = cv.take<float>(n);
    lv[l].x32b = cv.take<float>(n);
    lv[l].b32 = cv.take<float>(nb > n ? nb : n);
  }
  // tail images, per system in FP32 and FP64: the coefficient blocks of the
  // levels of at most EBIT_TAIL_IMG_CELLS cells, then the inverse of the
  // first level of at most EBIT_DENSE_MAX cells
  int img0 = nlev, dl = -1;
  for (int l = nlev - 1; l >= 1 && lv[l].d.N <= EBIT_TAIL_IMG_CELLS; --l) img0 = l;
  for (int l = 1; l < nlev && dl < 0; ++l)
    if (lv[l].d.N <= EBIT_DENSE_MAX) dl = l;
  if (img0 < nlev) {
    long long tot = 0;
    for (int l = img0; l < nlev; ++l) tot += ebit::tail_img_elems(lv[l].d);
    const long long ninv = dl >= 0 ? ebit::tail_pad(lv[dl].d.N * lv[dl].d.N) : 0;
    for (int s = 0; s < 2; ++s) {
      float* i32 = cv.take<float>(tot + ninv);
      double* i64 = cv.take<double>(tot + ninv);
      long long off = 0;
      for (int l = img0; l < nlev; ++l) {
        lv[l].img32[s] = i32 ? i32 + off : nullptr;
        lv[l].img64[s] = i64 ? i64 + off : nullptr;
        off += ebit::tail_img_elems(lv[l].d);
      }
      if (dl >= 0) {
        lv[dl].inv32[s] = i32 ? i32 + off : nullptr;
        lv[dl].inv64[s] = i64 ? i64 + off : nullptr;
      }
    }
    if (dl >= 0) lv[dl].inv_ok = cv.take<int>(2);
  }
  // room for a plan of either precision (a mixed solve can fall back to FP64)
  const size_t plan_bytes = std::max(ebit_plan_device_bytes(1, EBIT_FP64), ebit_plan_device_bytes(1, EBIT_MIXED));
  char* plan_mem = cv.take<char>(plan_bytes);
  char* build_tabs = cv.take<char>(ebit_build_table_bytes());
  // 2D marker motion: moved and fixed coordinates of every edge of both
  // families, two marker lists, and the error word
  char* adv = cv.take<char>(fd.dim == 2 ? ebit_advect_scratch_bytes(&fd) : 0);
  int* adv_err = cv.take<int>(fd.dim == 2 ? 4 : 0);
  const size_t total = (cv.off + ALIGN - 1) / ALIGN * ALIGN;
  if (ctx) {
    ctx->plan_mem = plan_mem;
    ctx->plan_bytes = plan_bytes;
    ctx->build_tabs = build_tabs;
    ctx->adv = adv;
    ctx->adv_err = adv_err;
    ctx->adv_ready = 0;
    ctx->fd = fd;
    ctx->flags = flags;
    for (int a = 0; a < 3; ++a) ctx->th[a] = th[a];
    ctx->cF = cF;
    ctx->nF = nF;
    ctx->bvec = bvec;
    ctx->B = B;
    ctx->nlev = nlev;
    memcpy(ctx->lv, lv, sizeof(lv));
  }
  (void)o;
  return total;
}

ebit_status fail(ebit_ctx* c, ebit_status s, const char* what) {
  if (c) snprintf(c->msg, sizeof(c->msg), "%s", what);
  return s;
}

ebit_status hip_fail(ebit_ctx* c, hipError_t e, const char* where) {
  c->herr = e;
  snprintf(c->msg, sizeof(c->msg), "%s: %s", where, hipGetErrorString(e));
  return EBIT_EHIP;
}

#define HIPCK(ctx, expr, where)                          \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

void set_ops(ebit_ctx* c) {
  const ebit_props& p = c->props;
  const double dt = c->dt;
  for (int sys = 0; sys < 2; ++sys) {
    FineOp& op = c->op[sys];
    op.d = c->fd;
    op.h = c->grid.h;
    op.ih2 = 1.0 / (c->grid.h * c->grid.h);
    op.sys = sys;
    op.rho[0] = p.rho_v;
    op.rho[1] = p.rho_l;
    op.dt = dt;
    op.Tsat = p.T_sat;
    op.theta_min = c->opts.theta_min;
    op.flags = c->flags;
    for (int a = 0; a < 3; ++a) op.th[a] = c->th[a];
    if (sys == EBIT_SYS_HEAT) {
      op.mass[0] = p.rho_v * p.cp_v / dt;
      op.mass[1] = p.rho_l * p.cp_l / dt;
      op.coef[0] = p.lam_v;
      op.coef[1] = p.lam_l;
      for (int s = 0; s < 6; ++s) {
        op.bc[s] = c->grid.T_bc[s];
        op.bcval[s] = c->grid.T_val[s];
      }
    } else {
      op.mass[0] = op.mass[1] = 0.0;
      op.coef[0] = dt / p.rho_v;
      op.coef[1] = dt / p.rho_l;
      for (int s = 0; s < 6; ++s) {
        op.bc[s] = c->grid.p_bc[s];
        op.bcval[s] = c->grid.p_val[s];
      }
    }
  }
}

ebit_status check_ready(ebit_ctx* c) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  if (!c->built) return fail(c, EBIT_ESTATE, "ebit_build_coeffs has not been called");
  return EBIT_OK;
}

ebit_status solve_status(const EbitSolveOut& r, ebit_stats* st) {
  if (st) {
    st->iters = r.iters;
    st->vcycles = r.iters;
    st->rel_res = r.rel_res;
    st->bnorm = r.bnorm;
    st->res_floor = r.res_floor;
  }
  if (r.status == 1) return EBIT_ENOCONV;
  if (r.status == 2) return EBIT_ENAN;
  return EBIT_OK;
}

hipError_t replan(EbitPlan** plan, ebit_ctx* const* ctx, int n, const ebit_opts* o, void* mem, size_t bytes);

// The FP64 fallback of a mixed-precision solve whose FP32 inner cycle
// stopped contracting: the same cases, re-planned in FP64 (the hierarchies
// hold FP64 coefficients and tail images in either precision), continue
// from the mixed iterate (a case already converged stops at once); the
// mixed plan is restored afterwards.
hipError_t solve_fp64_fallback(EbitPlan** plan, ebit_ctx* const* ctx, int n, const ebit_opts& mixed, void* mem,
                               size_t bytes, int sys, double* const* x, hipStream_t st, EbitProfiler* pf,
                               EbitSolveOut* r) {
  ebit_opts o64 = mixed;
  o64.precision = EBIT_FP64;
  hipError_t e = replan(plan, ctx, n, &o64, mem, bytes);
  if (e == hipSuccess) e = ebit_plan_solve(*plan, sys, x, 1, st, pf, r);
  const hipError_t e2 = replan(plan, ctx, n, &mixed, mem, bytes);
  return e != hipSuccess ? e : e2;
}

ebit_status run_solve(ebit_ctx* c, int sys, double* x, int use_guess, ebit_stats* st) {
  EbitSolveOut r;
  double* xs[1] = {x};
  hipError_t e = ebit_plan_solve(c->plan, sys, xs, use_guess, c->st, c->prof, &r);
  if (e != hipSuccess) return hip_fail(c, e, "solve");
  int fell = 0;
  if (r.status == 1 && r.stalled && c->opts.precision == EBIT_MIXED) {
    ebit_ctx* cs[1] = {c};
    e = solve_fp64_fallback(&c->plan, cs, 1, c->opts, c->plan_mem, c->plan_bytes, sys, xs, c->st, c->prof, &r);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 fallback solve");
    fell = 1;
  }
  const ebit_status s = solve_status(r, st);
  if (st) st->fp64_fallback = fell;
  if (s == EBIT_ENOCONV) return fail(c, s, "no convergence within max_iters");
  if (s == EBIT_ENAN) return fail(c, s, "NaN or Inf in a residual norm");
  return s;
}

// First half of a coefficient build: argument checks and the geometry pass
// (cut fractions, flags, facets); its error bits land in the context's Scal.
ebit_status build_launch(ebit_ctx* c, const double* const marker[3], const uint8_t* vcol, const uint8_t* ccol,
                         double dt, hipStream_t st) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  if (!marker || !vcol || !ccol) return fail(c, EBIT_EINVAL, "NULL marker or colour array");
  for (int a = 0; a < c->grid.dim; ++a)
    if (!marker[a]) return fail(c, EBIT_EINVAL, "NULL marker array");
  if (!(dt > 0) || !isfinite(dt)) return fail(c, EBIT_EINVAL, "dt must be positive");
  c->built = 0;
  c->dt = dt;
  HIPCK(c, ebit_launch_fill_f64((long long)(sizeof(Scal) / sizeof(double)), (double*)c->B.scal, 0.0, st), "reset");
  HIPCK(c, ebit_launch_geometry(&c->fd, c->grid.h, marker, vcol, ccol, c->flags, c->cF, c->nF, c->th, c->B.scal, st),
        "geometry");
  return EBIT_OK;
}

// Geometry errors the geometry pass left in the status scalars.
ebit_status geometry_check(ebit_ctx* c, const Scal& hs) {
  if (hs.err & ERR_GEOM_MARKER) return fail(c, EBIT_EGEOM, "a marker is inconsistent with the vertex colours");
  if (hs.err & ERR_GEOM_SEAM) return fail(c, EBIT_EGEOM, "periodic seam markers or colours disagree");
  if (hs.err & ERR_GEOM_NOFACET) return fail(c, EBIT_EGEOM, "a cut link has no interface cell on either side");
  return EBIT_OK;
}

// the operators and hierarchies (every index stays in range whatever the
// geometry, so this may run before the geometry status is known)
ebit_status build_operators(ebit_ctx* c, hipStream_t st) {
  set_ops(c);
  const int want32 = c->opts.precision == EBIT_MIXED;
  HIPCK(c, ebit_build_hierarchy(c->op, c->lv, c->nlev, want32, c->build_tabs, c->build_ls, st), "hierarchy");
  if (c->fd.dim == 3) HIPCK(c, ebit_launch_split_flags(&c->fd, c->flags, c->B.fsplit, st), "split flags");
  return EBIT_OK;
}

// Second half: report geometry errors, then the operators and hierarchies.
ebit_status build_finish(ebit_ctx* c, const Scal& hs, hipStream_t st) {
  ebit_status s = geometry_check(c, hs);
  if (s != EBIT_OK) return s;
  s = build_operators(c, st);
  if (s != EBIT_OK) return s;
  c->built = 1;
  return EBIT_OK;
}

void stats_init(ebit_stats* s) {
  if (!s) return;
  memset(s, 0, sizeof(*s));
}

// ---- batched per-case launches ------------------------------------------

unsigned blocks_of(long long n) { return (unsigned)((n + EBIT_BLOCK - 1) / EBIT_BLOCK); }

// Carve the batch tables (base == nullptr only measures); fills t when given.
size_t batch_tabs_layout(int n, char* base, BatchTabs* t) {
  Carver cv{base, 0};
  BatchTabs tt;
  memset(&tt, 0, sizeof(tt));
  auto tab = [&](Tab& x, size_t bytes) {
    x.dev = cv.take<char>(bytes);
    x.cap = bytes;
  };
  tab(tt.geo, n * sizeof(GeoArgs));
  tab(tt.fine, n * sizeof(BuildFineArgs));
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) tab(tt.coarse[q], n * sizeof(BuildCoarseArgs));
  tab(tt.small, n * sizeof(BuildSmallArgs));
  tab(tt.split, n * sizeof(SplitArgs));
  tab(tt.heat, n * sizeof(HeatRhsArgs));
  tab(tt.flux, n * sizeof(FluxArgs));
  tab(tt.proj, n * sizeof(ProjArgs));
  tab(tt.projfu, n * sizeof(ProjArgs));
  tab(tt.fin, n * sizeof(FinArgs));
  tab(tt.scal0, n * sizeof(ScalArgs));
  tab(tt.scalg, n * sizeof(ScalArgs));
  for (int k = 0; k < 5; ++k) tt.geo_start[k] = cv.take<int>(n + 1);
  tt.cell_start = cv.take<int>(n + 1);
  tt.red_start = cv.take<int>(n + 1);
  tt.fine_start = cv.take<int>(n + 1);
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) tt.coarse_start[q] = cv.take<int>(n + 1);
  tt.small_start = cv.take<int>(n + 1);
  tt.unit_start = cv.take<int>(n + 1);
  tt.split_start = cv.take<int>(n + 1);
  tt.gather = cv.take<Scal>(n);
  if (t) *t = tt;
  return (cv.off + ALIGN - 1) / ALIGN * ALIGN;
}

void batch_tabs_free(ebit_batch* b) {
  BatchTabs& t = b->t;
  Tab* all[] = {&t.geo, &t.fine, &t.small, &t.split, &t.heat, &t.flux, &t.proj, &t.projfu, &t.fin, &t.scal0,
                &t.scalg};
  for (Tab* x : all) {
    delete[] x->host;
    x->host = nullptr;
  }
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) {
    delete[] t.coarse[q].host;
    t.coarse[q].host = nullptr;
  }
}

// The tables' host images and the block offsets of every launch (uploaded
// here, once: they depend on the grids only).
bool batch_tabs_create(ebit_batch* b, char* base) {
  const int n = b->n;
  BatchTabs& t = b->t;
  batch_tabs_layout(n, base, &t);
  Tab* all[] = {&t.geo, &t.fine, &t.small, &t.split, &t.heat, &t.flux, &t.proj, &t.projfu, &t.fin, &t.scal0,
                &t.scalg};
  for (Tab* x : all) {
    x->host = new (std::nothrow) char[x->cap];
    if (!x->host) return false;
  }
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) {
    t.coarse[q].host = new (std::nothrow) char[t.coarse[q].cap];
    if (!t.coarse[q].host) return false;
  }
  const int stride = n + 1;
  const int nstarts = 5 + 3 + EBIT_MAX_LEVELS + 3;
  int* h = new (std::nothrow) int[(size_t)nstarts * stride];
  if (!h) return false;
  memset(h, 0, sizeof(int) * (size_t)nstarts * stride);
  int* geo = h;                        // 5 x stride
  int* cell = h + 5 * stride;
  int* red = cell + stride;
  int* fine = red + stride;
  int* coarse = fine + stride;         // EBIT_MAX_LEVELS x stride
  int* small = coarse + EBIT_MAX_LEVELS * stride;
  int* unit = small + stride;
  int* split = unit + stride;
  t.fine_n = 0;
  t.ncoarse = 0;
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) t.coarse_n[q] = 0;
  for (int c = 0; c < n; ++c) {
    const ebit_ctx* x = b->ctx[c];
    for (int k = 0; k < 5; ++k) geo[k * stride + c + 1] = geo[k * stride + c] + (int)ebit_geo_blocks(&x->fd, k);
    const int cb = (int)blocks_of(x->fd.N);
    cell[c + 1] = cell[c] + cb;
    red[c + 1] = red[c] + (cb < EBIT_RED_BLOCKS ? cb : EBIT_RED_BLOCKS);
    small[c + 1] = small[c] + 2;
    unit[c + 1] = unit[c] + 1;
    split[c + 1] = split[c] + (x->fd.dim == 3 ? (int)blocks_of(2 * split_half(x->fd)) : 0);
    if (x->build_ls > 1 && x->nlev > 1) {
      fine[t.fine_n + 1] = fine[t.fine_n] + 2 * (int)blocks_of(x->lv[1].d.N);
      ++t.fine_n;
    }
    for (int l = 2; l < x->build_ls && l < x->nlev; ++l) {
      const int q = l - 2;
      int* s = coarse + q * stride;
      s[t.coarse_n[q] + 1] = s[t.coarse_n[q]] + 2 * (int)blocks_of(x->lv[l].d.N);
      ++t.coarse_n[q];
      if (q + 1 > t.ncoarse) t.ncoarse = q + 1;
    }
  }
  for (int k = 0; k < 5; ++k) t.geo_blocks[k] = geo[k * stride + n];
  t.cell_blocks = cell[n];
  t.red_blocks = red[n];
  t.fine_blocks = fine[t.fine_n];
  for (int q = 0; q < EBIT_MAX_LEVELS; ++q) t.coarse_blocks[q] = coarse[q * stride + t.coarse_n[q]];
  t.split_blocks = split[n];
  hipError_t e = hipSuccess;
  for (int k = 0; k < 5 && e == hipSuccess; ++k)
    e = hipMemcpy(t.geo_start[k], geo + k * stride, sizeof(int) * stride, hipMemcpyHostToDevice);
  int* const src[] = {cell, red, fine, small, unit, split};
  int* const dst[] = {t.cell_start, t.red_start, t.fine_start, t.small_start, t.unit_start, t.split_start};
  for (int k = 0; k < 6 && e == hipSuccess; ++k)
    e = hipMemcpy(dst[k], src[k], sizeof(int) * stride, hipMemcpyHostToDevice);
  for (int q = 0; q < EBIT_MAX_LEVELS && e == hipSuccess; ++q)
    e = hipMemcpy(t.coarse_start[q], coarse + q * stride, sizeof(int) * stride, hipMemcpyHostToDevice);
  delete[] h;
  return e == hipSuccess;
}

// Upload a table's new content (len bytes at src) unless it is unchanged.
hipError_t tab_put(ebit_batch* b, Tab& x, const void* src, size_t len) {
  if (x.valid && x.len == len && memcmp(x.host, src, len) == 0) return hipSuccess;
  memcpy(x.host, src, len);
  x.len = len;
  x.valid = 1;
  return hipMemcpyAsync(x.dev, x.host, len, hipMemcpyHostToDevice, b->st);
}

}  // namespace

extern "C" {

void ebit_default_opts(ebit_opts* o) {
  if (!o) return;
  o->precision = EBIT_FP64;
  o->outer = EBIT_OUTER_PCG;
  o->rtol = 1e-9;
  o->max_iters = 200;
  o->nu1 = 2;
  o->nu2 = 2;
  o->theta_min = 1e-3;
  o->check_every = 1;
  o->tail_cells = 4096;
}

const char* ebit_status_string(ebit_status s) {
  switch (s) {
    case EBIT_OK: return "ok";
    case EBIT_EINVAL: return "invalid argument";
    case EBIT_ENOMEM: return "workspace too small";
    case EBIT_EGEOM: return "inconsistent interface geometry";
    case EBIT_ENOCONV: return "solver did not converge";
    case EBIT_ENAN: return "NaN or Inf in the solver";
    case EBIT_EHIP: return "HIP runtime error";
    case EBIT_ESTATE: return "call order violated";
    case EBIT_EIO: return "schedule cache file not writable";
  }
  return "unknown status";
}

size_t ebit_workspace_bytes(const ebit_grid* g, const ebit_opts* o) {
  char msg[256];
  if (!valid_grid(g, msg, sizeof msg)) return 0;
  return layout(g, o, nullptr, nullptr);
}

ebit_status ebit_create(ebit_ctx** out, const ebit_grid* g, const ebit_props* p, const ebit_opts* o, void* ws,
                        size_t bytes, void* stream) {
  if (!out) return EBIT_EINVAL;
  *out = nullptr;
  char msg[256];
  if (!valid_grid(g, msg, sizeof msg) || !valid_props(p, msg, sizeof msg) || !valid_opts(o, msg, sizeof msg))
    return EBIT_EINVAL;
  if (!ws || ((uintptr_t)ws % ALIGN) != 0) return EBIT_EINVAL;
  const size_t need = layout(g, o, nullptr, nullptr);
  if (bytes < need) return EBIT_ENOMEM;
  ebit_ctx* c = new (std::nothrow) ebit_ctx;
  if (!c) return EBIT_ENOMEM;
  memset(c, 0, sizeof(*c));
  if (const char* lp = getenv("EBIT_SOLVE_LOG")) snprintf(c->solve_log, sizeof(c->solve_log), "%s", lp);
  c->grid = *g;
  c->props = *p;
  if (o)
    c->opts = *o;
  else
    ebit_default_opts(&c->opts);
  if (c->opts.check_every < 1) c->opts.check_every = 1;
  c->st = (hipStream_t)stream;
  c->ws = (char*)ws;
  c->ws_bytes = bytes;
  layout(g, o, c->ws, c);
  c->B.prof = nullptr;
  c->B.tail_lds = ebit_tail_lds_setup();
  c->herr = hipSuccess;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return EBIT_EHIP;
  }
  {
    // hierarchy-build tables: fixed pointers, uploaded once
    const size_t tb = ebit_build_table_bytes();
    char* host = new (std::nothrow) char[tb];
    hipError_t e = host ? hipSuccess : hipErrorOutOfMemory;
    if (host) {
      ebit_build_tables(c->lv, c->nlev, c->opts.precision == EBIT_MIXED, host);
      c->build_ls = *(const int*)host;
      e = hipMemcpy(c->build_tabs, host, tb, hipMemcpyHostToDevice);
      delete[] host;
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      (void)hipEventDestroy(c->ev0);
      (void)hipEventDestroy(c->ev1);
      delete c;
      return EBIT_EHIP;
    }
  }
  const EbitPlanCase pc{c->lv, c->nlev, c->op, c->B, c->bvec};
  if (ebit_plan_create(&c->plan, 1, &pc, &c->opts, c->B.tail_lds, c->plan_mem, c->plan_bytes) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(c->ev0);
    (void)hipEventDestroy(c->ev1);
    delete c;
    return EBIT_EHIP;
  }
  *out = c;
  return EBIT_OK;
}

ebit_status ebit_destroy(ebit_ctx* c) {
  if (!c) return EBIT_EINVAL;
  ebit_plan_destroy(c->plan);
  (void)hipEventDestroy(c->ev0);
  (void)hipEventDestroy(c->ev1);
  if (c->prof) {
    for (int i = 0; i < EBIT_PROF_CAP; ++i) {
      (void)hipEventDestroy(c->prof->ev0[i]);
      (void)hipEventDestroy(c->prof->ev1[i]);
    }
    delete c->prof;
  }
  delete c;
  return EBIT_OK;
}

const char* ebit_last_error(const ebit_ctx* c) { return c ? c->msg : "null context"; }

ebit_status ebit_build_coeffs(ebit_ctx* c, const double* const marker[3], const uint8_t* vcol, const uint8_t* ccol,
                              double dt) {
  ebit_status s = build_launch(c, marker, vcol, ccol, dt, c ? c->st : nullptr);
  if (s != EBIT_OK) return s;
  // operators and hierarchy go out behind the geometry pass; its status is
  // read once, after them (an invalid geometry leaves the context unbuilt)
  s = build_operators(c, c->st);
  if (s != EBIT_OK) return s;
  Scal hs;
  HIPCK(c, hipMemcpyAsync(&hs, c->B.scal, sizeof(Scal), hipMemcpyDeviceToHost, c->st), "geometry status");
  HIPCK(c, hipStreamSynchronize(c->st), "geometry sync");
  s = geometry_check(c, hs);
  if (s != EBIT_OK) return s;
  c->built = 1;
  return EBIT_OK;
}

// One JSON line per solve call, appended to the file EBIT_SOLVE_LOG named
// when the context was created (nothing when it was unset); a file that
// cannot be opened is skipped.
static void log_solve(const ebit_ctx* c, const char* call, const ebit_stats* st) {
  if (!c->solve_log[0] || !st) return;
  FILE* f = fopen(c->solve_log, "a");
  if (!f) return;
  fprintf(f,
          "{\"call\": \"%s\", \"dim\": %d, \"n\": [%d, %d, %d], \"precision\": %d, \"status\": %d, "
          "\"iters\": %d, \"vcycles\": %d, \"rel_res\": %.17g, \"bnorm\": %.17g, \"res_floor\": %.17g, "
          "\"seconds\": %.9g, \"div_max\": %.17g, \"fp64_fallback\": %d}\n",
          call, c->grid.dim, c->grid.n[0], c->grid.n[1], c->grid.dim == 3 ? c->grid.n[2] : 1, c->opts.precision,
          st->status, st->iters, st->vcycles, st->rel_res, st->bnorm, st->res_floor, st->seconds, st->div_max,
          st->fp64_fallback);
  fclose(f);
}

ebit_status ebit_heat_solve(ebit_ctx* c, const double* Ts, double* T, int use_guess, ebit_stats* st_in) {
  ebit_stats st_loc;
  ebit_stats* st = st_in ? st_in : (c && c->solve_log[0] ? &st_loc : nullptr);
  stats_init(st);
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!Ts || !T) return fail(c, EBIT_EINVAL, "NULL field");
  HIPCK(c, hipEventRecord(c->ev0, c->st), "event");
  HIPCK(c, ebit_launch_heat_rhs(&c->op[EBIT_SYS_HEAT], Ts, c->bvec, c->st), "heat rhs");
  s = run_solve(c, EBIT_SYS_HEAT, T, use_guess, st);
  if (s == EBIT_EHIP) return s;
  HIPCK(c, hipEventRecord(c->ev1, c->st), "event");
  HIPCK(c, hipEventSynchronize(c->ev1), "event sync");
  if (st) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    st->seconds = ms * 1e-3;
    st->status = s;
  }
  log_solve(c, "heat_solve", st);
  return s;
}

ebit_status ebit_mass_flux(ebit_ctx* c, const double* T, double* mdot, double* const mface[3], ebit_stats* st) {
  stats_init(st);
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!T || !mdot) return fail(c, EBIT_EINVAL, "NULL field");
  if (mface)
    for (int a = 0; a < c->grid.dim; ++a)
      if (!mface[a]) return fail(c, EBIT_EINVAL, "mdot_face must be NULL or hold dim arrays");
  HIPCK(c, hipEventRecord(c->ev0, c->st), "event");
  HIPCK(c, ebit_launch_fill_f64((long long)(sizeof(Scal) / sizeof(double)), (double*)c->B.scal, 0.0, c->st),
        "reset");
  const double lam[2] = {c->props.lam_v, c->props.lam_l};
  HIPCK(c,
        ebit_launch_mass_flux(&c->fd, c->grid.h, lam, c->props.h_lg, c->props.T_sat, c->opts.theta_min, c->flags,
                              c->th, c->cF, c->nF, T, mdot, mface, c->B.scal, c->st),
        "mass flux");
  // without stats the call does not wait for the device
  if (!st) return EBIT_OK;
  HIPCK(c, hipEventRecord(c->ev1, c->st), "event");
  Scal hs;
  HIPCK(c, hipMemcpyAsync(&hs, c->B.scal, sizeof(Scal), hipMemcpyDeviceToHost, c->st), "status");
  HIPCK(c, hipStreamSynchronize(c->st), "sync");
  if (st) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    st->seconds = ms * 1e-3;
    st->fallbacks = hs.fallbacks;
    st->status = EBIT_OK;
  }
  return EBIT_OK;
}

ebit_status ebit_project_rhs(ebit_ctx* c, double* const ul[3], double* const uv[3], const double* mdot, double* b) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!ul || !uv || !mdot || !b) return fail(c, EBIT_EINVAL, "NULL field");
  for (int a = 0; a < c->grid.dim; ++a)
    if (!ul[a] || !uv[a]) return fail(c, EBIT_EINVAL, "NULL velocity array");
  const double rho[2] = {c->props.rho_v, c->props.rho_l};
  HIPCK(c,
        ebit_launch_proj_rhs(&c->fd, c->grid.h, rho, c->dt, c->grid.p_bc, c->grid.p_val, c->flags, c->th, c->nF,
                             mdot, ul, uv, b, c->st),
        "projection rhs");
  return EBIT_OK;
}

ebit_status ebit_project(ebit_ctx* c, double* const ul[3], double* const uv[3], const double* mdot, double* p,
                         int use_guess, ebit_stats* st_in) {
  ebit_stats st_loc;
  ebit_stats* st = st_in ? st_in : (c && c->solve_log[0] ? &st_loc : nullptr);
  stats_init(st);
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!p) return fail(c, EBIT_EINVAL, "NULL pressure");
  HIPCK(c, hipEventRecord(c->ev0, c->st), "event");
  s = ebit_project_rhs(c, ul, uv, mdot, c->bvec);
  if (s != EBIT_OK) return s;
  s = run_solve(c, EBIT_SYS_PRESSURE, p, use_guess, st);
  if (s == EBIT_EHIP) return s;
  const double rho[2] = {c->props.rho_v, c->props.rho_l};
  HIPCK(c,
        ebit_launch_face_update(&c->fd, c->grid.h, rho, c->dt, c->grid.p_bc, c->grid.p_val, c->flags, c->th, ul, uv,
                                p, c->B.partial, c->B.scal, c->st),
        "face update");
  HIPCK(c, hipEventRecord(c->ev1, c->st), "event");
  Scal hs;
  HIPCK(c, hipMemcpyAsync(&hs, c->B.scal, sizeof(Scal), hipMemcpyDeviceToHost, c->st), "status");
  HIPCK(c, hipStreamSynchronize(c->st), "sync");
  if (st) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    st->seconds = ms * 1e-3;
    st->div_max = hs.divmax;
    st->status = s;
  }
  log_solve(c, "project", st);
  return s;
}

ebit_status ebit_project_one_fluid(ebit_ctx* c, double* const u[3], const double* mdot, double* p, int use_guess,
                                   ebit_stats* st_in) {
  ebit_stats st_loc;
  ebit_stats* st = st_in ? st_in : (c && c->solve_log[0] ? &st_loc : nullptr);
  stats_init(st);
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!u || !mdot || !p) return fail(c, EBIT_EINVAL, "NULL field");
  for (int a = 0; a < c->grid.dim; ++a)
    if (!u[a]) return fail(c, EBIT_EINVAL, "NULL velocity array");
  const double rho[2] = {c->props.rho_v, c->props.rho_l};
  HIPCK(c, hipEventRecord(c->ev0, c->st), "event");
  HIPCK(c,
        ebit_launch_proj_rhs_one(&c->fd, c->grid.h, rho, c->dt, c->grid.p_bc, c->grid.p_val, c->flags, c->th, c->cF,
                                 c->nF, mdot, u, c->bvec, c->st),
        "one-fluid rhs");
  s = run_solve(c, EBIT_SYS_PRESSURE, p, use_guess, st);
  if (s == EBIT_EHIP) return s;
  HIPCK(c,
        ebit_launch_face_update_one(&c->fd, c->grid.h, rho, c->dt, c->grid.p_bc, c->grid.p_val, c->flags, c->th,
                                    c->cF, c->nF, mdot, u, p, c->B.partial, c->B.scal, c->st),
        "one-fluid face update");
  HIPCK(c, hipEventRecord(c->ev1, c->st), "event");
  Scal hs;
  HIPCK(c, hipMemcpyAsync(&hs, c->B.scal, sizeof(Scal), hipMemcpyDeviceToHost, c->st), "status");
  HIPCK(c, hipStreamSynchronize(c->st), "sync");
  if (st) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    st->seconds = ms * 1e-3;
    st->div_max = hs.divmax;
    st->status = s;
  }
  log_solve(c, "project_one_fluid", st);
  return s;
}

ebit_status ebit_get_geometry(ebit_ctx* c, double* const theta[3], uint8_t* flags, double* facet) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  const Dims& d = c->fd;
  if (theta)
    for (int a = 0; a < d.dim; ++a)
      if (theta[a])
        HIPCK(c, hipMemcpyAsync(theta[a], c->th[a], faces(d, a) * sizeof(double), hipMemcpyDeviceToDevice, c->st),
              "copy theta");
  if (flags) HIPCK(c, hipMemcpyAsync(flags, c->flags, d.N, hipMemcpyDeviceToDevice, c->st), "copy flags");
  if (facet) {
    HIPCK(c, hipMemcpyAsync(facet, c->cF, 3 * d.N * sizeof(double), hipMemcpyDeviceToDevice, c->st), "copy facet");
    HIPCK(c, hipMemcpyAsync(facet + 3 * d.N, c->nF, 3 * d.N * sizeof(double), hipMemcpyDeviceToDevice, c->st),
          "copy facet");
  }
  HIPCK(c, hipStreamSynchronize(c->st), "sync");
  return EBIT_OK;
}

ebit_status ebit_apply(ebit_ctx* c, int sys, const double* x, double* y) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (sys != EBIT_SYS_HEAT && sys != EBIT_SYS_PRESSURE) return fail(c, EBIT_EINVAL, "bad system");
  if (!x || !y) return fail(c, EBIT_EINVAL, "NULL vector");
  HIPCK(c, ebit_launch_apply(&c->op[sys], x, y, c->st), "apply");
  return EBIT_OK;
}

ebit_status ebit_extend(ebit_ctx* c, double* q, int mode, int iters) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!q) return fail(c, EBIT_EINVAL, "NULL field");
  if (mode != EBIT_EXT_LIQ_TO_VAP && mode != EBIT_EXT_VAP_TO_LIQ && mode != EBIT_EXT_IFACE_TO_BAND)
    return fail(c, EBIT_EINVAL, "bad extension mode");
  if (iters < 0) return fail(c, EBIT_EINVAL, "negative step count");
  // solver scratch: the band and target bytes in the FP32 iterate (4 N
  // bytes), the target list in the FP64 iterate, the weights in the
  // direction and product vectors, the targets' band normal sums in the
  // residual, the second FP64 iterate and (3D) the colour-split residual,
  // the list length in the reduction partials, the other iterate in b
  double* w[3] = {c->B.p[0], c->B.p[1], c->B.q};
  double* ns[3] = {c->B.r, c->B.z64b, c->fd.dim == 3 ? c->B.r64s : nullptr};
  HIPCK(c,
        ebit_launch_extend(&c->fd, mode, iters, c->flags, c->nF, q, c->bvec, (uint8_t*)c->B.z32,
                           (unsigned long long*)c->B.z64, w, ns, (int*)c->B.partial, c->st),
        "extend");
  return EBIT_OK;
}

ebit_status ebit_ghost_band(ebit_ctx* c, double* const u_l[3], double* const u_v[3], const double* mdot_band) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!u_l || !u_v || !mdot_band) return fail(c, EBIT_EINVAL, "NULL argument");
  for (int a = 0; a < c->fd.dim; ++a)
    if (!u_l[a] || !u_v[a]) return fail(c, EBIT_EINVAL, "NULL velocity array");
  // scratch as in ebit_extend: the band bytes in the FP32 iterate, the band
  // normals in the direction and product vectors, the dilation's counter in
  // the reduction partials
  const double jump = 1.0 / c->props.rho_l - 1.0 / c->props.rho_v;
  double* nb[3] = {c->B.p[0], c->B.p[1], c->B.q};
  HIPCK(c,
        ebit_launch_ghost_band(&c->fd, jump, c->flags, c->th, c->nF, mdot_band, u_l, u_v, (uint8_t*)c->B.z32, nb,
                               (int*)c->B.partial, c->st),
        "band ghost velocities");
  return EBIT_OK;
}

ebit_status ebit_interface_velocity(ebit_ctx* c, const double* const u_l[3], const double* const u_v[3],
                                    const double* mdot_cell, double* const u_gamma[3]) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  const int dim = c->fd.dim;
  if (!u_l || !u_v || !u_gamma || !mdot_cell) return fail(c, EBIT_EINVAL, "NULL argument");
  for (int a = 0; a < dim; ++a)
    if (!u_l[a] || !u_v[a] || !u_gamma[a]) return fail(c, EBIT_EINVAL, "NULL field");
  const double* ul[3] = {u_l[0], u_l[1], dim == 3 ? u_l[2] : nullptr};
  const double* uv[3] = {u_v[0], u_v[1], dim == 3 ? u_v[2] : nullptr};
  double* out[3] = {u_gamma[0], u_gamma[1], dim == 3 ? u_gamma[2] : nullptr};
  HIPCK(c,
        ebit_launch_iface_velocity(&c->fd, c->flags, c->nF, ul, uv, mdot_cell, c->props.rho_l, c->props.rho_v,
                                   out, c->st),
        "interface velocity");
  return EBIT_OK;
}

ebit_status ebit_advect_energy(ebit_ctx* c, const double* T_liq, const double* T_vap, const double* const u_l[3],
                               const double* const u_v[3], const uint8_t* cell_colour, double dt, double eps,
                               double* T_star) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  const int dim = c->fd.dim;
  if (!T_liq || !T_vap || !u_l || !u_v || !cell_colour || !T_star) return fail(c, EBIT_EINVAL, "NULL argument");
  for (int a = 0; a < dim; ++a)
    if (!u_l[a] || !u_v[a]) return fail(c, EBIT_EINVAL, "NULL face field");
  if (T_star == T_liq || T_star == T_vap) return fail(c, EBIT_EINVAL, "T_star must not be an input field");
  if (!(dt >= 0.0) || !isfinite(dt)) return fail(c, EBIT_EINVAL, "dt must be finite and >= 0");
  if (!(eps >= 1e-60 && eps <= 1e60)) return fail(c, EBIT_EINVAL, "eps must lie in [1e-60, 1e60]");
  const double* ul[3] = {u_l[0], u_l[1], dim == 3 ? u_l[2] : nullptr};
  const double* uv[3] = {u_v[0], u_v[1], dim == 3 ? u_v[2] : nullptr};
  HIPCK(c, ebit_launch_advect_energy(&c->fd, c->grid.h, T_liq, T_vap, ul, uv, cell_colour, dt, eps, T_star, c->st),
        "energy advection");
  return EBIT_OK;
}

ebit_status ebit_advect_markers(ebit_ctx* c, const double* const u_gamma[3], double* const marker[3],
                                uint8_t* vertex_colour, uint8_t* cell_colour, double dt) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  if (c->fd.dim != 2) return fail(c, EBIT_EINVAL, "marker motion is two-dimensional");
  if (c->fd.n[0] < 4 || c->fd.n[1] < 4) return fail(c, EBIT_EINVAL, "marker motion needs 4 cells per axis");
  if ((long long)c->fd.n[0] * (c->fd.n[1] + 1) + (long long)(c->fd.n[0] + 1) * c->fd.n[1] >= (1LL << 31))
    return fail(c, EBIT_EINVAL, "marker motion needs fewer than 2^31 edges");
  if (!u_gamma || !marker || !u_gamma[0] || !u_gamma[1] || !marker[0] || !marker[1] || !vertex_colour ||
      !cell_colour)
    return fail(c, EBIT_EINVAL, "NULL argument");
  if (!(dt >= 0.0) || !isfinite(dt)) return fail(c, EBIT_EINVAL, "dt must be finite and >= 0");
  HIPCK(c,
        ebit_launch_advect(&c->fd, c->grid.h, dt, u_gamma, marker, vertex_colour, cell_colour, c->adv,
                           !c->adv_ready, c->adv_err, c->st),
        "advect");
  c->adv_ready = 1;
  int herr = 0;
  HIPCK(c, hipMemcpyAsync(&herr, c->adv_err, sizeof(int), hipMemcpyDeviceToHost, c->st), "advect status");
  HIPCK(c, hipStreamSynchronize(c->st), "advect sync");
  if (herr & 1) return fail(c, EBIT_EINVAL, "a marker moves more than one cell in a pass (or by a non-finite amount)");
  if (herr & 2) return fail(c, EBIT_EGEOM, "a cell holds other than 0 or 2 markers (a saddle)");
  return EBIT_OK;
}

ebit_status ebit_volume_fraction(ebit_ctx* c, const double* const marker[3], const uint8_t* vertex_colour,
                                 double* frac) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  if (c->fd.dim != 2) return fail(c, EBIT_EINVAL, "the volume fraction is two-dimensional");
  if ((long long)c->fd.n[0] * (c->fd.n[1] + 1) + (long long)(c->fd.n[0] + 1) * c->fd.n[1] >= (1LL << 31))
    return fail(c, EBIT_EINVAL, "the volume fraction needs fewer than 2^31 edges");
  if (!marker || !marker[0] || !marker[1] || !vertex_colour || !frac) return fail(c, EBIT_EINVAL, "NULL argument");
  HIPCK(c, ebit_launch_volume_fraction(&c->fd, marker, vertex_colour, frac, c->adv_err, c->st), "volume fraction");
  int herr = 0;
  HIPCK(c, hipMemcpyAsync(&herr, c->adv_err, sizeof(int), hipMemcpyDeviceToHost, c->st), "volume fraction status");
  HIPCK(c, hipStreamSynchronize(c->st), "volume fraction sync");
  if (herr) return fail(c, EBIT_EGEOM, "a cell holds other than 0 or 2 markers, or its corner colours do not "
                                       "change exactly at its markers");
  return EBIT_OK;
}

ebit_status ebit_heat_rhs(ebit_ctx* c, const double* Ts, double* b) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!Ts || !b) return fail(c, EBIT_EINVAL, "NULL vector");
  HIPCK(c, ebit_launch_heat_rhs(&c->op[EBIT_SYS_HEAT], Ts, b, c->st), "heat rhs");
  return EBIT_OK;
}

ebit_status ebit_profile(ebit_ctx* c, int enable) {
  if (!c) return EBIT_EINVAL;
  if (c->herr != hipSuccess) return EBIT_EHIP;
  if (enable && !c->prof) {
    EbitProfiler* pr = new (std::nothrow) EbitProfiler;
    if (!pr) return EBIT_ENOMEM;
    memset(pr, 0, sizeof(*pr));
    for (int i = 0; i < EBIT_PROF_CAP; ++i) {
      if (hipEventCreate(&pr->ev0[i]) != hipSuccess || hipEventCreate(&pr->ev1[i]) != hipSuccess) {
        delete pr;
        return fail(c, EBIT_EHIP, "hipEventCreate failed");
      }
    }
    c->prof = pr;
  }
  if (c->prof) {
    HIPCK(c, ebit_prof_flush(c->prof), "profile flush");
    c->prof->on = enable ? 1 : 0;
    if (enable)
      for (int k = 0; k < EBIT_PROF_CLASSES; ++k) {
        c->prof->launches[k] = 0;
        c->prof->ms[k] = 0.0;
      }
  }
  c->B.prof = c->prof;
  return EBIT_OK;
}

ebit_status ebit_profile_read(ebit_ctx* c, int kc, long long* launches, double* ms) {
  if (!c || kc < 0 || kc >= EBIT_PROF_CLASSES || !launches || !ms) return EBIT_EINVAL;
  if (!c->prof) {
    *launches = 0;
    *ms = 0.0;
    return EBIT_OK;
  }
  HIPCK(c, ebit_prof_flush(c->prof), "profile flush");
  *launches = c->prof->launches[kc];
  *ms = c->prof->ms[kc];
  return EBIT_OK;
}

ebit_status ebit_levels(const ebit_ctx* c, int* nlevels, int* sizes) {
  if (!c || !nlevels) return EBIT_EINVAL;
  *nlevels = c->nlev;
  if (sizes)
    for (int l = 0; l < c->nlev; ++l)
      for (int a = 0; a < 3; ++a) sizes[3 * l + a] = c->lv[l].d.n[a];
  return EBIT_OK;
}

/* ---- batches ---------------------------------------------------------- */

size_t ebit_batch_workspace_bytes(int ncases, const ebit_opts* o) {
  if (ncases < 1) return 0;
  const size_t b = std::max(ebit_plan_device_bytes(ncases, EBIT_FP64), ebit_plan_device_bytes(ncases, EBIT_MIXED));
  return (b + ALIGN - 1) / ALIGN * ALIGN + batch_tabs_layout(ncases, nullptr, nullptr);
}

ebit_status ebit_batch_create(ebit_batch** out, int ncases, ebit_ctx* const ctx[], void* ws, size_t bytes,
                              void* stream) {
  if (!out) return EBIT_EINVAL;
  *out = nullptr;
  if (ncases < 1 || !ctx || !ws || ((uintptr_t)ws % ALIGN) != 0) return EBIT_EINVAL;
  for (int c = 0; c < ncases; ++c) {
    if (!ctx[c] || ctx[c]->herr != hipSuccess) return EBIT_EINVAL;
    const ebit_opts& a = ctx[0]->opts;
    const ebit_opts& b = ctx[c]->opts;
    if (ctx[c]->grid.dim != ctx[0]->grid.dim || a.precision != b.precision || a.outer != b.outer ||
        a.rtol != b.rtol || a.max_iters != b.max_iters || a.nu1 != b.nu1 || a.nu2 != b.nu2 ||
        a.check_every != b.check_every || a.tail_cells != b.tail_cells)
      return EBIT_EINVAL;
    for (int q = 0; q < c; ++q)
      if (ctx[q] == ctx[c]) return EBIT_EINVAL;
  }
  if (bytes < ebit_batch_workspace_bytes(ncases, &ctx[0]->opts)) return EBIT_ENOMEM;
  ebit_batch* b = new (std::nothrow) ebit_batch;
  if (!b) return EBIT_ENOMEM;
  memset(b, 0, sizeof(*b));
  b->n = ncases;
  b->opts = ctx[0]->opts;
  b->st = (hipStream_t)stream;
  b->ws = ws;
  b->ws_bytes = bytes;
  b->ctx = new (std::nothrow) ebit_ctx*[ncases];
  b->hsc = new (std::nothrow) Scal[ncases];
  EbitPlanCase* pc = new (std::nothrow) EbitPlanCase[ncases];
  if (!b->ctx || !b->hsc || !pc) {
    delete[] b->ctx;
    delete[] b->hsc;
    delete[] pc;
    delete b;
    return EBIT_ENOMEM;
  }
  for (int c = 0; c < ncases; ++c) {
    b->ctx[c] = ctx[c];
    pc[c] = EbitPlanCase{ctx[c]->lv, ctx[c]->nlev, ctx[c]->op, ctx[c]->B, ctx[c]->bvec};
  }
  const size_t pb = (std::max(ebit_plan_device_bytes(ncases, EBIT_FP64), ebit_plan_device_bytes(ncases, EBIT_MIXED)) +
                     ALIGN - 1) / ALIGN * ALIGN;
  hipError_t e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess) e = ebit_plan_create(&b->plan, ncases, pc, &b->opts, ctx[0]->B.tail_lds, ws, pb);
  delete[] pc;
  if (e == hipSuccess && !batch_tabs_create(b, (char*)ws + pb)) e = hipErrorOutOfMemory;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ebit_batch_destroy(b);
    return EBIT_EHIP;
  }
  *out = b;
  return EBIT_OK;
}

ebit_status ebit_batch_destroy(ebit_batch* b) {
  if (!b) return EBIT_EINVAL;
  batch_tabs_free(b);
  ebit_plan_destroy(b->plan);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete[] b->ctx;
  delete[] b->hsc;
  delete b;
  return EBIT_OK;
}

const char* ebit_batch_last_error(const ebit_batch* b) { return b ? b->msg : "null batch"; }

}  // extern "C"

namespace {

ebit_status bfail(ebit_batch* b, ebit_status s, int c, const char* what) {
  snprintf(b->msg, sizeof(b->msg), "case %d: %s", c, what);
  return s;
}

ebit_status bhip(ebit_batch* b, hipError_t e, const char* where) {
  b->herr = e;
  snprintf(b->msg, sizeof(b->msg), "%s: %s", where, hipGetErrorString(e));
  return EBIT_EHIP;
}

#define BHIPCK(b, expr, where)                          \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return bhip(b, _e, where);    \
  } while (0)

// the cases' status scalars: cleared, or gathered side by side (one launch)
ebit_status batch_scal(ebit_batch* b, bool gather) {
  BatchTabs& t = b->t;
  std::vector<ScalArgs> v(b->n);
  for (int c = 0; c < b->n; ++c) v[c] = ScalArgs{b->ctx[c]->B.scal, gather ? t.gather + c : nullptr};
  Tab& x = gather ? t.scalg : t.scal0;
  BHIPCK(b, tab_put(b, x, v.data(), v.size() * sizeof(ScalArgs)), "status table");
  BHIPCK(b, ebit_launch_scal_many(b->n, (const ScalArgs*)x.dev, t.unit_start, b->st), "status");
  return EBIT_OK;
}

// copy every context's status scalars to b->hsc (one gather, one copy, one
// synchronisation)
ebit_status batch_read_scal(ebit_batch* b) {
  ebit_status s = batch_scal(b, true);
  if (s != EBIT_OK) return s;
  BHIPCK(b, hipMemcpyAsync(b->hsc, b->t.gather, b->n * sizeof(Scal), hipMemcpyDeviceToHost, b->st), "status");
  BHIPCK(b, hipStreamSynchronize(b->st), "sync");
  return EBIT_OK;
}

ebit_status batch_ready(ebit_batch* b) {
  if (!b) return EBIT_EINVAL;
  if (b->herr != hipSuccess) return EBIT_EHIP;
  for (int c = 0; c < b->n; ++c) {
    ebit_status s = check_ready(b->ctx[c]);
    if (s != EBIT_OK) return bfail(b, s, c, b->ctx[c]->msg);
  }
  return EBIT_OK;
}

// A mixed batch solve in which some case's inner cycle stopped contracting
// continues in FP64 for all cases from their current iterates (the cases
// already converged stop at once); fell[c] marks the cases that stalled.
hipError_t batch_fallback(ebit_batch* b, int sys, double* const* x, EbitSolveOut* r, std::vector<int>& fell) {
  fell.assign(b->n, 0);
  bool any = false;
  for (int c = 0; c < b->n; ++c)
    if (r[c].status == 1 && r[c].stalled) fell[c] = 1, any = true;
  if (!any || b->opts.precision != EBIT_MIXED) {
    fell.assign(b->n, 0);
    return hipSuccess;
  }
  const size_t pb = (std::max(ebit_plan_device_bytes(b->n, EBIT_FP64), ebit_plan_device_bytes(b->n, EBIT_MIXED)) +
                     ALIGN - 1) / ALIGN * ALIGN;
  return solve_fp64_fallback(&b->plan, b->ctx, b->n, b->opts, b->ws, pb, sys, x, b->st, nullptr, r);
}

// per-case solve results into stats; the first failing status is returned
ebit_status batch_results(ebit_batch* b, const EbitSolveOut* r, ebit_stats* stats, double seconds) {
  ebit_status first = EBIT_OK;
  for (int c = 0; c < b->n; ++c) {
    ebit_stats* st = stats ? &stats[c] : nullptr;
    if (st) memset(st, 0, sizeof(*st));
    const ebit_status s = solve_status(r[c], st);
    if (st) {
      st->seconds = seconds;
      st->status = s;
    }
    if (s != EBIT_OK && first == EBIT_OK) {
      first = s;
      bfail(b, s, c, s == EBIT_ENAN ? "NaN or Inf in a residual norm" : "no convergence within max_iters");
    }
  }
  return first;
}

}  // namespace

extern "C" {

ebit_status ebit_batch_build_coeffs(ebit_batch* b, const double* const marker[], const uint8_t* const vcol[],
                                    const uint8_t* const ccol[], const double dt[]) {
  if (!b) return EBIT_EINVAL;
  if (b->herr != hipSuccess) return EBIT_EHIP;
  if (!marker || !vcol || !ccol || !dt) return bfail(b, EBIT_EINVAL, -1, "NULL argument array");
  // every case's arguments are checked before the first launch
  for (int c = 0; c < b->n; ++c) {
    if (!vcol[c] || !ccol[c]) return bfail(b, EBIT_EINVAL, c, "NULL colour array");
    for (int a = 0; a < b->ctx[c]->grid.dim; ++a)
      if (!marker[3 * c + a]) return bfail(b, EBIT_EINVAL, c, "NULL marker array");
    if (!(dt[c] > 0) || !isfinite(dt[c])) return bfail(b, EBIT_EINVAL, c, "dt must be positive");
  }
  const int n = b->n;
  BatchTabs& t = b->t;
  const int dim = b->ctx[0]->fd.dim;
  const int want32 = b->opts.precision == EBIT_MIXED;
  std::vector<GeoArgs> geo(n);
  std::vector<BuildFineArgs> fine(t.fine_n > 0 ? t.fine_n : 1);
  std::vector<BuildCoarseArgs> coarse((size_t)EBIT_MAX_LEVELS * n);
  std::vector<BuildSmallArgs> small(n);
  std::vector<SplitArgs> split(n);
  int nf = 0, nc[EBIT_MAX_LEVELS] = {0};
  for (int c = 0; c < n; ++c) {
    ebit_ctx* x = b->ctx[c];
    x->built = 0;
    x->dt = dt[c];
    set_ops(x);
    ebit_geo_args(&geo[c], &x->fd, x->grid.h, marker + 3 * c, vcol[c], ccol[c], x->flags, x->cF, x->nF, x->th,
                  x->B.scal);
    BuildFineArgs f;
    BuildCoarseArgs cl[EBIT_MAX_LEVELS];
    const int ncl = ebit_build_args(x->op, x->lv, x->nlev, want32, x->build_ls, &f, cl);
    if (x->build_ls > 1 && x->nlev > 1) fine[nf++] = f;
    for (int q = 0; q < ncl; ++q) coarse[(size_t)q * n + nc[q]++] = cl[q];
    small[c].tabs = x->build_tabs;
    split[c] = SplitArgs{x->fd, x->flags, x->B.fsplit};
  }
  // the geometry of every case, then its status
  ebit_status s = batch_scal(b, false);
  if (s != EBIT_OK) return s;
  BHIPCK(b, tab_put(b, t.geo, geo.data(), n * sizeof(GeoArgs)), "geometry table");
  const int* gs[5] = {t.geo_start[0], t.geo_start[1], t.geo_start[2], t.geo_start[3], t.geo_start[4]};
  BHIPCK(b, ebit_launch_geometry_many(n, dim, (const GeoArgs*)t.geo.dev, gs, t.geo_blocks, b->st), "geometry");
  // the hierarchies (every index stays in range whatever the geometry)
  if (nf > 0) {
    BHIPCK(b, tab_put(b, t.fine, fine.data(), nf * sizeof(BuildFineArgs)), "build table");
    BHIPCK(b, ebit_launch_build_fine_many(nf, (const BuildFineArgs*)t.fine.dev, t.fine_start, t.fine_blocks, b->st),
           "hierarchy");
  }
  for (int q = 0; q < t.ncoarse; ++q) {
    if (!nc[q]) continue;
    BHIPCK(b, tab_put(b, t.coarse[q], &coarse[(size_t)q * n], nc[q] * sizeof(BuildCoarseArgs)), "build table");
    BHIPCK(b,
           ebit_launch_build_coarse_many(nc[q], dim, (const BuildCoarseArgs*)t.coarse[q].dev, t.coarse_start[q],
                                         t.coarse_blocks[q], b->st),
           "hierarchy");
  }
  BHIPCK(b, tab_put(b, t.small, small.data(), n * sizeof(BuildSmallArgs)), "build table");
  BHIPCK(b, ebit_launch_build_small_many(n, dim, (const BuildSmallArgs*)t.small.dev, t.small_start, b->st),
         "hierarchy");
  if (dim == 3) {
    BHIPCK(b, tab_put(b, t.split, split.data(), n * sizeof(SplitArgs)), "split table");
    BHIPCK(b,
           ebit_launch_split_flags_many(n, (const SplitArgs*)t.split.dev, t.split_start, t.split_blocks, b->st),
           "split flags");
  }
  s = batch_read_scal(b);
  if (s != EBIT_OK) return s;
  for (int c = 0; c < n; ++c) {
    s = geometry_check(b->ctx[c], b->hsc[c]);
    if (s != EBIT_OK) return bfail(b, s, c, b->ctx[c]->msg);
  }
  for (int c = 0; c < n; ++c) b->ctx[c]->built = 1;
  return EBIT_OK;
}

ebit_status ebit_batch_heat_solve(ebit_batch* b, const double* const T_star[], double* const T[], int use_guess,
                                  ebit_stats stats[]) {
  ebit_status s = batch_ready(b);
  if (s != EBIT_OK) return s;
  if (!T_star || !T) return bfail(b, EBIT_EINVAL, -1, "NULL argument array");
  for (int c = 0; c < b->n; ++c)
    if (!T_star[c] || !T[c]) return bfail(b, EBIT_EINVAL, c, "NULL field");
  BHIPCK(b, hipEventRecord(b->ev0, b->st), "event");
  {
    std::vector<HeatRhsArgs> v(b->n);
    for (int c = 0; c < b->n; ++c) v[c] = HeatRhsArgs{b->ctx[c]->op[EBIT_SYS_HEAT], T_star[c], b->ctx[c]->bvec};
    BHIPCK(b, tab_put(b, b->t.heat, v.data(), v.size() * sizeof(HeatRhsArgs)), "heat table");
    BHIPCK(b,
           ebit_launch_heat_rhs_many(b->n, (const HeatRhsArgs*)b->t.heat.dev, b->t.cell_start, b->t.cell_blocks,
                                     b->st),
           "heat rhs");
  }
  EbitSolveOut* r = new (std::nothrow) EbitSolveOut[b->n];
  if (!r) return EBIT_ENOMEM;
  hipError_t e = ebit_plan_solve(b->plan, EBIT_SYS_HEAT, T, use_guess, b->st, nullptr, r);
  std::vector<int> fell;
  if (e == hipSuccess) e = batch_fallback(b, EBIT_SYS_HEAT, T, r, fell);
  if (e != hipSuccess) {
    delete[] r;
    return bhip(b, e, "solve");
  }
  float ms = 0;
  if (hipEventRecord(b->ev1, b->st) == hipSuccess && hipEventSynchronize(b->ev1) == hipSuccess)
    (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
  s = batch_results(b, r, stats, ms * 1e-3);
  if (stats)
    for (int c = 0; c < b->n; ++c) stats[c].fp64_fallback = fell[c];
  delete[] r;
  return s;
}

ebit_status ebit_batch_mass_flux(ebit_batch* b, const double* const T[], double* const mdot[], ebit_stats stats[]) {
  ebit_status s = batch_ready(b);
  if (s != EBIT_OK) return s;
  if (!T || !mdot) return bfail(b, EBIT_EINVAL, -1, "NULL argument array");
  for (int c = 0; c < b->n; ++c)
    if (!T[c] || !mdot[c]) return bfail(b, EBIT_EINVAL, c, "NULL field");
  BHIPCK(b, hipEventRecord(b->ev0, b->st), "event");
  s = batch_scal(b, false);
  if (s != EBIT_OK) return s;
  {
    std::vector<FluxArgs> v(b->n);
    for (int c = 0; c < b->n; ++c) {
      ebit_ctx* x = b->ctx[c];
      const double lam[2] = {x->props.lam_v, x->props.lam_l};
      ebit_flux_args(&v[c], &x->fd, x->grid.h, lam, x->props.h_lg, x->props.T_sat, x->opts.theta_min, x->flags,
                     x->th, x->cF, x->nF, T[c], mdot[c], nullptr, x->B.scal);
    }
    BHIPCK(b, tab_put(b, b->t.flux, v.data(), v.size() * sizeof(FluxArgs)), "flux table");
    BHIPCK(b,
           ebit_launch_mass_flux_many(b->n, b->ctx[0]->fd.dim, (const FluxArgs*)b->t.flux.dev, b->t.cell_start,
                                      b->t.cell_blocks, b->st),
           "mass flux");
  }
  // without stats the call does not wait for the device
  if (!stats) return EBIT_OK;
  BHIPCK(b, hipEventRecord(b->ev1, b->st), "event");
  s = batch_read_scal(b);
  if (s != EBIT_OK) return s;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
  if (stats)
    for (int c = 0; c < b->n; ++c) {
      memset(&stats[c], 0, sizeof(stats[c]));
      stats[c].seconds = ms * 1e-3;
      stats[c].fallbacks = b->hsc[c].fallbacks;
    }
  return EBIT_OK;
}

ebit_status ebit_batch_project(ebit_batch* b, double* const u_l[], double* const u_v[], const double* const mdot[],
                               double* const p[], int use_guess, ebit_stats stats[]) {
  ebit_status s = batch_ready(b);
  if (s != EBIT_OK) return s;
  if (!u_l || !u_v || !mdot || !p) return bfail(b, EBIT_EINVAL, -1, "NULL argument array");
  for (int c = 0; c < b->n; ++c) {
    if (!mdot[c] || !p[c]) return bfail(b, EBIT_EINVAL, c, "NULL field");
    for (int a = 0; a < b->ctx[c]->grid.dim; ++a)
      if (!u_l[3 * c + a] || !u_v[3 * c + a]) return bfail(b, EBIT_EINVAL, c, "NULL velocity array");
  }
  BHIPCK(b, hipEventRecord(b->ev0, b->st), "event");
  {
    std::vector<ProjArgs> v(b->n);
    for (int c = 0; c < b->n; ++c) {
      ebit_ctx* x = b->ctx[c];
      const double rho[2] = {x->props.rho_v, x->props.rho_l};
      ebit_proj_args(&v[c], &x->fd, x->grid.h, rho, x->dt, x->grid.p_bc, x->grid.p_val, x->flags, x->th, x->nF,
                     mdot[c], u_l + 3 * c, u_v + 3 * c, nullptr, x->bvec, nullptr);
    }
    BHIPCK(b, tab_put(b, b->t.proj, v.data(), v.size() * sizeof(ProjArgs)), "projection table");
    BHIPCK(b,
           ebit_launch_proj_rhs_many(b->n, (const ProjArgs*)b->t.proj.dev, b->t.cell_start, b->t.cell_blocks, b->st),
           "projection rhs");
  }
  EbitSolveOut* r = new (std::nothrow) EbitSolveOut[b->n];
  if (!r) return EBIT_ENOMEM;
  hipError_t e = ebit_plan_solve(b->plan, EBIT_SYS_PRESSURE, p, use_guess, b->st, nullptr, r);
  std::vector<int> fell;
  if (e == hipSuccess) e = batch_fallback(b, EBIT_SYS_PRESSURE, p, r, fell);
  if (e != hipSuccess) {
    delete[] r;
    return bhip(b, e, "solve");
  }
  {
    std::vector<ProjArgs> v(b->n);
    std::vector<FinArgs> fv(b->n);
    for (int c = 0; c < b->n; ++c) {
      ebit_ctx* x = b->ctx[c];
      const double rho[2] = {x->props.rho_v, x->props.rho_l};
      ebit_proj_args(&v[c], &x->fd, x->grid.h, rho, x->dt, x->grid.p_bc, x->grid.p_val, x->flags, x->th, nullptr,
                     nullptr, u_l + 3 * c, u_v + 3 * c, p[c], nullptr, x->B.partial);
      const int cb = (int)blocks_of(x->fd.N);
      fv[c] = FinArgs{x->B.partial, cb < EBIT_RED_BLOCKS ? cb : EBIT_RED_BLOCKS, 1, FIN_MAX, x->B.scal};
    }
    hipError_t e2 = tab_put(b, b->t.projfu, v.data(), v.size() * sizeof(ProjArgs));
    if (e2 == hipSuccess) e2 = tab_put(b, b->t.fin, fv.data(), fv.size() * sizeof(FinArgs));
    if (e2 == hipSuccess)
      e2 = ebit_launch_face_update_many(b->n, (const ProjArgs*)b->t.projfu.dev, b->t.cell_start, b->t.cell_blocks,
                                        b->t.red_start, b->t.red_blocks, b->st);
    if (e2 == hipSuccess) e2 = ebit_launch_finalize_many(b->n, (const FinArgs*)b->t.fin.dev, b->t.unit_start, b->st);
    if (e2 != hipSuccess) {
      delete[] r;
      return bhip(b, e2, "face update");
    }
  }
  BHIPCK(b, hipEventRecord(b->ev1, b->st), "event");
  s = batch_read_scal(b);
  if (s != EBIT_OK) {
    delete[] r;
    return s;
  }
  float ms = 0;
  (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
  s = batch_results(b, r, stats, ms * 1e-3);
  if (stats)
    for (int c = 0; c < b->n; ++c) {
      stats[c].div_max = b->hsc[c].divmax;
      stats[c].fp64_fallback = fell[c];
    }
  delete[] r;
  return s;
}


/* ---- autotuning ------------------------------------------------------- */

}  // extern "C"

namespace {

// Candidate schedules: (nu1 = nu2) x tail_cells x check_every.
const int TUNE_NU[] = {1, 2, 3};
const int TUNE_TAIL[] = {256, 1024, 4096, 16384};
const int TUNE_K[] = {1, 2, 4};

// Re-plan a set of cases with new options (same plan memory).
hipError_t replan(EbitPlan** plan, ebit_ctx* const* ctx, int n, const ebit_opts* o, void* mem, size_t bytes) {
  ebit_plan_destroy(*plan);
  *plan = nullptr;
  EbitPlanCase* pc = new (std::nothrow) EbitPlanCase[n];
  if (!pc) return hipErrorOutOfMemory;
  for (int c = 0; c < n; ++c) pc[c] = EbitPlanCase{ctx[c]->lv, ctx[c]->nlev, ctx[c]->op, ctx[c]->B, ctx[c]->bvec};
  const hipError_t e = ebit_plan_create(plan, n, pc, o, ctx[0]->B.tail_lds, mem, bytes);
  delete[] pc;
  return e;
}

// Time every candidate on cold-start solves of the given right-hand sides
// (per case, per system; a null system is skipped) and keep the fastest one
// whose solves all converge.  The right-hand sides are copied into the
// contexts' own right-hand-side buffers.
hipError_t tune(EbitPlan** plan, ebit_ctx* const* ctx, int n, const ebit_opts& base, const double* const* bh,
                const double* const* bp, double* const* x, void* mem, size_t bytes, hipStream_t st, hipEvent_t ev0,
                hipEvent_t ev1, ebit_opts* best, double* best_ms) {
  hipError_t e;
  *best = base;
  *best_ms = INFINITY;
  EbitSolveOut* r = new (std::nothrow) EbitSolveOut[n];
  if (!r) return hipErrorOutOfMemory;
  for (int nu : TUNE_NU)
    for (int tail : TUNE_TAIL)
      for (int k : TUNE_K) {
        ebit_opts o = base;
        o.nu1 = o.nu2 = nu;
        o.tail_cells = tail;
        o.check_every = k;
        if ((e = replan(plan, ctx, n, &o, mem, bytes)) != hipSuccess) {
          delete[] r;
          return e;
        }
        double ms_tot = 0.0;
        bool ok = true;
        for (int sys = 0; sys < 2 && ok; ++sys) {
          const double* const* bs = sys == EBIT_SYS_HEAT ? bh : bp;
          if (!bs) continue;
          // the first run captures the graphs; the faster of the next two
          // counts (one timed run alone let a few percent of noise decide)
          double ms_sys = INFINITY;
          for (int rep = 0; rep < 3 && ok; ++rep) {
            for (int c = 0; c < n; ++c)
              if ((e = hipMemcpyAsync(ctx[c]->bvec, bs[c], ctx[c]->fd.N * sizeof(double), hipMemcpyDeviceToDevice,
                                      st)) != hipSuccess)
                break;
            if (e == hipSuccess) e = hipEventRecord(ev0, st);
            if (e == hipSuccess) e = ebit_plan_solve(*plan, sys, x, 0, st, nullptr, r);
            if (e == hipSuccess) e = hipEventRecord(ev1, st);
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
            if (e != hipSuccess) {
              delete[] r;
              return e;
            }
            for (int c = 0; c < n; ++c) ok = ok && r[c].status == 0;
            if (rep > 0 && ms < ms_sys) ms_sys = ms;
          }
          ms_tot += ms_sys;
        }
        if (ok && ms_tot < *best_ms) {
          *best_ms = ms_tot;
          *best = o;
        }
      }
  delete[] r;
  return replan(plan, ctx, n, best, mem, bytes);
}

}  // namespace

extern "C" {

ebit_status ebit_autotune(ebit_ctx* c, const double* b_heat, const double* b_press, double* x, ebit_opts* chosen,
                          double* best_ms) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!x || (!b_heat && !b_press)) return fail(c, EBIT_EINVAL, "need x and at least one right-hand side");
  ebit_opts best;
  double ms = 0;
  ebit_ctx* const cs[1] = {c};
  double* const xs[1] = {x};
  const double* const bh[1] = {b_heat};
  const double* const bp[1] = {b_press};
  const hipError_t e = tune(&c->plan, cs, 1, c->opts, b_heat ? bh : nullptr, b_press ? bp : nullptr, xs, c->plan_mem,
                            c->plan_bytes, c->st, c->ev0, c->ev1, &best, &ms);
  if (e != hipSuccess) return hip_fail(c, e, "autotune");
  c->opts = best;
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = ms;
  if (!isfinite(ms)) return fail(c, EBIT_ENOCONV, "no candidate schedule converged");
  return EBIT_OK;
}

ebit_status ebit_batch_autotune(ebit_batch* b, const double* const b_heat[], const double* const b_press[],
                                double* const x[], ebit_opts* chosen, double* best_ms) {
  ebit_status s = batch_ready(b);
  if (s != EBIT_OK) return s;
  if (!x || (!b_heat && !b_press)) return bfail(b, EBIT_EINVAL, -1, "need x and at least one right-hand side");
  ebit_opts best;
  double ms = 0;
  const hipError_t e =
      tune(&b->plan, b->ctx, b->n, b->opts, b_heat, b_press, x, b->ws, b->ws_bytes, b->st, b->ev0, b->ev1, &best, &ms);
  if (e != hipSuccess) return bhip(b, e, "autotune");
  b->opts = best;
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = ms;
  if (!isfinite(ms)) return bfail(b, EBIT_ENOCONV, -1, "no candidate schedule converged");
  return EBIT_OK;
}

/* ---- the tuned-schedule cache ------------------------------------------- */

}  // extern "C"

namespace {

// "dim n0 n1 n2 precision outer" of a grid under options o
std::string ctx_key(const ebit_grid* g, const ebit_opts* o) {
  char k[128];
  snprintf(k, sizeof(k), "%d %d %d %d %d %d", g->dim, g->n[0], g->n[1], g->n[2], o->precision, o->outer);
  return k;
}

std::string batch_key(const ebit_batch* b, const ebit_opts* o) {
  long long tot = 0, big = 0;
  for (int c = 0; c < b->n; ++c) {
    tot += b->ctx[c]->fd.N;
    big = std::max(big, b->ctx[c]->fd.N);
  }
  char k[160];
  snprintf(k, sizeof(k), "batch %d %d %lld %lld %d %d", b->ctx[0]->fd.dim, b->n, tot, big, o->precision, o->outer);
  return k;
}

// the last line of the file with this key: nu, tail, check, ms
bool cache_find(const char* path, const std::string& key, int* nu, int* tail, int* k, double* ms) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  bool hit = false;
  char line[512];
  const std::string head = "ebit-schedule " + key + " ";
  while (fgets(line, sizeof(line), f)) {
    if (strncmp(line, head.c_str(), head.size()) != 0) continue;
    int a, t, c;
    double m;
    if (sscanf(line + head.size(), "%d %d %d %lf", &a, &t, &c, &m) == 4 && a >= 1 && a <= 8 && t >= 1 && c >= 1) {
      *nu = a;
      *tail = t;
      *k = c;
      *ms = m;
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

bool cache_put(const char* path, const std::string& key, const ebit_opts* o, double ms) {
  FILE* f = fopen(path, "a");
  if (!f) return false;
  const int w = fprintf(f, "ebit-schedule %s %d %d %d %.6g\n", key.c_str(), o->nu1, o->tail_cells, o->check_every, ms);
  const int cl = fclose(f);
  return w > 0 && cl == 0;
}

void apply_schedule(ebit_opts* o, int nu, int tail, int k) {
  o->nu1 = o->nu2 = nu;
  o->tail_cells = tail;
  o->check_every = k;
}

}  // namespace

extern "C" {

ebit_status ebit_tune_lookup(const char* path, const ebit_grid* grid, const ebit_opts* base, ebit_opts* chosen,
                             int* found) {
  char msg[256];
  if (!path || !grid || !base || !chosen || !found) return EBIT_EINVAL;
  if (!valid_grid(grid, msg, sizeof(msg))) return EBIT_EINVAL;
  *chosen = *base;
  *found = 0;
  int nu, tail, k;
  double ms;
  if (cache_find(path, ctx_key(grid, base), &nu, &tail, &k, &ms)) {
    apply_schedule(chosen, nu, tail, k);
    *found = 1;
  }
  return EBIT_OK;
}

ebit_status ebit_tune_store(const char* path, const ebit_grid* grid, const ebit_opts* chosen, double ms) {
  char msg[256];
  if (!path || !grid || !chosen) return EBIT_EINVAL;
  if (!valid_grid(grid, msg, sizeof(msg))) return EBIT_EINVAL;
  return cache_put(path, ctx_key(grid, chosen), chosen, ms) ? EBIT_OK : EBIT_EIO;
}

ebit_status ebit_autotune_cached(ebit_ctx* c, const char* path, const double* b_heat, const double* b_press, double* x,
                                 ebit_opts* chosen, double* best_ms, int* from_cache) {
  ebit_status s = check_ready(c);
  if (s != EBIT_OK) return s;
  if (!path) return fail(c, EBIT_EINVAL, "NULL cache path");
  int nu, tail, k;
  double ms;
  if (cache_find(path, ctx_key(&c->grid, &c->opts), &nu, &tail, &k, &ms)) {
    ebit_opts o = c->opts;
    apply_schedule(&o, nu, tail, k);
    ebit_ctx* const cs[1] = {c};
    const hipError_t e = replan(&c->plan, cs, 1, &o, c->plan_mem, c->plan_bytes);
    if (e != hipSuccess) return hip_fail(c, e, "re-plan with the cached schedule");
    c->opts = o;
    if (chosen) *chosen = o;
    if (best_ms) *best_ms = ms;
    if (from_cache) *from_cache = 1;
    return EBIT_OK;
  }
  double m = 0;
  s = ebit_autotune(c, b_heat, b_press, x, chosen, &m);
  if (best_ms) *best_ms = m;
  if (from_cache) *from_cache = 0;
  if (s != EBIT_OK) return s;
  if (!cache_put(path, ctx_key(&c->grid, &c->opts), &c->opts, m)) return fail(c, EBIT_EIO, "cannot write the cache");
  return EBIT_OK;
}

ebit_status ebit_batch_autotune_cached(ebit_batch* b, const char* path, const double* const b_heat[],
                                       const double* const b_press[], double* const x[], ebit_opts* chosen,
                                       double* best_ms, int* from_cache) {
  ebit_status s = batch_ready(b);
  if (s != EBIT_OK) return s;
  if (!path) return bfail(b, EBIT_EINVAL, -1, "NULL cache path");
  int nu, tail, k;
  double ms;
  if (cache_find(path, batch_key(b, &b->opts), &nu, &tail, &k, &ms)) {
    ebit_opts o = b->opts;
    apply_schedule(&o, nu, tail, k);
    const hipError_t e = replan(&b->plan, b->ctx, b->n, &o, b->ws, b->ws_bytes);
    if (e != hipSuccess) return bhip(b, e, "re-plan with the cached schedule");
    b->opts = o;
    if (chosen) *chosen = o;
    if (best_ms) *best_ms = ms;
    if (from_cache) *from_cache = 1;
    return EBIT_OK;
  }
  double m = 0;
  s = ebit_batch_autotune(b, b_heat, b_press, x, chosen, &m);
  if (best_ms) *best_ms = m;
  if (from_cache) *from_cache = 0;
  if (s != EBIT_OK) return s;
  if (!cache_put(path, batch_key(b, &b->opts), &b->opts, m)) return bfail(b, EBIT_EIO, -1, "cannot write the cache");
  return EBIT_OK;
}

/* ---- the geometry pass without allocation --------------------------------
 * The facets and the status word of ebit_cut_fractions_noalloc live in one
 * file-scope device array.  Host code must not pass its name to a kernel:
 * in host code the name is a host-side stand-in.  The array's device
 * address is looked up once per device with hipGetSymbolAddress (on the
 * entry point's first call on that device, with the device current) and
 * only that address is used. */

}  // extern "C"

namespace {

constexpr size_t NOALLOC_STATUS_BYTES = 256;   // one Scal, rounded up to the array's alignment
constexpr size_t NOALLOC_BYTES = NOALLOC_STATUS_BYTES + (size_t)6 * EBIT_NOALLOC_MAX_CELLS * sizeof(double);
static_assert(sizeof(Scal) <= NOALLOC_STATUS_BYTES, "the status word must fit its slot");

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's copy of the scratch array (nullptr on failure).
hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

ebit_status ebit_cut_fractions_noalloc(const ebit_grid* grid, const double* const marker[3],
                                       const uint8_t* vertex_colour, const uint8_t* cell_colour,
                                       double* const theta[3], uint8_t* flags, void* hip_stream) {
  char msg[160];
  if (!valid_grid(grid, msg, sizeof msg)) return EBIT_EINVAL;
  if (!marker || !vertex_colour || !cell_colour || !theta || !flags) return EBIT_EINVAL;
  for (int a = 0; a < grid->dim; ++a)
    if (!marker[a] || !theta[a]) return EBIT_EINVAL;
  const Dims d = dims_of(grid);
  if (d.N > (long long)EBIT_NOALLOC_MAX_CELLS) return EBIT_EINVAL;
  void* base = nullptr;
  if (noalloc_scratch(&base) != hipSuccess) return EBIT_EHIP;
  hipStream_t st = (hipStream_t)hip_stream;
  Scal* scal = (Scal*)base;
  double* cF = (double*)((char*)base + NOALLOC_STATUS_BYTES);
  double* nF = cF + 3 * d.N;
  // the error bits are ORed in by the kernels: clear the status word first
  // (a fill kernel, not a memset node, so the call may be captured)
  if (ebit_launch_fill_f64((long long)(sizeof(Scal) / sizeof(double)), (double*)scal, 0.0, st) != hipSuccess)
    return EBIT_EHIP;
  if (ebit_launch_geometry(&d, grid->h, marker, vertex_colour, cell_colour, flags, cF, nF, theta, scal, st) !=
      hipSuccess)
    return EBIT_EHIP;
  int err = 0;
  if (hipMemcpyAsync(&err, &scal->err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return EBIT_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return EBIT_EHIP;
  if (err & (ERR_GEOM_MARKER | ERR_GEOM_SEAM | ERR_GEOM_NOFACET)) return EBIT_EGEOM;
  return EBIT_OK;
}

}  // extern "C"
