// Internal definitions of the EBIT elliptic-path library (gfx950).
//
// Layout reminders (see include/ebit.h): cells x-fastest, c = i + nx*(j + ny*k);
// axis-a face arrays carry n_a + 1 entries along a; cell flags are one byte:
// bits 0..5 = cut link on side (-x,+x,-y,+y,-z,+z), bit 6 = liquid,
// bit 7 = interface cell.
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>
#include <stdint.h>

#include "ebit.h"

#define EBIT_BLOCK 256
#define EBIT_RED_BLOCKS 2048

namespace ebit {

enum : uint8_t { F_LIQ = 1u << 6, F_IF = 1u << 7, F_CUT = 0x3f };

// device-side error bits (Scal::err)
enum : int { ERR_GEOM_MARKER = 1, ERR_GEOM_NOFACET = 2, ERR_GEOM_SEAM = 4, ERR_NAN = 8 };

// Per-solve scalars kept on the device (no host round trip per iteration).
struct Scal {
  double bb, rr, gamma, delta, alpha, beta, zq, divmax;
  double sa[2], sg[2];  // alpha and gamma by iteration parity (read by one kernel while the next is written)
  double aa;      // || |b| + |A| |x| ||^2: sets the rounding floor of the residual
  double red[7];
  int err;
  int fallbacks;
  int iters;      // outer iterations taken (solves)
  int pad;
};

// Geometry of one grid level.
struct Dims {
  int dim;
  int n[3];
  int per[3];  // periodic axis flags
  long long N;
};

// Colour-split order of the 3D fine level: the cells of colour c
// ((i + j + k) & 1 == c) sit at slot (i >> 1) + hw (j + n1 k), hw = (n0 + 1) / 2,
// of the half c * H .. c * H + H - 1 of an array of 2 H entries, H = hw n1 n2.
// A red or black half-sweep then reads the other colour's half and writes
// its own, both contiguous.
__host__ __device__ inline long long split_half(const Dims& d) {
  return (long long)((d.n[0] + 1) / 2) * d.n[1] * d.n[2];
}
__host__ __device__ inline long long split_index(const Dims& d, long long H, int i, int j, int k) {
  return ((i + j + k) & 1) * H + (i >> 1) + (long long)((d.n[0] + 1) / 2) * (j + (long long)d.n[1] * k);
}

// Tail image: the coarse levels of at most EBIT_TAIL_IMG_CELLS cells keep,
// per system, their coefficients in one contiguous array, level after level
// from fine to coarse (fields diag, 1/diag, off[0 .. dim-1]), followed by
// the dense coarsest inverse; the tail kernel copies a suffix of it
// straight into LDS.  Within a field the cells of colour 0 ((i + j + k)
// even) come first, then those of colour 1, each half (hs elements, a
// multiple of four) in row order at slot (i >> 1) + hw (j + n1 k) with
// hw = (n0 + 1) / 2.
#define EBIT_TAIL_IMG_CELLS 8192
__host__ __device__ inline long long tail_pad(long long n) { return (n + 3) & ~3LL; }
__host__ __device__ inline long long tail_half(const Dims& d) {
  return tail_pad((long long)((d.n[0] + 1) / 2) * d.n[1] * d.n[2]);
}
__host__ __device__ inline long long tail_img_elems(const Dims& d) { return (2 + d.dim) * 2 * tail_half(d); }
__host__ __device__ inline long long tail_el(const Dims& d, long long hs, int i, int j, int k) {
  return ((i + j + k) & 1) * hs + (i >> 1) + (long long)((d.n[0] + 1) / 2) * (j + (long long)d.n[1] * k);
}

__host__ __device__ inline long long cell_index(const Dims& d, int i, int j, int k) {
  return (long long)i + (long long)d.n[0] * ((long long)j + (long long)d.n[1] * k);
}

// Face index of the face on side s of cell (i,j,k) in the axis-(s/2) face array.
__host__ __device__ inline long long face_of_side(const Dims& d, int i, int j, int k, int s) {
  const int a = s >> 1, up = s & 1;
  if (a == 0) return (long long)(i + up) + (long long)(d.n[0] + 1) * ((long long)j + (long long)d.n[1] * k);
  if (a == 1) return (long long)i + (long long)d.n[0] * ((long long)(j + up) + (long long)(d.n[1] + 1) * k);
  return (long long)i + (long long)d.n[0] * ((long long)j + (long long)d.n[1] * (k + up));
}

// Neighbour across side s; returns false at a non-periodic wall.
__host__ __device__ inline bool neighbour(const Dims& d, int i, int j, int k, int s, int& ni, int& nj,
                                          int& nk) {
  const int a = s >> 1;
  const int step = (s & 1) ? 1 : -1;
  int q[3] = {i, j, k};
  q[a] += step;
  if (q[a] < 0 || q[a] >= d.n[a]) {
    if (!d.per[a]) return false;
    q[a] = (q[a] + d.n[a]) % d.n[a];
  }
  ni = q[0];
  nj = q[1];
  nk = q[2];
  return true;
}

// Matrix-free description of a fine-level operator (heat or pressure).
struct FineOp {
  Dims d;
  double h, ih2;
  int sys;            // EBIT_SYS_HEAT / EBIT_SYS_PRESSURE
  double mass[2];     // heat: rho_k cp_k / dt per phase (index 0 vapour, 1 liquid); pressure: 0
  double coef[2];     // heat: lam_k; pressure: dt / rho_k
  double rho[2];
  double dt;
  double Tsat;
  int bc[6];
  double bcval[6];
  double theta_min;
  const uint8_t* flags;
  const double* th[3];
};

// One row of the fine operator at cell (i,j,k):  A x = diag x_c + sum_s off[s] x_nb(s).
// Heat (Eqs. energy_diffusion, Txx_ghost): diag = mass + sum of lam/h^2 weights with
// 1/theta' on cut links and 2 on Dirichlet walls; off = -lam/h^2 on same-phase links.
// Pressure (SPD form -L of Eq. Poisson_equation): off = -beta_f/h^2 with
// beta_f = dt/rho_f, rho_f the link property average on cut links; Dirichlet
// (outflow) walls add 2 beta/h^2 to the diagonal.  The boundary and interface
// terms of the right-hand side are added, side by side, to rhs_bc (heat:
// + lam T_sat/(theta' h^2) and + 2 lam T_w/h^2; pressure: + 2 beta p_w/h^2);
// the caller initialises rhs_bc.  mexc = diag + sum_s off[s] accumulated
// without cancellation (mass, interface and wall terms only): the row in
// difference form is  A x = mexc x_c + sum_s (-off[s]) (x_c - x_nb(s)).
// SYS >= 0 fixes the system at compile time (a kernel specialised per
// system carries only that system's terms); -1 reads it from op.
template <typename T, int SYS = -1>
__device__ inline void fine_row(const FineOp& op, int i, int j, int k, uint8_t f, T& diag, T off[6],
                                T& mass, T& rhs_bc, T* mexc = nullptr) {
  const int sys = SYS >= 0 ? SYS : op.sys;
  // per-phase values by selection, not by a run-time index, so a register
  // copy of the operator never needs a memory home
  const bool liq = (f & F_LIQ) != 0;
  const T ih2 = (T)op.ih2;
  const double coef = liq ? op.coef[1] : op.coef[0];
  const double rho_k = liq ? op.rho[1] : op.rho[0];
  const double rho_o = liq ? op.rho[0] : op.rho[1];
  mass = (T)(liq ? op.mass[1] : op.mass[0]);
  diag = mass;
  T mx = mass;
  const int ns = 2 * op.d.dim;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    off[s] = (T)0;
    if (s >= ns) continue;
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    const bool wall = !op.d.per[a] && (up ? (ia == op.d.n[a] - 1) : (ia == 0));
    if (sys == EBIT_SYS_HEAT) {
      const T lam = (T)coef;
      if (wall) {
        if (op.bc[s] == EBIT_BC_DIRICHLET) {
          diag += (T)2 * lam * ih2;
          mx += (T)2 * lam * ih2;
          rhs_bc += (T)2 * lam * (T)op.bcval[s] * ih2;
        }
      } else if ((f >> s) & 1) {
        const double tf = op.th[a][face_of_side(op.d, i, j, k, s)];
        double tc = up ? tf : 1.0 - tf;
        if (tc < op.theta_min) tc = op.theta_min;
        diag += lam * ih2 / (T)tc;
        mx += lam * ih2 / (T)tc;
        rhs_bc += lam * (T)op.Tsat * ih2 / (T)tc;
      } else {
        diag += lam * ih2;
        off[s] = -lam * ih2;
      }
    } else {
      if (wall) {
        if (op.bc[s] == EBIT_BC_DIRICHLET) {
          const T beta = (T)coef;
          diag += (T)2 * beta * ih2;
          mx += (T)2 * beta * ih2;
          rhs_bc += (T)2 * beta * (T)op.bcval[s] * ih2;
        }
      } else {
        T beta;
        if ((f >> s) & 1) {
          const double tf = op.th[a][face_of_side(op.d, i, j, k, s)];
          // lower cell of the link: this cell on a + side, the neighbour on a - side
          const double rlo = up ? rho_k : rho_o;
          const double rup = up ? rho_o : rho_k;
          const double rf = tf * rlo + (1.0 - tf) * rup;
          beta = (T)(op.dt / rf);
        } else {
          beta = (T)coef;
        }
        diag += beta * ih2;
        off[s] = -beta * ih2;
      }
    }
  }
  if (mexc) *mexc = mx;
}

// Explicit coarse level: symmetric 5/7-point operator, off[a][c] couples c and c + e_a.
template <typename T>
struct CoarseOp {
  Dims d;
  const T* diag;
  const T* off[3];
  const double* mass;  // used by the hierarchy builder only
};

__device__ inline void cell_ijk(const Dims& d, long long c, int& i, int& j, int& k) {
  if (c < 0x7fffffffLL) {
    // 32-bit division (a 64-bit one is a long emulated sequence)
    const unsigned u = (unsigned)c, n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
    const unsigned r = u / n0;
    i = (int)(u - r * n0);
    k = (int)(r / n1);
    j = (int)(r - (unsigned)k * n1);
    return;
  }
  i = (int)(c % d.n[0]);
  j = (int)((c / d.n[0]) % d.n[1]);
  k = (int)(c / ((long long)d.n[0] * d.n[1]));
}

// Tile (or first row block) taken by the lb-th of a case's nb blocks.  The
// chip hands work-groups to its 8 XCDs round-robin by global index, and each
// XCD has its own L2; the blocks of one XCD (equal lb mod 8, whatever the
// case's first global block) take a contiguous range of tiles, so the halo
// rows and planes that neighbouring tiles share are read once per XCD
// rather than once per tile.  A bijection of [0, nb) that depends on lb and
// nb alone, so a case maps the same way alone and in a batch.
__device__ inline int xcd_tile(int lb, int nb) {
  const int r = lb & 7, B = nb >> 3, R = nb & 7;
  return r * B + (r < R ? r : R) + (lb >> 3);
}

// ---------------------------------------------------------------------------
// Arguments of the per-case kernels outside the solves, and their launch over
// many cases: case e of a batch owns the blocks start[e] .. start[e+1]-1 of
// the grid (start[n] = the grid).  A single-case launch passes n = 0 and
// its arguments in `one`; a batch passes a device table of n entries.
// ---------------------------------------------------------------------------
template <typename A>
struct Many {
  A one;
  const A* tab;
  const int* start;
  int n;
};

// The block's case arguments, its block index within the case and the
// case's block count.  B is the kernel's compile-time choice between the
// two forms: a single case reads its arguments straight from the kernel
// argument, a batch from the device table, so no copy of the (large)
// argument struct is ever made in private memory.
template <bool B, typename A>
__device__ inline const A& many_case(const Many<A>& m, long long& lb, long long& nb) {
  if constexpr (!B) {
    lb = blockIdx.x;
    nb = gridDim.x;
    return m.one;
  } else {
    const int b = blockIdx.x;
    int lo = 0, hi = m.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (m.start[mid] <= b)
        lo = mid;
      else
        hi = mid - 1;
    }
    lb = b - m.start[lo];
    nb = m.start[lo + 1] - m.start[lo];
    return m.tab[lo];
  }
}

template <typename A>
inline Many<A> many_one(const A& a) {
  Many<A> m;
  m.one = a;
  m.tab = nullptr;
  m.start = nullptr;
  m.n = 0;
  return m;
}

template <typename A>
inline Many<A> many_tab(const A* tab, const int* start, int n) {
  Many<A> m;
  memset(&m.one, 0, sizeof(A));
  m.tab = tab;
  m.start = start;
  m.n = n;
  return m;
}

struct GeoArgs {
  Dims d;
  double h;
  const double* mk[3];
  const uint8_t* vcol;
  const uint8_t* ccol;
  uint8_t* flags;
  double* cF;  // [3][N]
  double* nF;  // [3][N]
  double* th[3];
  Scal* scal;
};

struct FluxArgs {
  Dims d;
  double h;
  double lam[2];  // [vapour, liquid]
  double h_lg, Tsat, theta_min;
  const uint8_t* flags;
  const double* th[3];
  const double* cF;  // [3][N]
  const double* nF;
  const double* T;
  double* mdot;
  double* mface[3];
  Scal* scal;
};

struct ProjArgs {
  Dims d;
  double h;
  double jump;  // [1/rho] = 1/rho_l - 1/rho_v
  double rho[2];
  double dt;
  int pbc[6];
  double pval[6];
  const uint8_t* flags;
  const double* th[3];
  const double* nF;
  const double* mdot;
  double* ul[3];
  double* uv[3];
  const double* p;
  double* b;
  double* partial;
  // one-fluid mode: the single field is ul; cF and the source factor
  // (1/rho_v - 1/rho_l) / h^d serve the interface cells' volume source
  int one;
  const double* cF;
  double src;
};

struct BuildOut {
  Dims cd;
  double* diag;
  double* mass;
  double* off[3];
  float* d32;     // FP32 copies of diag and off (null: none)
  float* o32[3];
  float* i32;     // the level's block of the FP32 or FP64 tail image (null: none)
  double* i64;
};

// heat right-hand side of one case
struct HeatRhsArgs {
  FineOp op;
  const double* Ts;
  double* b;
};

// finalize kinds
enum { FIN_INIT = 0, FIN_GAMMA = 1, FIN_DELTA = 2, FIN_RR = 3, FIN_MAX = 4, FIN_SUM1 = 5, FIN_START = 6, FIN_PEND = 7 };

// a single-block reduction of a case's partials into its status scalars
struct FinArgs {
  const double* partial;
  int nb, nv, kind;
  Scal* sc;
};

// one hierarchy level of both systems of a case: from the fine operator
// (level 1) or from the level above
struct BuildFineArgs {
  FineOp op[2];
  BuildOut o[2];
  unsigned nb;
};
struct BuildCoarseArgs {
  CoarseOp<double> op[2];
  BuildOut o[2];
  unsigned nb;
};
// the one-work-group part of a case's build: its two device tables
struct BuildSmallArgs {
  const void* tabs;
};
struct SplitArgs {
  Dims d;
  const uint8_t* flags;
  uint8_t* fs;
};
// a case's status scalars: cleared, or copied into a gathered array
struct ScalArgs {
  Scal* scal;
  Scal* dst;
};

// Neighbour of (i, j, k) at offsets (di, dj, dk): false beyond a wall,
// periodic axes wrap.
__device__ inline bool nbr_cell(const Dims& d, int i, int j, int k, int di, int dj, int dk, long long& m) {
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

// Sum of the facet normals (nF: 3 arrays of N) of the interface cells in
// the 3^d block of (i, j, k), the x offset slowest, z fastest (the band
// normal of Eq. extrapolation before normalisation); false if it vanishes.
__device__ inline bool band_normal_sum(const Dims& d, const uint8_t* flags, const double* nF, int i, int j, int k,
                                       double s[3]) {
  const int rz = d.dim == 3 ? 1 : 0;
  s[0] = s[1] = s[2] = 0.0;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj)
      for (int dk = -rz; dk <= rz; ++dk) {
        long long m;
        if (!nbr_cell(d, i, j, k, di, dj, dk, m)) continue;
        if (!((flags[m] >> 7) & 1)) continue;
        s[0] += nF[m];
        s[1] += nF[d.N + m];
        if (d.dim == 3) s[2] += nF[2 * d.N + m];
      }
  return sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) > 0.0;
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed grid, fixed order)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Block-wide sum of up to NV values per thread; result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* sh /* [NV * 4] */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q * 4 + w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = sh[q * 4 + 0] + sh[q * 4 + 1] + sh[q * 4 + 2] + sh[q * 4 + 3];
  }
}

}  // namespace ebit

// Host view of one multigrid level (level 0 = the matrix-free fine grid).
struct EbitLevelHost {
  ebit::Dims d;
  double* diag64[2];   // [system]
  double* mass64[2];
  double* off64[2][3];
  float* diag32[2];
  float* off32[2][3];
  double* x64;
  double* x64b;        // second iterate buffer (out-of-place fused sweeps)
  double* b64;
  float* x32;
  float* x32b;
  float* b32;
  // the first level of at most EBIT_DENSE_MAX cells also holds the inverse
  // of its operator per system (transposed, FP64 and FP32), used as the
  // exact coarsest solve, and a flag per system: 1 if the inversion
  // succeeded (null elsewhere)
  double* inv64[2];
  float* inv32[2];
  int* inv_ok;
  // this level's block of its system's tail image (FP32 and FP64; null
  // above EBIT_TAIL_IMG_CELLS cells)
  float* img32[2];
  double* img64[2];
};

#define EBIT_DENSE_MAX 64

// Optional per-kernel timing with hipEvents recorded around individual
// launches on the context's stream (kernel classes: ebit_kernel_class).
#define EBIT_PROF_CAP 1024
#define EBIT_PROF_CLASSES 8
struct EbitProfiler {
  int on;
  int npend;
  hipEvent_t ev0[EBIT_PROF_CAP];
  hipEvent_t ev1[EBIT_PROF_CAP];
  int kid[EBIT_PROF_CAP];
  int count[EBIT_PROF_CAP];  // launches inside each bracket
  long long launches[EBIT_PROF_CLASSES];
  double ms[EBIT_PROF_CLASSES];
};

// Work vectors of the outer loop (fine level).
struct EbitSolveBufs {
  double* r;
  float* r32;          // FP32 copy of r: the right-hand side the mixed-precision V-cycle reads
                       // (3D: in the colour-split order of the fine smoother)
  double* r64s;        // 3D, FP64 V-cycles: r in the colour-split order
  uint8_t* fsplit;     // 3D: the cell flags in the colour-split order
  double* z64;
  double* z64b;
  float* z32;
  float* z32b;
  double* p[2];
  double* q;
  double* partial;     // [2][EBIT_RED_BLOCKS]
  ebit::Scal* scal;
  EbitProfiler* prof;  // may be null
  int tail_lds;        // LDS bytes the coarse-tail kernel may take
};

extern "C" {
hipError_t ebit_launch_geometry(const ebit::Dims* d, double h, const double* const mk[3], const uint8_t* vcol,
                                const uint8_t* ccol, uint8_t* flags, double* cF, double* nF, double* const th[3],
                                ebit::Scal* scal, hipStream_t st);
hipError_t ebit_launch_fill_f64(long long n, double* x, double v, hipStream_t st);
hipError_t ebit_launch_split_flags(const ebit::Dims* d, const uint8_t* flags, uint8_t* fsplit, hipStream_t st);
// Narrow-band extension.  Scratch: bytes (2 N), list (N entries),
// w[0..dim-1] and ns[0..dim-1] (N doubles each), counter (one int); work (N
// doubles) holds every other iterate.
hipError_t ebit_launch_extend(const ebit::Dims* d, int mode, int iters, const uint8_t* flags, const double* nF,
                              double* q, double* work, uint8_t* bytes, unsigned long long* list,
                              double* const w[3], double* const ns[3], int* counter, hipStream_t st);
hipError_t ebit_launch_fill_f32(long long n, float* x, float v, hipStream_t st);
// Batched (many-case) forms of the per-case kernels: a device table of
// arguments and n + 1 block offsets (start) per launch.
void ebit_geo_args(ebit::GeoArgs* g, const ebit::Dims* d, double h, const double* const mk[3], const uint8_t* vcol,
                   const uint8_t* ccol, uint8_t* flags, double* cF, double* nF, double* const th[3],
                   ebit::Scal* scal);
long long ebit_geo_blocks(const ebit::Dims* d, int kind);
hipError_t ebit_launch_geometry_many(int n, int dim, const ebit::GeoArgs* tab, const int* const start[5],
                                     const int blocks[5], hipStream_t st);
void ebit_flux_args(ebit::FluxArgs* g, const ebit::Dims* d, double h, const double lam[2], double h_lg, double Tsat,
                    double theta_min, const uint8_t* flags, const double* const th[3], const double* cF,
                    const double* nF, const double* T, double* mdot, double* const mface[3], ebit::Scal* scal);
hipError_t ebit_launch_mass_flux_many(int n, int dim, const ebit::FluxArgs* tab, const int* start, int blocks,
                                      hipStream_t st);
void ebit_proj_args(ebit::ProjArgs* g, const ebit::Dims* d, double h, const double rho[2], double dt,
                    const int pbc[6], const double pval[6], const uint8_t* flags, const double* const th[3],
                    const double* nF, const double* mdot, double* const ul[3], double* const uv[3],
                    const double* p, double* b, double* partial);
hipError_t ebit_launch_proj_rhs_many(int n, const ebit::ProjArgs* tab, const int* start, int blocks,
                                     hipStream_t st);
hipError_t ebit_launch_face_update_many(int n, const ebit::ProjArgs* tab, const int* start, int blocks,
                                        const int* rstart, int rblocks, hipStream_t st);
int ebit_build_args(const ebit::FineOp* op, const EbitLevelHost* lv, int nlev, int want32, int ls,
                    ebit::BuildFineArgs* fine, ebit::BuildCoarseArgs* coarse);
hipError_t ebit_launch_build_fine_many(int n, const ebit::BuildFineArgs* tab, const int* start, int blocks,
                                       hipStream_t st);
hipError_t ebit_launch_build_coarse_many(int n, int dim, const ebit::BuildCoarseArgs* tab, const int* start,
                                         int blocks, hipStream_t st);
hipError_t ebit_launch_build_small_many(int n, int dim, const ebit::BuildSmallArgs* tab, const int* start,
                                        hipStream_t st);
hipError_t ebit_launch_heat_rhs_many(int n, const ebit::HeatRhsArgs* tab, const int* start, int blocks,
                                     hipStream_t st);
hipError_t ebit_launch_finalize_many(int n, const ebit::FinArgs* tab, const int* start, hipStream_t st);
hipError_t ebit_launch_scal_many(int n, const ebit::ScalArgs* tab, const int* start, hipStream_t st);
hipError_t ebit_launch_split_flags_many(int n, const ebit::SplitArgs* tab, const int* start, int blocks,
                                        hipStream_t st);
// Interfacial velocity at the cell centres (out[a], a < dim).
// Eq. energy_advection: T* of every cell from its own phase (energy.hip).
hipError_t ebit_launch_advect_energy(const ebit::Dims* d, double h, const double* T_liq, const double* T_vap,
                                     const double* const u_l[3], const double* const u_v[3], const uint8_t* ccol,
                                     double dt, double eps, double* out, hipStream_t st);
hipError_t ebit_launch_iface_velocity(const ebit::Dims* d, const uint8_t* flags, const double* nF,
                                      const double* const ul[3], const double* const uv[3], const double* mdot,
                                      double rho_l, double rho_v, double* const out[3], hipStream_t st);
// 2D marker motion (x pass, y pass, cell colours).  scratch:
// ebit_advect_scratch_bytes(d) bytes whose coordinate arrays hold NaN
// between calls (init != 0 sets them first); err: one int, cleared here.
size_t ebit_advect_scratch_bytes(const ebit::Dims* d);
hipError_t ebit_launch_advect(const ebit::Dims* d, double h, double dt, const double* const ug[3],
                              double* const mk[3], uint8_t* vcol, uint8_t* ccol, void* scratch, int init,
                              int* err, hipStream_t st);
// 2D liquid volume fraction of every cell from the markers and vertex
// colours; err: one int, cleared here, geometry bit set for a bad cell.
hipError_t ebit_launch_volume_fraction(const ebit::Dims* d, const double* const mk[3], const uint8_t* vcol,
                                       double* frac, int* err, hipStream_t st);
// Hierarchy builds: host tables of the one-work-group part (2 systems,
// ebit_build_table_bytes() bytes) are filled once and uploaded by the
// caller; ls is the first level that part builds.
void ebit_build_tables(const EbitLevelHost* lv, int nlev, int want32, void* host_tabs);
size_t ebit_build_table_bytes(void);
hipError_t ebit_build_hierarchy(const ebit::FineOp* op, EbitLevelHost* lv, int nlev, int want32, const void* dev_tabs,
                                int ls, hipStream_t st);
hipError_t ebit_launch_apply(const ebit::FineOp* op, const double* x, double* y, hipStream_t st);
hipError_t ebit_launch_heat_rhs(const ebit::FineOp* op, const double* Ts, double* b, hipStream_t st);
hipError_t ebit_launch_finalize_max(const double* partial, int nb, ebit::Scal* sc, hipStream_t st);
hipError_t ebit_launch_mass_flux(const ebit::Dims* d, double h, const double lam[2], double h_lg, double Tsat,
                                 double theta_min, const uint8_t* flags, const double* const th[3], const double* cF,
                                 const double* nF, const double* T, double* mdot, double* const mface[3],
                                 ebit::Scal* scal, hipStream_t st);
hipError_t ebit_launch_proj_rhs(const ebit::Dims* d, double h, const double rho[2], double dt, const int pbc[6],
                                const double pval[6], const uint8_t* flags, const double* const th[3],
                                const double* nF, const double* mdot, double* const ul[3], double* const uv[3],
                                double* b, hipStream_t st);
hipError_t ebit_launch_proj_rhs_one(const ebit::Dims* d, double h, const double rho[2], double dt,
                                   const int pbc[6], const double pval[6], const uint8_t* flags,
                                   const double* const th[3], const double* cF, const double* nF,
                                   const double* mdot, double* const u[3], double* b, hipStream_t st);
hipError_t ebit_launch_face_update_one(const ebit::Dims* d, double h, const double rho[2], double dt,
                                      const int pbc[6], const double pval[6], const uint8_t* flags,
                                      const double* const th[3], const double* cF, const double* nF,
                                      const double* mdot, double* const u[3], const double* p, double* partial,
                                      ebit::Scal* scal, hipStream_t st);
hipError_t ebit_launch_face_update(const ebit::Dims* d, double h, const double rho[2], double dt, const int pbc[6],
                                   const double pval[6], const uint8_t* flags, const double* const th[3],
                                   double* const ul[3], double* const uv[3], const double* p, double* partial,
                                   ebit::Scal* scal, hipStream_t st);
hipError_t ebit_prof_flush(EbitProfiler* pr);
int ebit_tail_lds_setup(void);
}

// One case as a solve plan sees it: its hierarchy, both fine operators
// (read at every solve, so rebuilt coefficients are picked up), its work
// vectors and the right-hand-side buffer the solves read.
struct EbitPlanCase {
  const EbitLevelHost* lv;
  int nlev;
  const ebit::FineOp* op;  // [2]: EBIT_SYS_HEAT, EBIT_SYS_PRESSURE
  EbitSolveBufs B;
  const double* b;
};

// Result of one case's solve: status 0 converged, 1 not converged
// (max_iters, or stagnation above the rounding floor), 2 NaN/Inf.
struct EbitSolveOut {
  int status;
  int stalled;  // status 1 because the inner cycle stopped contracting
  int iters;
  double rel_res, bnorm, res_floor;
};

// A solve plan: device tables and work lists of a batch of cases (carved
// from caller memory of ebit_plan_device_bytes()), the graphs of its
// iteration blocks and its own stream.
struct EbitPlan;
extern "C" {
size_t ebit_plan_device_bytes(int ncases, int precision);
hipError_t ebit_plan_create(EbitPlan** out, int ncases, const EbitPlanCase* cases, const ebit_opts* o, int tail_lds,
                            void* mem, size_t bytes);
void ebit_plan_destroy(EbitPlan* p);
hipError_t ebit_plan_solve(EbitPlan* p, int sys, double* const* x, int use_guess, hipStream_t ust, EbitProfiler* pf,
                           EbitSolveOut* out);
}
