// Mass flux from one-sided gradients (Eqs. mass_flux_computation,
// normal_gradient) with the one-layer FP64 ghost values of Eq. ghost_T, and
// the ghost-fluid projection around the Poisson solve (Eqs. ghost_velocity,
// poisson_ghost_fluid, face update).
//
// Sign reading: the facet normal points from vapour into liquid; the
// gradient into each phase is taken along +n (liquid) and -n (vapour), so
// mdot > 0 is evaporation, and the ghosts are u_liq^g = u_vap - mdot [1/rho] n,
// u_vap^g = u_liq + mdot [1/rho] n with [1/rho] = 1/rho_liq - 1/rho_vap.
//
// Everything here is FP64: the ghost extrapolation amplifies T by
// (1 - theta)/theta, which exceeds 19 for theta < 0.05.
#pragma clang fp contract(off)

#include "ebit_internal.h"
#include "ghost.h"

namespace ebit {

// T of phase k at cell (i,j,k) (periodic wrap), from the cell itself or its
// ghost value (mean of Eq. ghost_T over its cut links); false if unavailable.
template <int DIM>
__device__ inline bool value_k(const FluxArgs& g, int kph, int i, int j, int k, double& v) {
  const Dims& d = g.d;
  int q[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (q[a] < 0 || q[a] >= d.n[a]) {
      if (!d.per[a]) return false;
      q[a] = ((q[a] % d.n[a]) + d.n[a]) % d.n[a];
    }
  }
  const long long c = cell_index(d, q[0], q[1], q[2]);
  const uint8_t f = g.flags[c];
  const int ph = (f & F_LIQ) ? 1 : 0;
  if (ph == kph) {
    v = g.T[c];
    return true;
  }
  double acc = 0.0;
  int cnt = 0;
#pragma unroll
  for (int s = 0; s < 2 * DIM; ++s) {
    if (!((f >> s) & 1)) continue;
    int ni, nj, nk;
    neighbour(d, q[0], q[1], q[2], s, ni, nj, nk);
    const double tf = g.th[s >> 1][face_of_side(d, q[0], q[1], q[2], s)];
    const double th_g = (s & 1) ? tf : 1.0 - tf;  // from the ghost cell's centre
    double th_c = 1.0 - th_g;                     // from the phase-k cell's centre
    if (th_c < g.theta_min) th_c = g.theta_min;
    const double Tc = g.T[cell_index(d, ni, nj, nk)];
    acc += g.Tsat + (g.Tsat - Tc) * (1.0 - th_c) / th_c;
    ++cnt;
  }
  if (cnt == 0) return false;
  v = acc / (double)cnt;
  return true;
}

__device__ inline void lagrange3(double t, double w[3]) {
  w[0] = 0.5 * t * (t - 1.0);
  w[1] = (1.0 - t) * (1.0 + t);
  w[2] = 0.5 * t * (t + 1.0);
}

template <int DIM>
__device__ inline void clamp_block(const FluxArgs& g, int ctr[3]) {
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (!g.d.per[a]) ctr[a] = min(max(ctr[a], 1), g.d.n[a] - 2);
}

template <int DIM>
__device__ inline bool interp_block(const FluxArgs& g, int kph, const double P[3], const int ctr[3], double& out) {
  const double h = g.h;
  // Lagrange weights per axis as scalars (picked by selects below, so the
  // stencil loop indexes no local array)
  double w[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < DIM) {
      const double t = (P[a] - (ctr[a] + 0.5) * h) / h;
      lagrange3(t, w[a]);
    } else {
      w[a][0] = 0.0;
      w[a][1] = 1.0;
      w[a][2] = 0.0;
    }
  }
  double tot = 0.0;
  constexpr int kr = (DIM == 3) ? 1 : 0;
#pragma unroll 1
  for (int dk = -kr; dk <= kr; ++dk) {
    const double wz = dk < 0 ? w[2][0] : (dk == 0 ? w[2][1] : w[2][2]);
#pragma unroll 1
    for (int dj = -1; dj <= 1; ++dj) {
      const double wy = dj < 0 ? w[1][0] : (dj == 0 ? w[1][1] : w[1][2]);
#pragma unroll 1
      for (int di = -1; di <= 1; ++di) {
        const double wx = di < 0 ? w[0][0] : (di == 0 ? w[0][1] : w[0][2]);
        double v;
        if (!value_k<DIM>(g, kph, ctr[0] + di, ctr[1] + dj, ctr[2] + dk, v)) return false;
        tot += wx * wy * wz * v;
      }
    }
  }
  out = tot;
  return true;
}

template <int DIM>
__device__ inline bool point_value(const FluxArgs& g, int kph, const double P[3], const double sd[3], double& v) {
  int ctr[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) ctr[a] = (int)floor(P[a] / g.h);
  clamp_block<DIM>(g, ctr);
  if (interp_block<DIM>(g, kph, P, ctr, v)) return true;
  // step the block one cell along the dominant direction component
  int am = 0;
#pragma unroll
  for (int a = 1; a < DIM; ++a)
    if (fabs(sd[a]) > fabs(am == 0 ? sd[0] : sd[1])) am = a;
  const int step = (am == 0 ? sd[0] : am == 1 ? sd[1] : sd[2]) > 0 ? 1 : -1;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (a == am) ctr[a] += step;
  clamp_block<DIM>(g, ctr);
  return interp_block<DIM>(g, kph, P, ctr, v);
}

// first-order fallback from the nearest phase-k centre around P1
template <int DIM>
__device__ inline double fallback_grad(const FluxArgs& g, int kph, const double cF[3], const double sd[3],
                                       const double P1[3]) {
  const Dims& d = g.d;
  const double h = g.h;
  int ctr[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) ctr[a] = (int)floor(P1[a] / h);
  double best_d = 0.0, best_p = 0.0, best_T = 0.0;
  long long best_c = -1;
  constexpr int kr = (DIM == 3) ? 1 : 0;
#pragma unroll 1
  for (int dk = -kr; dk <= kr; ++dk)
#pragma unroll 1
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll 1
      for (int di = -1; di <= 1; ++di) {
        int q[3] = {ctr[0] + di, ctr[1] + dj, ctr[2] + dk};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (q[a] < 0 || q[a] >= d.n[a]) {
            if (d.per[a])
              q[a] = ((q[a] % d.n[a]) + d.n[a]) % d.n[a];
            else
              ok = false;
          }
        if (!ok) continue;
        const long long c = cell_index(d, q[0], q[1], q[2]);
        if (((g.flags[c] & F_LIQ) ? 1 : 0) != kph) continue;
        const double x[3] = {(ctr[0] + di + 0.5) * h, (ctr[1] + dj + 0.5) * h,
                             (d.dim == 3) ? (ctr[2] + dk + 0.5) * h : 0.0};
        const double proj = (x[0] - cF[0]) * sd[0] + (x[1] - cF[1]) * sd[1] + (x[2] - cF[2]) * sd[2];
        if (proj <= 0) continue;
        const double dist = (x[0] - P1[0]) * (x[0] - P1[0]) + (x[1] - P1[1]) * (x[1] - P1[1]) +
                            (x[2] - P1[2]) * (x[2] - P1[2]);
        if (best_c < 0 || dist < best_d || (dist == best_d && c < best_c)) {
          best_c = c;
          best_d = dist;
          best_p = proj;
          best_T = g.T[c];
        }
      }
  if (best_c < 0) return 0.0;
  return (best_T - g.Tsat) / best_p;
}

// The same per cell, with its four point values (two phases x two points
// along the normal) taken by four lanes of one wave: each lane walks one
// point's interpolation stencil, so the chain of dependent loads of an
// interface cell is a quarter as long, and the lanes of the non-interface
// cells of a wave are few (a wave holds 16 cells).  Lane 0 of the four
// combines them exactly as k_mass_flux does (the same arithmetic on the
// same values: the results are the same bits).
template <int DIM>
__global__ __launch_bounds__(EBIT_BLOCK) void k_mass_flux4(FluxArgs g) {
  const Dims& d = g.d;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long c = t >> 2;
  const int q = (int)(t & 3);
  if (c >= d.N) return;
  const uint8_t f = g.flags[c];
  if (!(f & F_IF)) {
    if (q == 0) g.mdot[c] = 0.0;
    return;
  }
  // lane q: phase kph = 1 - (q >> 1) (liquid first), point q & 1
  const int kph = (q >> 1) ? 0 : 1;
  const int pt = q & 1;
  const double h = g.h;
  double cF[3], nF[3];
  for (int r = 0; r < 3; ++r) {
    cF[r] = g.cF[r * d.N + c];
    nF[r] = g.nF[r * d.N + c];
  }
  const double d1 = h, d2 = 2.0 * h;
  const double sg = kph ? 1.0 : -1.0;
  double sd[3], P[3];
  for (int r = 0; r < 3; ++r) {
    sd[r] = sg * nF[r];
    P[r] = cF[r] + (pt ? d2 : d1) * sd[r];
  }
  double T = 0.0;
  const bool ok = point_value<DIM>(g, kph, P, sd, T);
  // the group's four values and flags to its lane 0 (the four lanes of a
  // cell are consecutive and all active here)
  const int base = (int)(threadIdx.x & 63) & ~3;
  double Tq[4];
  int okq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Tq[r] = __shfl(T, base + r, 64);
    okq[r] = __shfl(ok ? 1 : 0, base + r, 64);
  }
  if (q != 0) return;
  double D[2];
  int fb = 0;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int ph = kk == 0 ? 1 : 0;  // liquid first, as the oracle does
    const int r0 = kk * 2;
    if (okq[r0] && okq[r0 + 1]) {
      D[ph] = (d2 / d1 * (Tq[r0] - g.Tsat) - d1 / d2 * (Tq[r0 + 1] - g.Tsat)) / (d2 - d1);
    } else {
      ++fb;
      const double s2 = ph ? 1.0 : -1.0;
      double sd2[3], P1[3];
      for (int r = 0; r < 3; ++r) {
        sd2[r] = s2 * nF[r];
        P1[r] = cF[r] + d1 * sd2[r];
      }
      D[ph] = fallback_grad<DIM>(g, ph, cF, sd2, P1);
    }
  }
  g.mdot[c] = (g.lam[1] * D[1] + g.lam[0] * D[0]) / g.h_lg;
  if (fb) atomicAdd(&g.scal->fallbacks, fb);
}

template <int DIM, bool B>
__global__ void k_mass_flux(Many<FluxArgs> m) {
  long long lb, nb;
  const FluxArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  const uint8_t f = g.flags[c];
  if (!(f & F_IF)) {
    g.mdot[c] = 0.0;
    return;
  }
  const double h = g.h;
  double cF[3], nF[3];
  for (int r = 0; r < 3; ++r) {
    cF[r] = g.cF[r * d.N + c];
    nF[r] = g.nF[r * d.N + c];
  }
  const double d1 = h, d2 = 2.0 * h;
  double D[2];
  int fb = 0;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int kph = kk == 0 ? 1 : 0;  // liquid first, as the oracle does
    const double sg = kph ? 1.0 : -1.0;
    double sd[3], P1[3], P2[3];
    for (int r = 0; r < 3; ++r) {
      sd[r] = sg * nF[r];
      P1[r] = cF[r] + d1 * sd[r];
      P2[r] = cF[r] + d2 * sd[r];
    }
    double T1, T2;
    const bool ok1 = point_value<DIM>(g, kph, P1, sd, T1);
    const bool ok2 = ok1 && point_value<DIM>(g, kph, P2, sd, T2);
    if (ok1 && ok2) {
      D[kph] = (d2 / d1 * (T1 - g.Tsat) - d1 / d2 * (T2 - g.Tsat)) / (d2 - d1);
    } else {
      ++fb;
      D[kph] = fallback_grad<DIM>(g, kph, cF, sd, P1);
    }
  }
  g.mdot[c] = (g.lam[1] * D[1] + g.lam[0] * D[0]) / g.h_lg;
  if (fb) atomicAdd(&g.scal->fallbacks, fb);
}

// mdot on cut faces: value of the cell holding the crossing (theta <= 1/2 ->
// lower cell), the other one if that cell has no facet.  NaN elsewhere.
__global__ void k_mass_flux_faces(FluxArgs g) {
  const Dims& d = g.d;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const uint8_t f = g.flags[c];
  const double qnan = __builtin_nan("");
  for (int s = 0; s < 2 * d.dim; ++s) {
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    if (!(up || ia == 0)) continue;
    const long long fi = face_of_side(d, i, j, k, s);
    double v = qnan;
    if ((f >> s) & 1) {
      int ni, nj, nk;
      neighbour(d, i, j, k, s, ni, nj, nk);
      const long long nb = cell_index(d, ni, nj, nk);
      const long long lo = up ? c : nb, hi = up ? nb : c;
      const double t = g.th[a][fi];
      long long hold = (t <= 0.5) ? lo : hi;
      if (!(g.flags[hold] & F_IF)) hold = (hold == lo) ? hi : lo;
      v = g.mdot[hold];
    }
    g.mface[a][fi] = v;
  }
}

// ---------------------------------------------------------------------------
// projection
// ---------------------------------------------------------------------------
// Area (3D) or length (2D) of the facet plane of interface cell (i, j, k)
// clipped to the cell.  The plane meets the cell's edges (strict sign
// change of the signed distance) and corners (distance zero) in the
// clipped polygon's corners.  2D: the distance between the two extreme
// ones along the facet.  3D: the polygon's side on each face of the cell
// is the segment between that face's two points, oriented along n x F for
// the face's outward normal F (counter-clockwise about n); the area is half
// the sum of (a - c) x (b - c) . n over the sides.  A face lying in the
// plane contributes no side (its four edges are the neighbouring faces'
// sides).  Static indices only.
template <int DIM>
__device__ double facet_area(const Dims& d, double h, int i, int j, int k, const double* cF, const double* nF) {
  constexpr int NV = DIM == 3 ? 8 : 4;
  const long long cc = cell_index(d, i, j, k);
  double c[3], n[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    c[r] = (DIM == 3 || r < 2) ? cF[r * d.N + cc] : 0.0;
    n[r] = (DIM == 3 || r < 2) ? nF[r * d.N + cc] : 0.0;
  }
  double V[NV][3], s[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    V[q][0] = (i + (q & 1)) * h;
    V[q][1] = (j + ((q >> 1) & 1)) * h;
    V[q][2] = DIM == 3 ? (k + (q >> 2)) * h : 0.0;
    s[q] = (V[q][0] - c[0]) * n[0] + (V[q][1] - c[1]) * n[1] + (V[q][2] - c[2]) * n[2];
  }
  if (DIM == 2) {
    // the corners in cyclic order 0, 1, 3, 2 and the edges between them
    constexpr int cyc[4] = {0, 1, 3, 2};
    double tmin = 0.0, tmax = 0.0;
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int qa = cyc[m], qb = cyc[(m + 1) & 3];
      if (s[qa] == 0.0) {
        const double t = -(V[qa][0] - c[0]) * n[1] + (V[qa][1] - c[1]) * n[0];
        tmin = cnt ? fmin(tmin, t) : t;
        tmax = cnt ? fmax(tmax, t) : t;
        ++cnt;
      }
      if (s[qa] * s[qb] < 0.0) {
        const double w = s[qa] / (s[qa] - s[qb]);
        const double X = V[qa][0] + w * (V[qb][0] - V[qa][0]), Y = V[qa][1] + w * (V[qb][1] - V[qa][1]);
        const double tc = -(X - c[0]) * n[1] + (Y - c[1]) * n[0];
        tmin = cnt ? fmin(tmin, tc) : tc;
        tmax = cnt ? fmax(tmax, tc) : tc;
        ++cnt;
      }
    }
    return cnt >= 2 ? tmax - tmin : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
      int fq[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int bu = (m == 1 || m == 2) ? 1 : 0, bv = (m >= 2) ? 1 : 0;
        fq[m] = (sd << ax) | (bu << u) | (bv << v);
      }
      double A[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
      int cnt = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int qa = fq[m], qb = fq[(m + 1) & 3];
        if (s[qa] == 0.0) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            A[r] = cnt == 0 ? V[qa][r] : A[r];
            B[r] = cnt == 1 ? V[qa][r] : B[r];
          }
          ++cnt;
        }
        if (s[qa] * s[qb] < 0.0) {
          const double w = s[qa] / (s[qa] - s[qb]);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const double p = V[qa][r] + w * (V[qb][r] - V[qa][r]);
            A[r] = cnt == 0 ? p : A[r];
            B[r] = cnt == 1 ? p : B[r];
          }
          ++cnt;
        }
      }
      if (cnt != 2) continue;
      // direction n x F with F = +-e_ax
      double dv[3] = {0.0, 0.0, 0.0};
      const double F = sd ? 1.0 : -1.0;
      dv[(ax + 2) % 3] = n[(ax + 1) % 3] * F;
      dv[(ax + 1) % 3] = -n[(ax + 2) % 3] * F;
      const double along = (B[0] - A[0]) * dv[0] + (B[1] - A[1]) * dv[1] + (B[2] - A[2]) * dv[2];
      double a3[3], b3[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        a3[r] = (along < 0.0 ? B[r] : A[r]) - c[r];
        b3[r] = (along < 0.0 ? A[r] : B[r]) - c[r];
      }
      acc += (a3[1] * b3[2] - a3[2] * b3[1]) * n[0] + (a3[2] * b3[0] - a3[0] * b3[2]) * n[1] +
             (a3[0] * b3[1] - a3[1] * b3[0]) * n[2];
    }
  return 0.5 * fabs(acc);
}

// the one-fluid volume source of cell c (zero off the interface)
__device__ inline double one_fluid_source(const ProjArgs& g, int i, int j, int k, long long c) {
  if (!(g.flags[c] & F_IF)) return 0.0;
  const double A = g.d.dim == 3 ? facet_area<3>(g.d, g.h, i, j, k, g.cF, g.nF)
                                : facet_area<2>(g.d, g.h, i, j, k, g.cF, g.nF);
  return g.mdot[c] * A * g.src;
}

// Ghost value on every cut face (Eq. ghost_velocity, the rule of
// cut_face_ghost).  Each cell handles its + faces and, on the first layer,
// face 0 (the periodic copy of face n).
template <bool B>
__global__ void k_ghost_vel(Many<ProjArgs> m) {
  long long lb, nb;
  const ProjArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const uint8_t f = g.flags[c];
  for (int s = 0; s < 2 * d.dim; ++s) {
    if (!((f >> s) & 1)) continue;
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    if (!(up || ia == 0)) continue;
    int ni, nj, nk;
    neighbour(d, i, j, k, s, ni, nj, nk);
    const long long nb = cell_index(d, ni, nj, nk);
    const long long lo = up ? c : nb, hi = up ? nb : c;
    const long long fi = face_of_side(d, i, j, k, s);
    cut_face_ghost(d, g.flags, g.nF, g.mdot, g.jump, a, lo, hi, g.th[a][fi], fi, g.ul[a], g.uv[a]);
  }
}

// b = bc - div_c u_{k(c)}  (right-hand side of the SPD system -L p = b)
template <bool ONE, bool B>
__global__ void k_proj_rhs(Many<ProjArgs> m) {
  long long lb, nb;
  const ProjArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const uint8_t f = g.flags[c];
  const int ph = (f & F_LIQ) ? 1 : 0;
  double div = 0.0;
  for (int a = 0; a < d.dim; ++a) {
    const double* u = (ph || ONE) ? g.ul[a] : g.uv[a];
    div += u[face_of_side(d, i, j, k, 2 * a + 1)] - u[face_of_side(d, i, j, k, 2 * a)];
  }
  div = div / g.h;
  // one-fluid: div u = S_pc in the interface cells
  if constexpr (ONE) div -= one_fluid_source(g, i, j, k, c);
  double bc = 0.0;
  const double ih2 = 1.0 / (g.h * g.h);
  for (int s = 0; s < 2 * d.dim; ++s) {
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    const bool wall = !d.per[a] && (up ? (ia == d.n[a] - 1) : (ia == 0));
    if (wall && g.pbc[s] == EBIT_BC_DIRICHLET) bc += 2.0 * (g.dt / g.rho[ph]) * g.pval[s] * ih2;
  }
  g.b[c] = bc - div;
}

// beta_f and the gradient across side s of cell (i,j,k); false if no update
__device__ inline bool face_grad(const ProjArgs& g, int i, int j, int k, long long c, int s, double& beta,
                                 double& grad) {
  const Dims& d = g.d;
  const int a = s >> 1, up = s & 1;
  const int ia = (a == 0) ? i : (a == 1) ? j : k;
  const uint8_t f = g.flags[c];
  const int ph = (f & F_LIQ) ? 1 : 0;
  const bool wall = !d.per[a] && (up ? (ia == d.n[a] - 1) : (ia == 0));
  const double pc = g.p[c];
  if (wall) {
    if (g.pbc[s] != EBIT_BC_DIRICHLET) return false;
    beta = g.dt / g.rho[ph];
    grad = up ? 2.0 * (g.pval[s] - pc) / g.h : 2.0 * (pc - g.pval[s]) / g.h;
    return true;
  }
  int ni, nj, nk;
  neighbour(d, i, j, k, s, ni, nj, nk);
  const long long nb = cell_index(d, ni, nj, nk);
  if ((f >> s) & 1) {
    const double tf = g.th[a][face_of_side(d, i, j, k, s)];
    const double rlo = up ? g.rho[ph] : g.rho[1 - ph];
    const double rup = up ? g.rho[1 - ph] : g.rho[ph];
    beta = g.dt / (tf * rlo + (1.0 - tf) * rup);
  } else {
    beta = g.dt / g.rho[ph];
  }
  grad = up ? (g.p[nb] - pc) / g.h : (pc - g.p[nb]) / g.h;
  return true;
}

// u <- u - beta_f grad p on both fields; each cell writes its + faces and, on
// the first layer, face 0 (so every face is written exactly once).
template <bool B>
__global__ void k_face_update(Many<ProjArgs> m) {
  long long lb, nb;
  const ProjArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  for (int s = 0; s < 2 * d.dim; ++s) {
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    if (!(up || ia == 0)) continue;
    double beta, grad;
    if (!face_grad(g, i, j, k, c, s, beta, grad)) continue;
    const long long fi = face_of_side(d, i, j, k, s);
    const double dl = beta * grad;
    g.ul[a][fi] = g.ul[a][fi] - dl;
    if (!g.one) g.uv[a][fi] = g.uv[a][fi] - dl;
  }
}

// max_c |div_c u_{k(c)}| of the updated fields (a separate pass: every face
// is final when it is read)
template <bool ONE, bool B>
__global__ void k_divmax(Many<ProjArgs> m) {
  long long lb, nb;
  const ProjArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  double vmax = 0.0;
  for (long long c = lb * blockDim.x + threadIdx.x; c < d.N; c += nb * blockDim.x) {
    int i, j, k;
    cell_ijk(d, c, i, j, k);
    const int ph = (g.flags[c] & F_LIQ) ? 1 : 0;
    double div = 0.0;
    for (int a = 0; a < d.dim; ++a) {
      const double* u = (ph || ONE) ? g.ul[a] : g.uv[a];
      div += u[face_of_side(d, i, j, k, 2 * a + 1)] - u[face_of_side(d, i, j, k, 2 * a)];
    }
    div = div / g.h;
    if constexpr (ONE) div -= one_fluid_source(g, i, j, k, c);
    vmax = fmax(vmax, fabs(div));
  }
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double wm = wave_max(vmax);
  if (lane == 0) sh[w] = wm;
  __syncthreads();
  if (threadIdx.x == 0) g.partial[lb] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

static inline unsigned nblk(long long n) { return (unsigned)((n + EBIT_BLOCK - 1) / EBIT_BLOCK); }

}  // namespace ebit

using namespace ebit;

extern "C" void ebit_flux_args(FluxArgs* g, const Dims* d, double h, const double lam[2], double h_lg, double Tsat,
                               double theta_min, const uint8_t* flags, const double* const th[3], const double* cF,
                               const double* nF, const double* T, double* mdot, double* const mface[3], Scal* scal) {
  memset(g, 0, sizeof(*g));
  g->d = *d;
  g->h = h;
  g->lam[0] = lam[0];
  g->lam[1] = lam[1];
  g->h_lg = h_lg;
  g->Tsat = Tsat;
  g->theta_min = theta_min;
  g->flags = flags;
  for (int a = 0; a < 3; ++a) {
    g->th[a] = (a < d->dim) ? th[a] : nullptr;
    g->mface[a] = (mface && a < d->dim) ? mface[a] : nullptr;
  }
  g->cF = cF;
  g->nF = nF;
  g->T = T;
  g->mdot = mdot;
  g->scal = scal;
}

extern "C" hipError_t ebit_launch_mass_flux(const Dims* d, double h, const double lam[2], double h_lg, double Tsat,
                                            double theta_min, const uint8_t* flags, const double* const th[3],
                                            const double* cF, const double* nF, const double* T, double* mdot,
                                            double* const mface[3], Scal* scal, hipStream_t st) {
  FluxArgs g;
  ebit_flux_args(&g, d, h, lam, h_lg, Tsat, theta_min, flags, th, cF, nF, T, mdot, mface, scal);
  if (d->dim == 3)
    hipLaunchKernelGGL(k_mass_flux4<3>, dim3(nblk(4 * d->N)), dim3(EBIT_BLOCK), 0, st, g);
  else
    hipLaunchKernelGGL((k_mass_flux<2, false>), dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  if (mface) hipLaunchKernelGGL(k_mass_flux_faces, dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, g);
  return hipGetLastError();
}

// n cases' mass fluxes in one launch: start (n + 1 block offsets, one block
// per EBIT_BLOCK cells of each case), blocks = start[n]
extern "C" hipError_t ebit_launch_mass_flux_many(int n, int dim, const FluxArgs* tab, const int* start, int blocks,
                                                 hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL((k_mass_flux<3, true>), dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  else
    hipLaunchKernelGGL((k_mass_flux<2, true>), dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}

extern "C" void ebit_proj_args(ProjArgs* g, const Dims* d, double h, const double rho[2], double dt,
                               const int pbc[6], const double pval[6], const uint8_t* flags,
                               const double* const th[3], const double* nF, const double* mdot, double* const ul[3],
                               double* const uv[3], const double* p, double* b, double* partial) {
  memset(g, 0, sizeof(*g));
  g->d = *d;
  g->h = h;
  g->rho[0] = rho[0];
  g->rho[1] = rho[1];
  g->jump = 1.0 / rho[1] - 1.0 / rho[0];
  g->dt = dt;
  for (int s = 0; s < 6; ++s) {
    g->pbc[s] = pbc[s];
    g->pval[s] = pval[s];
  }
  g->flags = flags;
  for (int a = 0; a < 3; ++a) {
    g->th[a] = (a < d->dim) ? th[a] : nullptr;
    g->ul[a] = (a < d->dim && ul) ? ul[a] : nullptr;
    g->uv[a] = (a < d->dim && uv) ? uv[a] : nullptr;
  }
  g->nF = nF;
  g->mdot = mdot;
  g->p = p;
  g->b = b;
  g->partial = partial;
  g->one = 0;
  g->cF = nullptr;
  g->src = 0.0;
}

static ProjArgs make_proj(const Dims* d, double h, const double rho[2], double dt, const int pbc[6],
                          const double pval[6], const uint8_t* flags, const double* const th[3], const double* nF,
                          const double* mdot, double* const ul[3], double* const uv[3], const double* p, double* b,
                          double* partial) {
  ProjArgs g;
  ebit_proj_args(&g, d, h, rho, dt, pbc, pval, flags, th, nF, mdot, ul, uv, p, b, partial);
  return g;
}

extern "C" hipError_t ebit_launch_proj_rhs(const Dims* d, double h, const double rho[2], double dt, const int pbc[6],
                                           const double pval[6], const uint8_t* flags, const double* const th[3],
                                           const double* nF, const double* mdot, double* const ul[3],
                                           double* const uv[3], double* b, hipStream_t st) {
  ProjArgs g = make_proj(d, h, rho, dt, pbc, pval, flags, th, nF, mdot, ul, uv, nullptr, b, nullptr);
  hipLaunchKernelGGL(k_ghost_vel<false>, dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  hipLaunchKernelGGL((k_proj_rhs<false, false>), dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  return hipGetLastError();
}

// n cases' ghost velocities and right-hand sides, one launch each
extern "C" hipError_t ebit_launch_proj_rhs_many(int n, const ProjArgs* tab, const int* start, int blocks,
                                                hipStream_t st) {
  hipLaunchKernelGGL(k_ghost_vel<true>, dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  hipLaunchKernelGGL((k_proj_rhs<false, true>), dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  return hipGetLastError();
}

// One-fluid mode: the right-hand side from the single field u and the
// interface cells' volume source; the face update of u alone and the largest
// |div u - S_pc| after it.
extern "C" hipError_t ebit_launch_proj_rhs_one(const Dims* d, double h, const double rho[2], double dt,
                                               const int pbc[6], const double pval[6], const uint8_t* flags,
                                               const double* const th[3], const double* cF, const double* nF,
                                               const double* mdot, double* const u[3], double* b, hipStream_t st) {
  ProjArgs g = make_proj(d, h, rho, dt, pbc, pval, flags, th, nF, mdot, u, u, nullptr, b, nullptr);
  g.one = 1;
  g.cF = cF;
  g.src = (1.0 / rho[0] - 1.0 / rho[1]) / (d->dim == 3 ? h * h * h : h * h);
  hipLaunchKernelGGL((k_proj_rhs<true, false>), dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  return hipGetLastError();
}

extern "C" hipError_t ebit_launch_face_update_one(const Dims* d, double h, const double rho[2], double dt,
                                                  const int pbc[6], const double pval[6], const uint8_t* flags,
                                                  const double* const th[3], const double* cF, const double* nF,
                                                  const double* mdot, double* const u[3], const double* p,
                                                  double* partial, Scal* scal, hipStream_t st) {
  ProjArgs g = make_proj(d, h, rho, dt, pbc, pval, flags, th, nF, mdot, u, u, p, nullptr, partial);
  g.one = 1;
  g.cF = cF;
  g.src = (1.0 / rho[0] - 1.0 / rho[1]) / (d->dim == 3 ? h * h * h : h * h);
  hipLaunchKernelGGL(k_face_update<false>, dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  hipLaunchKernelGGL((k_divmax<true, false>), dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, many_one(g));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return ebit_launch_finalize_max(partial, EBIT_RED_BLOCKS, scal, st);
}

extern "C" hipError_t ebit_launch_face_update(const Dims* d, double h, const double rho[2], double dt,
                                              const int pbc[6], const double pval[6], const uint8_t* flags,
                                              const double* const th[3], double* const ul[3], double* const uv[3],
                                              const double* p, double* partial, Scal* scal, hipStream_t st) {
  ProjArgs g = make_proj(d, h, rho, dt, pbc, pval, flags, th, nullptr, nullptr, ul, uv, p, nullptr, partial);
  hipLaunchKernelGGL(k_face_update<false>, dim3(nblk(d->N)), dim3(EBIT_BLOCK), 0, st, many_one(g));
  hipLaunchKernelGGL((k_divmax<false, false>), dim3(EBIT_RED_BLOCKS), dim3(EBIT_BLOCK), 0, st, many_one(g));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return ebit_launch_finalize_max(partial, EBIT_RED_BLOCKS, scal, st);
}

// n cases' face updates (start: one block per EBIT_BLOCK cells) and
// divergence maxima (rstart: each case's reduction blocks, as many as its
// finalize entry reduces), one launch each
extern "C" hipError_t ebit_launch_face_update_many(int n, const ProjArgs* tab, const int* start, int blocks,
                                                   const int* rstart, int rblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_face_update<true>, dim3((unsigned)blocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start, n));
  hipLaunchKernelGGL((k_divmax<false, true>), dim3((unsigned)rblocks), dim3(EBIT_BLOCK), 0, st, many_tab(tab, rstart, n));
  return hipGetLastError();
}
