// EBIT markers -> interface facets -> cut fractions and cell flags (Sec. 2.1;
// theta of Eq. ghost_T; centroid and normal of Eq. normal_gradient).
//
// One thread per edge / vertex / cell; every pass reads its inputs once,
// coalesced along x.  The facet of an interface cell is its marker centroid
// and the unit normal from vapour into liquid (two-marker perpendicular in 2D,
// least-squares plane otherwise, via cyclic Jacobi on the 3x3 covariance).
#pragma clang fp contract(off)

#include "ebit_internal.h"

namespace ebit {

__host__ __device__ inline int nvz_of(const Dims& d) { return d.dim == 3 ? d.n[2] + 1 : 1; }

__device__ inline long long vidx(const Dims& d, int i, int j, int k) {
  return (long long)i + (long long)(d.n[0] + 1) * ((long long)j + (long long)(d.n[1] + 1) * k);
}

// edge (i,j,k) along axis a: vertex layout with one fewer entry along a
__device__ inline long long eidx(const Dims& d, int a, int i, int j, int k) {
  const int ex = d.n[0] + (a == 0 ? 0 : 1);
  const int ey = d.n[1] + (a == 1 ? 0 : 1);
  return (long long)i + (long long)ex * ((long long)j + (long long)ey * k);
}

// Marker present <=> end colours differ; s in [0, 1]; periodic seams agree.
template <bool B>
__global__ void k_check_markers(Many<GeoArgs> m, int a) {
  long long lb, nb;
  const GeoArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const int ex = d.n[0] + (a == 0 ? 0 : 1);
  const int ey = d.n[1] + (a == 1 ? 0 : 1);
  const int ez = (d.dim == 3) ? d.n[2] + (a == 2 ? 0 : 1) : 1;
  const long long t = lb * blockDim.x + threadIdx.x;
  if (t >= (long long)ex * ey * ez) return;
  const int i = (int)(t % ex);
  const int j = (int)((t / ex) % ey);
  const int k = (int)(t / ((long long)ex * ey));
  int q[3] = {i, j, k};
  const uint8_t c0 = g.vcol[vidx(d, i, j, k)];
  q[a] += 1;
  const uint8_t c1 = g.vcol[vidx(d, q[0], q[1], q[2])];
  const double s = g.mk[a][t];
  const bool has = !isnan(s);
  int bad = 0;
  if (has != (c0 != c1)) bad |= ERR_GEOM_MARKER;
  if (has && !(s >= 0.0 && s <= 1.0)) bad |= ERR_GEOM_MARKER;
  // periodic seam: an edge on the layer 0 of a periodic axis b != a equals its copy on layer n_b
  for (int b = 0; b < d.dim; ++b) {
    if (b == a || !d.per[b]) continue;
    int r[3] = {i, j, k};
    if (r[b] != 0) continue;
    r[b] = d.n[b];
    const double s2 = g.mk[a][eidx(d, a, r[0], r[1], r[2])];
    const bool same = (isnan(s) && isnan(s2)) || (s == s2);
    if (!same) bad |= ERR_GEOM_SEAM;
  }
  if (bad) atomicOr(&g.scal->err, bad);
}

template <bool B>
__global__ void k_check_seam_vertices(Many<GeoArgs> m) {
  long long lb, nb;
  const GeoArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const int vx = d.n[0] + 1, vy = d.n[1] + 1, vz = nvz_of(d);
  const long long t = lb * blockDim.x + threadIdx.x;
  if (t >= (long long)vx * vy * vz) return;
  const int i = (int)(t % vx);
  const int j = (int)((t / vx) % vy);
  const int k = (int)(t / ((long long)vx * vy));
  int q[3] = {i, j, k};
  for (int b = 0; b < d.dim; ++b) {
    if (!d.per[b] || q[b] != 0) continue;
    int r[3] = {i, j, k};
    r[b] = d.n[b];
    if (g.vcol[t] != g.vcol[vidx(d, r[0], r[1], r[2])]) atomicOr(&g.scal->err, (int)ERR_GEOM_SEAM);
  }
}

// Smallest-eigenvalue eigenvector of a symmetric M x M matrix (M = 2 or 3)
// by cyclic Jacobi rotations.
template <int M>
__device__ inline void min_eigvec(double A[3][3], double v[3]) {
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  bool polish = false;
  for (int sweep = 0; sweep < 32; ++sweep) {
    double offn = 0.0, tot = 0.0;
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
      for (int q = 0; q < M; ++q) {
        tot += A[p][q] * A[p][q];
        if (p != q) offn += A[p][q] * A[p][q];
      }
    // stop one sweep after the off-diagonal part reaches the matrix's
    // rounding level (its Frobenius norm times 4 ulps; the last sweep
    // polishes the eigenvectors): each rotation leaves a rounding residue of
    // about that size, so a test much tighter never passes and runs every
    // sweep
    if (polish) break;
    if (offn <= 7.888609052210118e-31 * tot) polish = true;
#pragma unroll
    for (int p = 0; p < M - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < M; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + tt * tt), s = tt * c;
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const double vrp = V[r][p], vrq = V[r][q];
          V[r][p] = c * vrp - s * vrq;
          V[r][q] = s * vrp + c * vrq;
        }
      }
  }
  int best = 0;
#pragma unroll
  for (int p = 1; p < M; ++p)
    if (A[p][p] < (best == 0 ? A[0][0] : A[1][1])) best = p;
#pragma unroll
  for (int r = 0; r < 3; ++r) v[r] = (r < M) ? (best == 0 ? V[r][0] : best == 1 ? V[r][1] : V[r][2]) : 0.0;
}

// Cell corner at which slot (a, o) of a cell's edge markers sits: the edge
// along axis a, offset by o & 1 along the first other axis and by o >> 1
// along the second (3D), in increasing axis order.
__device__ inline void slot_corner(int a, int o, int i, int j, int k, int dim, int& q0, int& q1, int& q2) {
  const int ob = o & 1, oc = o >> 1;
  q0 = i;
  q1 = j;
  q2 = k;
  if (a == 0) {
    q1 += ob;
    if (dim == 3) q2 += oc;
  } else if (a == 1) {
    q0 += ob;
    if (dim == 3) q2 += oc;
  } else {
    q0 += ob;
    q1 += oc;
  }
}

// Facet of every interface cell; writes flags = liquid bit | interface bit.
// The markers of the cell's edges are gathered into slot a * 4 + o (NaN: no
// marker, or no such slot) with every index known at compile time, so a
// cell without markers (almost all of them) finishes from registers.
template <bool B>
__global__ void k_facets(Many<GeoArgs> m) {
  long long lb, nb;
  const GeoArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  int i, j, k;
  cell_ijk(d, c, i, j, k);
  const uint8_t liq = g.ccol[c] ? F_LIQ : 0;
  {
    // corners of one colour: no edge of the cell carries a marker (markers
    // sit exactly on the edges whose end colours differ; the marker check
    // rejects inputs that break this), so the 12 marker loads are skipped
    const long long vx = d.n[0] + 1, vxy = vx * (d.n[1] + 1), v0 = vidx(d, i, j, k);
    const uint8_t c0 = g.vcol[v0];
    bool same = g.vcol[v0 + 1] == c0 && g.vcol[v0 + vx] == c0 && g.vcol[v0 + vx + 1] == c0;
    if (d.dim == 3)
      same = same && g.vcol[v0 + vxy] == c0 && g.vcol[v0 + vxy + 1] == c0 && g.vcol[v0 + vxy + vx] == c0 &&
             g.vcol[v0 + vxy + vx + 1] == c0;
    if (same) {
      g.flags[c] = liq;
      return;
    }
  }
  const double h = g.h;
  const int noff = (d.dim == 3) ? 4 : 2;
  double sv[12];
  int cnt = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      double s = __builtin_nan("");
      if (a < d.dim && o < noff) {
        int q0, q1, q2;
        slot_corner(a, o, i, j, k, d.dim, q0, q1, q2);
        s = g.mk[a][eidx(d, a, q0, q1, q2)];
      }
      sv[a * 4 + o] = s;
      cnt += isnan(s) ? 0 : 1;
    }
  const int need = (d.dim == 2) ? 2 : 3;
  if (cnt < need) {
    g.flags[c] = liq;
    return;
  }
  // marker points in slot order: centroid, and the first two (2D)
  double cen[3] = {0, 0, 0}, p0[3] = {0, 0, 0}, p1[3] = {0, 0, 0};
  double P[12][3];
  int seen = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const double s = sv[a * 4 + o];
      int q0, q1, q2;
      slot_corner(a, o, i, j, k, d.dim, q0, q1, q2);
      double pos[3] = {q0 * h, q1 * h, (d.dim == 3) ? q2 * h : 0.0};
      pos[a] = pos[a] + s * h;
#pragma unroll
      for (int r = 0; r < 3; ++r) P[a * 4 + o][r] = pos[r];
      if (!isnan(s)) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          cen[r] += pos[r];
          if (seen == 0) p0[r] = pos[r];
          if (seen == 1) p1[r] = pos[r];
        }
        ++seen;
      }
    }
  for (int r = 0; r < 3; ++r) cen[r] = cen[r] / (double)cnt;
  double n[3] = {0, 0, 0};
  bool ok = false;
  if (d.dim == 2 && cnt == 2) {
    const double dx = p1[0] - p0[0], dy = p1[1] - p0[1];
    const double L = hypot(dx, dy);
    if (L > 0) {
      n[0] = -dy / L;
      n[1] = dx / L;
      ok = true;
    }
  } else {
    double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      if (isnan(sv[q])) continue;
      double x[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) x[r] = P[q][r] - cen[r];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) C[r][s2] += x[r] * x[s2];
    }
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2) mx = fmax(mx, fabs(C[r][s2]));
    if (mx > 0) {
      if (d.dim == 3)
        min_eigvec<3>(C, n);
      else
        min_eigvec<2>(C, n);
      const double L = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int r = 0; r < 3; ++r) n[r] /= L;
      ok = true;
    }
  }
  // corners, in the order (dk, dj, di) (slots with dk = 1 unused in 2D)
  double gsum[3] = {0, 0, 0};
  double corner_pos[8][3];
  double corner_w[8];
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const int q = dk * 4 + dj * 2 + di;
        const bool use = dk == 0 || d.dim == 3;
        const double col = use ? (double)g.vcol[vidx(d, i + di, j + dj, k + dk)] : 0.0;
        corner_pos[q][0] = (i + di) * h;
        corner_pos[q][1] = (j + dj) * h;
        corner_pos[q][2] = (d.dim == 3) ? (k + dk) * h : 0.0;
        corner_w[q] = 2.0 * col - 1.0;
      }
  const int ncorner = d.dim == 3 ? 8 : 4;
  if (!ok) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= ncorner) continue;
#pragma unroll
      for (int r = 0; r < 3; ++r) gsum[r] += corner_w[q] * (corner_pos[q][r] - cen[r]);
    }
    const double L = sqrt(gsum[0] * gsum[0] + gsum[1] * gsum[1] + gsum[2] * gsum[2]);
    for (int r = 0; r < 3; ++r) n[r] = gsum[r] / L;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q >= ncorner) continue;
    const double dot = n[0] * (corner_pos[q][0] - cen[0]) + n[1] * (corner_pos[q][1] - cen[1]) +
                       n[2] * (corner_pos[q][2] - cen[2]);
    s += corner_w[q] * dot;
  }
  if (s == 0.0) {
    const double xc[3] = {(i + 0.5) * h, (j + 0.5) * h, (d.dim == 3) ? (k + 0.5) * h : 0.0};
    const double fc = (double)g.ccol[c];
    s = (2.0 * fc - 1.0) *
        (n[0] * (xc[0] - cen[0]) + n[1] * (xc[1] - cen[1]) + n[2] * (xc[2] - cen[2]));
  }
  if (s < 0.0)
    for (int r = 0; r < 3; ++r) n[r] = -n[r];
  for (int r = 0; r < 3; ++r) {
    g.cF[r * d.N + c] = cen[r];
    g.nF[r * d.N + c] = n[r];
  }
  g.flags[c] = liq | F_IF;
}

// theta of the link from lower cell (li,lj,lk) to upper cell (ui,uj,uk) along
// axis a, measured from the lower cell; wrap = the upper cell is across the
// periodic seam.  Returns false if neither cell carries a facet.
__device__ inline bool link_theta(const GeoArgs& g, int a, int li, int lj, int lk, int ui, int uj,
                                  int uk, bool wrap, double& theta) {
  const Dims& d = g.d;
  const double h = g.h;
  const long long lo = cell_index(d, li, lj, lk), hi = cell_index(d, ui, uj, uk);
  const double xc[3] = {(li + 0.5) * h, (lj + 0.5) * h, (d.dim == 3) ? (lk + 0.5) * h : 0.0};
  double tv[2];
  bool valid[2], exist[2];
  int nfacet = 0;
  for (int side = 0; side < 2; ++side) {
    const long long X = side ? hi : lo;
    valid[side] = exist[side] = false;
    if (!(g.flags[X] & F_IF)) continue;
    ++nfacet;
    double n[3], cen[3];
    for (int r = 0; r < 3; ++r) {
      n[r] = g.nF[r * d.N + X];
      cen[r] = g.cF[r * d.N + X];
    }
    if (fabs(n[a]) < 1e-12) continue;
    if (side == 1 && wrap) cen[a] += d.n[a] * h;
    const double dot = (cen[0] - xc[0]) * n[0] + (cen[1] - xc[1]) * n[1] + (cen[2] - xc[2]) * n[2];
    const double t = dot / (h * n[a]);
    tv[side] = t;
    exist[side] = true;
    valid[side] = side ? (t >= 0.5 && t <= 1.0) : (t >= 0.0 && t <= 0.5);
  }
  if (nfacet == 0) {
    theta = 0.5;
    return false;
  }
  if (valid[0] && valid[1])
    theta = 0.5 * (tv[0] + tv[1]);
  else if (valid[0])
    theta = tv[0];
  else if (valid[1])
    theta = tv[1];
  else if (exist[0] || exist[1]) {
    double sum = 0.0;
    int m = 0;
    for (int side = 0; side < 2; ++side)
      if (exist[side]) {
        sum += tv[side];
        ++m;
      }
    double t = sum / m;
    theta = fmin(fmax(t, 0.0), 1.0);
  } else {
    theta = 0.5;
  }
  return true;
}

// Cut bits of every side, and theta on the + faces (and face 0 of each axis).
template <bool B>
__global__ void k_theta_flags(Many<GeoArgs> m) {
  long long lb, nb;
  const GeoArgs& g = many_case<B>(m, lb, nb);
  const Dims& d = g.d;
  const long long c = lb * blockDim.x + threadIdx.x;
  if (c >= d.N) return;
  const int i = (int)(c % d.n[0]);
  const int j = (int)((c / d.n[0]) % d.n[1]);
  const int k = (int)(c / ((long long)d.n[0] * d.n[1]));
  uint8_t f = g.flags[c];
  const uint8_t myc = g.ccol[c];
  const double qnan = __builtin_nan("");
  for (int s = 0; s < 2 * d.dim; ++s) {
    int ni, nj, nk;
    const bool has = neighbour(d, i, j, k, s, ni, nj, nk);
    const int a = s >> 1, up = s & 1;
    const int ia = (a == 0) ? i : (a == 1) ? j : k;
    const bool cut = has && (g.ccol[cell_index(d, ni, nj, nk)] != myc);
    if (cut) f |= (uint8_t)(1u << s);
    // faces this cell writes: its + face, and face 0 when it is the first cell
    if (up || ia == 0) {
      double th = qnan;
      if (cut) {
        bool ok;
        if (up)
          ok = link_theta(g, a, i, j, k, ni, nj, nk, ia == d.n[a] - 1, th);
        else
          ok = link_theta(g, a, ni, nj, nk, i, j, k, true, th);
        if (!ok) atomicOr(&g.scal->err, (int)ERR_GEOM_NOFACET);
      }
      g.th[a][face_of_side(d, i, j, k, s)] = th;
    }
  }
  g.flags[c] = f;
}

}  // namespace ebit

using namespace ebit;

// host launcher used by the API layer
extern "C" hipError_t ebit_launch_geometry(const Dims* d, double h, const double* const mk[3],
                                           const uint8_t* vcol, const uint8_t* ccol, uint8_t* flags,
                                           double* cF, double* nF, double* const th[3], Scal* scal,
                                           hipStream_t st) {
  GeoArgs g;
  ebit_geo_args(&g, d, h, mk, vcol, ccol, flags, cF, nF, th, scal);
  const Many<GeoArgs> m = many_one(g);
  for (int a = 0; a < d->dim; ++a)
    hipLaunchKernelGGL(k_check_markers<false>, dim3((unsigned)ebit_geo_blocks(d, a)), dim3(EBIT_BLOCK), 0, st, m, a);
  hipLaunchKernelGGL(k_check_seam_vertices<false>, dim3((unsigned)ebit_geo_blocks(d, 3)), dim3(EBIT_BLOCK), 0, st, m);
  const unsigned nb = (unsigned)ebit_geo_blocks(d, 4);
  hipLaunchKernelGGL(k_facets<false>, dim3(nb), dim3(EBIT_BLOCK), 0, st, m);
  hipLaunchKernelGGL(k_theta_flags<false>, dim3(nb), dim3(EBIT_BLOCK), 0, st, m);
  return hipGetLastError();
}

extern "C" void ebit_geo_args(GeoArgs* g, const Dims* d, double h, const double* const mk[3], const uint8_t* vcol,
                              const uint8_t* ccol, uint8_t* flags, double* cF, double* nF, double* const th[3],
                              Scal* scal) {
  memset(g, 0, sizeof(*g));
  g->d = *d;
  g->h = h;
  for (int a = 0; a < 3; ++a) {
    g->mk[a] = (a < d->dim) ? mk[a] : nullptr;
    g->th[a] = (a < d->dim) ? th[a] : nullptr;
  }
  g->vcol = vcol;
  g->ccol = ccol;
  g->flags = flags;
  g->cF = cF;
  g->nF = nF;
  g->scal = scal;
}

// Blocks of the geometry pass's index spaces: the axis-a edges (kind a < 3),
// the vertices (3), the cells (4).
extern "C" long long ebit_geo_blocks(const Dims* d, int kind) {
  long long n;
  if (kind < 3)
    n = kind >= d->dim ? 0
                       : (long long)(d->n[0] + (kind == 0 ? 0 : 1)) * (d->n[1] + (kind == 1 ? 0 : 1)) *
                             ((d->dim == 3) ? d->n[2] + (kind == 2 ? 0 : 1) : 1);
  else if (kind == 3)
    n = (long long)(d->n[0] + 1) * (d->n[1] + 1) * nvz_of(*d);
  else
    n = d->N;
  return (n + EBIT_BLOCK - 1) / EBIT_BLOCK;
}

// The geometry pass of n cases in one launch per kernel: tab (device, n
// entries), start[kind] (device, n + 1 block offsets for each index space)
// and blocks[kind] (their totals).
extern "C" hipError_t ebit_launch_geometry_many(int n, int dim, const GeoArgs* tab, const int* const start[5],
                                                const int blocks[5], hipStream_t st) {
  for (int a = 0; a < dim; ++a)
    hipLaunchKernelGGL(k_check_markers<true>, dim3((unsigned)blocks[a]), dim3(EBIT_BLOCK), 0, st,
                       many_tab(tab, start[a], n), a);
  hipLaunchKernelGGL(k_check_seam_vertices<true>, dim3((unsigned)blocks[3]), dim3(EBIT_BLOCK), 0, st,
                     many_tab(tab, start[3], n));
  hipLaunchKernelGGL(k_facets<true>, dim3((unsigned)blocks[4]), dim3(EBIT_BLOCK), 0, st, many_tab(tab, start[4], n));
  hipLaunchKernelGGL(k_theta_flags<true>, dim3((unsigned)blocks[4]), dim3(EBIT_BLOCK), 0, st,
                     many_tab(tab, start[4], n));
  return hipGetLastError();
}
