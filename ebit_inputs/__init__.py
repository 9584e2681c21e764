"""Seeded synthetic inputs for the EBIT phase-change elliptic path.

This module produces *data only*: a uniform Cartesian grid, EBIT edge markers
placed at the exact crossings of an analytic level set (one marker per cell
edge at most, as the EBIT method stores them), the colour-vertex colours
(1 = liquid, 0 = vapour), the initial temperature and the face velocities.
It holds none of the method's arithmetic (no cut fractions, no operators, no
fluxes), so both the plain CPU oracle and the HIP path may consume it.

Array conventions (numpy, C order, x fastest; a 2D grid has nz = 1):
  cells            [nz][ny][nx]
  vertices         [nvz][ny+1][nx+1]        nvz = nz+1 in 3D, 1 in 2D
  x-edges          [nvz][ny+1][nx]          edge from vertex (i,j,k) to (i+1,j,k)
  y-edges          [nvz][ny][nx+1]
  z-edges (3D)     [nz][ny+1][nx+1]
  axis-a faces     cell shape with n_a + 1 entries along a
A marker is the fractional position s in [0, 1] of the crossing along its edge,
measured from the edge's lower vertex; NaN means "no marker on this edge".
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

NEUMANN, DIRICHLET, PERIODIC = 0, 1, 2


@dataclasses.dataclass
class Props:
    rho_l: float = 1.0
    rho_v: float = 1e-3
    lam_l: float = 1.0
    lam_v: float = 0.1
    cp_l: float = 1.0
    cp_v: float = 1.0
    h_lg: float = 1000.0
    T_sat: float = 0.0


@dataclasses.dataclass
class Case:
    """One synthetic problem instance (all arrays are float64 / uint8 numpy)."""
    name: str
    dim: int
    n: Tuple[int, int, int]          # cells per axis (nz = 1 in 2D)
    h: float
    props: Props
    dt: float
    # boundary conditions per domain side, order (-x, +x, -y, +y, -z, +z):
    T_bc: List[Tuple[int, float]]
    p_bc: List[Tuple[int, float]]
    markers: List[np.ndarray]        # dim edge arrays
    vcol: np.ndarray                 # vertex colours, uint8
    ccol: np.ndarray                 # cell colours, uint8
    T0: np.ndarray                   # initial temperature per cell
    u_l: List[np.ndarray]            # dim face arrays
    u_v: List[np.ndarray]

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


# ----------------------------------------------------------------------------
# shapes
# ----------------------------------------------------------------------------

def cell_shape(dim, n):
    nx, ny, nz = n
    return (nz if dim == 3 else 1, ny, nx)


def vertex_shape(dim, n):
    nx, ny, nz = n
    return (nz + 1 if dim == 3 else 1, ny + 1, nx + 1)


def edge_shape(dim, n, a):
    nvz, nvy, nvx = vertex_shape(dim, n)
    s = [nvz, nvy, nvx]
    s[2 - a] -= 1
    return tuple(s)


def face_shape(dim, n, a):
    s = list(cell_shape(dim, n))
    s[2 - a] += 1
    return tuple(s)


def _vertex_coords(dim, n, h):
    nvz, nvy, nvx = vertex_shape(dim, n)
    z, y, x = np.meshgrid(np.arange(nvz) * h, np.arange(nvy) * h, np.arange(nvx) * h, indexing="ij")
    if dim == 2:
        z = np.zeros_like(z)
    return x, y, z


def _cell_coords(dim, n, h):
    nz, ny, nx = cell_shape(dim, n)
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    if dim == 2:
        z = np.zeros_like(z)
    return x, y, z


class LevelSet:
    """phi > 0 (or = 0) is liquid.  ``root`` returns the crossing of an edge."""

    def phi(self, x, y, z):  # pragma: no cover - interface
        raise NotImplementedError

    def root(self, a, x0, y0, z0, h, start_liquid):  # pragma: no cover
        raise NotImplementedError


class Plane(LevelSet):
    """phi = m . (x - p): liquid on the side m points to."""

    def __init__(self, m, p):
        self.m = np.asarray(m, float)
        self.p = np.asarray(p, float)

    def phi(self, x, y, z):
        return self.m[0] * (x - self.p[0]) + self.m[1] * (y - self.p[1]) + self.m[2] * (z - self.p[2])

    def root(self, a, x0, y0, z0, h, start_liquid):
        f0 = self.phi(x0, y0, z0)
        return -f0 / (self.m[a] * h)


class Ball(LevelSet):
    """Circle (2D, z ignored) or sphere; sign=+1: vapour bubble (liquid outside)."""

    def __init__(self, c, R, sign=+1.0, dim=3):
        self.c = np.asarray(c, float)
        self.R = float(R)
        self.sign = float(sign)
        self.dim = dim

    def _r(self, x, y, z):
        dz = (z - self.c[2]) if self.dim == 3 else 0.0
        return np.sqrt((x - self.c[0]) ** 2 + (y - self.c[1]) ** 2 + dz ** 2)

    def phi(self, x, y, z):
        return self.sign * (self._r(x, y, z) - self.R)

    def root(self, a, x0, y0, z0, h, start_liquid):
        p = [x0, y0, z0]
        q = np.zeros_like(np.asarray(x0, float))
        for b in range(self.dim):
            if b != a:
                q = q + (p[b] - self.c[b]) ** 2
        disc = np.sqrt(np.maximum(self.R * self.R - q, 0.0))
        # going +e_a: leaving the ball if the start is inside, entering otherwise
        start_inside = (start_liquid == 1) if self.sign < 0 else (start_liquid == 0)
        xs = np.where(start_inside, self.c[a] + disc, self.c[a] - disc)
        return (xs - p[a]) / h


class Film(LevelSet):
    """phi = y - H(x, z), H given at vertex columns and bilinear in between."""

    def __init__(self, H, h, dim):
        self.H = np.asarray(H, float)  # [nvz][nvx]
        self.h = h
        self.dim = dim

    def _H(self, x, z):
        h = self.h
        nvz, nvx = self.H.shape
        fi = np.clip(x / h, 0, nvx - 1 - 1e-12)
        i = np.floor(fi).astype(int)
        i = np.minimum(i, nvx - 2)
        tx = fi - i
        if self.dim == 2:
            return (1 - tx) * self.H[0, i] + tx * self.H[0, i + 1]
        fk = np.clip(z / h, 0, nvz - 1 - 1e-12)
        k = np.floor(fk).astype(int)
        k = np.minimum(k, nvz - 2)
        tz = fk - k
        return ((1 - tx) * (1 - tz) * self.H[k, i] + tx * (1 - tz) * self.H[k, i + 1]
                + (1 - tx) * tz * self.H[k + 1, i] + tx * tz * self.H[k + 1, i + 1])

    def phi(self, x, y, z):
        return y - self._H(x, z)

    def root(self, a, x0, y0, z0, h, start_liquid):
        i = np.rint(x0 / h).astype(int)
        k = np.rint(z0 / h).astype(int) if self.dim == 3 else np.zeros_like(i)
        if a == 1:
            return (self.H[k, i] - y0) / h
        if a == 0:
            H0, H1 = self.H[k, i], self.H[k, i + 1]
        else:
            H0, H1 = self.H[k, i], self.H[k + 1, i]
        return (y0 - H0) / (H1 - H0)


# ----------------------------------------------------------------------------
# markers and colours from a level set
# ----------------------------------------------------------------------------

def colours_and_markers(dim, n, h, ls: LevelSet):
    """Vertex colours, cell colours and edge markers at exact crossings.

    An edge gets a marker iff its end vertices have different colours (at most
    one marker per edge); ties phi = 0 count as liquid.
    """
    vx, vy, vz = _vertex_coords(dim, n, h)
    vcol = (ls.phi(vx, vy, vz) >= 0).astype(np.uint8)
    cx, cy, cz = _cell_coords(dim, n, h)
    ccol = (ls.phi(cx, cy, cz) >= 0).astype(np.uint8)
    markers = []
    for a in range(dim):
        es = edge_shape(dim, n, a)
        sl = tuple(slice(0, e) for e in es)
        hi = [slice(0, e) for e in es]
        hi[2 - a] = slice(1, es[2 - a] + 1)
        c0 = vcol[sl]
        c1 = vcol[tuple(hi)]
        cut = c0 != c1
        s = np.full(es, np.nan)
        x0, y0, z0 = vx[sl], vy[sl], vz[sl]
        r = ls.root(a, x0[cut], y0[cut], z0[cut], h, c0[cut])
        s[cut] = np.clip(r, 0.0, 1.0)
        markers.append(s)
    return vcol, ccol, markers


def _bcs(dim, kinds_T, kinds_p):
    return list(kinds_T[: 2 * dim]), list(kinds_p[: 2 * dim])


def _zero_faces(dim, n):
    return [np.zeros(face_shape(dim, n, a)) for a in range(dim)]


# ----------------------------------------------------------------------------
# the benchmark workloads
# ----------------------------------------------------------------------------

def stefan_2d(n=64, x_gamma_cells=19.2, props=None, dt=1e-4, T_wall=1.0, name="stefan64"):
    """Planar vapour layer against a heated wall at x = 0 (x < x_Gamma vapour).

    Markers sit on every horizontal grid line at the exact position x_Gamma;
    vapour T is linear from T_wall at the wall to T_sat at the interface,
    liquid at T_sat, velocities zero.  Walls: x = 0 heated wall (p Neumann),
    x = 1 outflow (p = 0, T Neumann), y sides symmetry (Neumann).
    """
    props = props or Props()
    dim = 2
    h = 1.0 / n
    nn = (n, n, 1)
    ig = int(math.floor(x_gamma_cells))
    s_val = x_gamma_cells - ig
    vx, vy, vz = _vertex_coords(dim, nn, h)
    vcol = (np.arange(n + 1)[None, None, :] >= ig + (1 if s_val > 0 else 0)).astype(np.uint8)
    vcol = np.broadcast_to(vcol, vertex_shape(dim, nn)).copy()
    ccol = ((np.arange(n) + 0.5)[None, None, :] >= x_gamma_cells).astype(np.uint8)
    ccol = np.broadcast_to(ccol, cell_shape(dim, nn)).copy()
    mx = np.full(edge_shape(dim, nn, 0), np.nan)
    if s_val > 0:
        mx[:, :, ig] = s_val
    else:
        mx[:, :, ig - 1] = 1.0
    my = np.full(edge_shape(dim, nn, 1), np.nan)
    xg = x_gamma_cells * h
    xc = (np.arange(n) + 0.5) * h
    T0 = np.where(ccol == 0, props.T_sat + (T_wall - props.T_sat) * (1.0 - xc[None, None, :] / xg), props.T_sat)
    T_bc = [(DIRICHLET, T_wall), (NEUMANN, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    p_bc = [(NEUMANN, 0.0), (DIRICHLET, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    return Case(name, dim, nn, h, props, dt, T_bc, p_bc, [mx, my], vcol, ccol,
                T0.astype(np.float64), _zero_faces(dim, nn), _zero_faces(dim, nn))


def bubble(dim, n, R, dT, delta, rho_ratio, lam_ratio, sigma_u=0.0, seed=None, dt=1e-4,
           centre=None, name=None, rng=None):
    """Vapour bubble (circle / sphere) at T_sat in a liquid with an erf profile.

    Liquid T = T_sat + dT*erf((r - R)/delta); every side is an outflow
    (p = 0, T Neumann).  Face velocities, if sigma_u > 0, are i.i.d. normal
    draws, identical in both phase fields.
    """
    rho_v = 1.0 / rho_ratio
    props = Props(rho_l=1.0, rho_v=rho_v, lam_l=1.0, lam_v=lam_ratio, cp_l=1.0, cp_v=1.0,
                  h_lg=dT / rho_v, T_sat=0.0)
    h = 1.0 / n
    nn = (n, n, n if dim == 3 else 1)
    c = centre if centre is not None else (0.5, 0.5, 0.5)
    ls = Ball(c, R, +1.0, dim)
    vcol, ccol, markers = colours_and_markers(dim, nn, h, ls)
    cx, cy, cz = _cell_coords(dim, nn, h)
    r = ls._r(cx, cy, cz)
    from scipy.special import erf
    T0 = np.where(ccol == 1, props.T_sat + dT * erf((r - R) / delta), props.T_sat)
    T_bc = [(NEUMANN, 0.0)] * (2 * dim)
    p_bc = [(DIRICHLET, 0.0)] * (2 * dim)
    if sigma_u > 0:
        rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
        u = [rng.normal(0.0, sigma_u, face_shape(dim, nn, a)) for a in range(dim)]
        u_l = [x.copy() for x in u]
        u_v = [x.copy() for x in u]
    else:
        u_l, u_v = _zero_faces(dim, nn), _zero_faces(dim, nn)
    return Case(name or f"bubble{dim}d_{n}", dim, nn, h, props, dt, T_bc, p_bc, markers,
                vcol, ccol, T0.astype(np.float64), u_l, u_v)


class Slab(LevelSet):
    """Liquid in |y - yc| < w / 2 (a horizontal slab in 2D)."""

    def __init__(self, yc, w):
        self.yc, self.w = yc, w

    def phi(self, x, y, z):
        return 0.5 * self.w - np.abs(y - self.yc)

    def root(self, a, x0, y0, z0, h, start_liquid):
        lo = (self.yc - 0.5 * self.w - y0) / h
        hi = (self.yc + 0.5 * self.w - y0) / h
        return np.where((lo >= 0.0) & (lo <= 1.0), lo, hi)


def thin_slab_2d(nx=32, ny=20, yc_cells=9.63, w_cells=1.45, name="slab2d"):
    """A liquid slab thinner than two cells across a 2D box periodic in x
    with walls in y (T Neumann, p Dirichlet), h = 1/nx: a single row of
    liquid centres, the interface cells in the rows either side.  T is zero
    (the caller sets the liquid row's values)."""
    dim, n = 2, (nx, ny, 1)
    h = 1.0 / nx
    ls = Slab(yc_cells * h, w_cells * h)
    vcol, ccol, mk = colours_and_markers(dim, n, h, ls)
    zero = _zero_faces(dim, n)
    bc_T = [(PERIODIC, 0.0), (PERIODIC, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    bc_p = [(PERIODIC, 0.0), (PERIODIC, 0.0), (DIRICHLET, 0.0), (DIRICHLET, 0.0)]
    return Case(name, dim, n, h, Props(rho_l=1.0, rho_v=0.05), 1e-4, bc_T, bc_p, mk, vcol, ccol,
                np.zeros(cell_shape(dim, n)), zero, [z.copy() for z in zero])


def translating_bubble(n, U, dt, dT=0.2):
    """A vapour disc (R = 0.203, off the grid's symmetry lines) in a unit box
    periodic in x with walls in y, carried by a uniform flow U along x in
    both phases; the liquid holds T_sat + dT (1 + sin 2 pi x) sin^2 pi y,
    the vapour T_sat, so the flow carries a temperature field with
    gradients and the interface evaporates where the liquid is warm.  Unit
    properties but for rho_v = lam_v = 0.5 and h_lg = 100 (the evaporation
    speed mdot / rho_v stays a fraction of U)."""
    h = 1.0 / n
    nn = (n, n, 1)
    ls = Ball((0.513, 0.507, 0.0), 0.203, 1.0, 2)
    vcol, ccol, markers = colours_and_markers(2, nn, h, ls)
    pr = Props(rho_l=1.0, rho_v=0.5, lam_l=1.0, lam_v=0.5, cp_l=1.0, cp_v=1.0, h_lg=100.0, T_sat=0.0)
    x, y = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h)
    Tl = dT * (1.0 + np.sin(2 * np.pi * x)) * np.sin(np.pi * y) ** 2
    T0 = np.where(ccol[0] == 1, Tl, 0.0)[None].astype(np.float64)
    T_bc = [(PERIODIC, 0.0), (PERIODIC, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    p_bc = [(PERIODIC, 0.0), (PERIODIC, 0.0), (DIRICHLET, 0.0), (DIRICHLET, 0.0)]
    ux = np.full(face_shape(2, nn, 0), U)
    uy = np.zeros(face_shape(2, nn, 1))
    return Case(f"translating_bubble_{n}", 2, nn, h, pr, dt, T_bc, p_bc, markers, vcol, ccol, T0,
                [ux, uy], [ux.copy(), uy.copy()])


def film_3d(n=256, seed=5, rho_ratio=200.0, lam_ratio=0.2, T_wall=1.0, dt=1e-4, name=None):
    """Film-boiling-like layer: vapour below y = H(x, z), heated wall at y = 0.

    H = 0.25 + 0.02 cos(2 pi x) cos(2 pi z) + 1e-3 xi at vertex columns
    (xi ~ U[-1, 1], periodic in x and z), bilinear in between.  Vapour T is
    linear from T_wall at the wall to T_sat at the interface.
    """
    rho_v = 1.0 / rho_ratio
    props = Props(rho_l=1.0, rho_v=rho_v, lam_l=1.0, lam_v=lam_ratio, cp_l=1.0, cp_v=1.0,
                  h_lg=T_wall / rho_v, T_sat=0.0)
    dim = 3
    h = 1.0 / n
    nn = (n, n, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.uniform(-1.0, 1.0, (n, n))           # [k][i] on the periodic columns
    xi = np.pad(xi, ((0, 1), (0, 1)), mode="wrap")
    xs = np.arange(n + 1) * h
    H = 0.25 + 0.02 * np.cos(2 * np.pi * xs)[None, :] * np.cos(2 * np.pi * xs)[:, None] + 1e-3 * xi
    H[:, -1] = H[:, 0]
    H[-1, :] = H[0, :]
    ls = Film(H, h, dim)
    vcol, ccol, markers = colours_and_markers(dim, nn, h, ls)
    cx, cy, cz = _cell_coords(dim, nn, h)
    Hc = ls._H(cx, cz)
    T0 = np.where(ccol == 0, props.T_sat + (T_wall - props.T_sat) * (1.0 - cy / Hc), props.T_sat)
    T_bc = [(PERIODIC, 0.0), (PERIODIC, 0.0), (DIRICHLET, T_wall), (NEUMANN, 0.0), (PERIODIC, 0.0), (PERIODIC, 0.0)]
    p_bc = [(PERIODIC, 0.0), (PERIODIC, 0.0), (NEUMANN, 0.0), (DIRICHLET, 0.0), (PERIODIC, 0.0), (PERIODIC, 0.0)]
    return Case(name or f"film3d_{n}", dim, nn, h, props, dt, T_bc, p_bc, markers, vcol, ccol,
                T0.astype(np.float64), _zero_faces(dim, nn), _zero_faces(dim, nn))


def stefan_layer(n, x_gamma, dT, rho_ratio, lam_ratio, sigma_u=0.0, rng=None, dt=1e-4, name=None):
    """Planar vapour layer x < x_gamma on a wall at T_sat + dT (2D, any side n)."""
    rho_v = 1.0 / rho_ratio
    props = Props(rho_l=1.0, rho_v=rho_v, lam_l=1.0, lam_v=lam_ratio, cp_l=1.0, cp_v=1.0,
                  h_lg=dT / rho_v, T_sat=0.0)
    dim = 2
    h = 1.0 / n
    nn = (n, n, 1)
    ls = Plane((1.0, 0.0, 0.0), (x_gamma, 0.0, 0.0))
    vcol, ccol, markers = colours_and_markers(dim, nn, h, ls)
    cx, cy, cz = _cell_coords(dim, nn, h)
    T0 = np.where(ccol == 0, props.T_sat + dT * (1.0 - cx / x_gamma), props.T_sat)
    T_bc = [(DIRICHLET, props.T_sat + dT), (NEUMANN, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    p_bc = [(NEUMANN, 0.0), (DIRICHLET, 0.0), (NEUMANN, 0.0), (NEUMANN, 0.0)]
    if sigma_u > 0:
        u = [rng.normal(0.0, sigma_u, face_shape(dim, nn, a)) for a in range(dim)]
        u[0][:, :, 0] = 0.0   # no flow through the heated wall
        u_l = [x.copy() for x in u]
        u_v = [x.copy() for x in u]
    else:
        u_l, u_v = _zero_faces(dim, nn), _zero_faces(dim, nn)
    return Case(name or f"stefan2d_{n}", dim, nn, h, props, dt, T_bc, p_bc, markers, vcol, ccol,
                T0.astype(np.float64), u_l, u_v)


def batch_cases(ncases=64, seed=4, sides=(64, 96, 128, 192, 256)):
    """Uneven batch of 2D cases: even index -> bubble, odd -> Stefan layer.

    Per case the draws are taken in the order (side, R, dT, rho ratio,
    lambda ratio) from one PCG64 stream, then the velocity noise.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for c in range(ncases):
        side = int(sides[rng.integers(0, len(sides))])
        R = rng.uniform(0.05, 0.2)
        dT = rng.uniform(0.5, 5.0)
        rho_ratio = 10.0 ** rng.uniform(1.0, 3.0)
        lam_ratio = rng.uniform(0.02, 0.5)
        if c % 2 == 0:
            cs = bubble(2, side, R, dT, 0.02, rho_ratio, lam_ratio, sigma_u=1e-3, rng=rng,
                        name=f"batch{c}_bubble{side}")
        else:
            cs = stefan_layer(side, 2 * R, dT, rho_ratio, lam_ratio, sigma_u=1e-3, rng=rng,
                              name=f"batch{c}_stefan{side}")
        cases.append(cs)
    return cases


def config(idx: int, n: Optional[int] = None):
    """The five synthetic workloads (index 0..4); ``n`` overrides the side."""
    if idx == 0:
        return stefan_2d(n or 64, x_gamma_cells=0.3 * (n or 64) if n else 19.2, name="stefan2d_64")
    if idx == 1:
        return bubble(2, n or 256, 0.1, 1.0, 0.02, 1000.0, 0.1, sigma_u=1e-3, seed=2,
                      name=f"bubble2d_{n or 256}")
    if idx == 2:
        return bubble(3, n or 128, 0.15, 2.0, 0.03, 1000.0, 0.05, name=f"bubble3d_{n or 128}")
    if idx == 3:
        return batch_cases()
    if idx == 4:
        return film_3d(n or 256)
    raise ValueError(idx)


def random_case(dim, n, seed, kind="ball", rho_ratio=100.0, lam_ratio=0.2, bc="outflow"):
    """Small random cases for parity tests: random ball or tilted plane."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    nn = (n, n, n if dim == 3 else 1)
    if kind == "ball":
        c = rng.uniform(0.35, 0.65, 3)
        R = rng.uniform(0.15, 0.3)
        sign = 1.0 if rng.uniform() < 0.7 else -1.0
        ls = Ball(c, R, sign, dim)
    else:
        m = rng.normal(size=3)
        if dim == 2:
            m[2] = 0.0
        m /= np.linalg.norm(m)
        p = np.array([0.5, 0.5, 0.5]) + rng.uniform(-0.1, 0.1, 3)
        ls = Plane(m, p)
    vcol, ccol, markers = colours_and_markers(dim, nn, h, ls)
    props = Props(rho_l=1.0, rho_v=1.0 / rho_ratio, lam_l=1.0, lam_v=lam_ratio, cp_l=1.0, cp_v=1.0,
                  h_lg=rho_ratio, T_sat=0.0)
    T0 = rng.uniform(-1.0, 1.0, cell_shape(dim, nn))
    u = [rng.normal(0.0, 1e-2, face_shape(dim, nn, a)) for a in range(dim)]
    uv = [x + rng.normal(0.0, 1e-3, x.shape) for x in u]
    if bc == "outflow":
        T_bc = [(NEUMANN, 0.0)] * (2 * dim)
        p_bc = [(DIRICHLET, 0.0)] * (2 * dim)
    elif bc == "mixed":
        T_bc = [(DIRICHLET, 1.0), (NEUMANN, 0.0)] + [(NEUMANN, 0.0)] * (2 * dim - 2)
        p_bc = [(NEUMANN, 0.0), (DIRICHLET, 0.0)] + [(NEUMANN, 0.0)] * (2 * dim - 2)
        u[0][..., 0] = 0.0
        uv[0][..., 0] = 0.0
    else:
        raise ValueError(bc)
    return Case(f"rand{dim}d_{kind}_{n}_{seed}", dim, nn, h, props, 1e-4 * (64.0 / n) ** 2, T_bc, p_bc,
                markers, vcol, ccol, T0, u, uv)
