"""Helpers of the marker-motion tests: the thin Stefan problem of Sec. 3.1 on
the oracle (a time loop in the order of Sec. 2.5), straight and circular
test interfaces with exact markers, and marker comparisons that accept the
two spellings of a marker sitting on a vertex."""
import dataclasses
import math

import numpy as np

import ebit_inputs as ei
from oracle import advect, closed, energy, extend, flux, geometry, heat, project, solve

# Sec. 3.1: water at 1 bar, wall 10 K above saturation, 10 mm domain, the
# layer 322.5 um thick at t = 0.282 s
STEFAN_PROPS = dict(rho_l=958.0, rho_v=0.6, lam_l=0.68, lam_v=0.025, cp_l=4216.0, cp_v=2080.0,
                    h_lg=2.256e6, T_sat=373.15)
STEFAN_TW = 383.15
STEFAN_L = 0.01
STEFAN_X0 = 322.5e-6
STEFAN_T0 = 0.282
EXT_ITERS = 8


def stefan_constants():
    pr = ei.Props(**STEFAN_PROPS)
    beta = closed.stefan_beta(pr.cp_v, STEFAN_TW - pr.T_sat, pr.h_lg)
    alpha = pr.lam_v / (pr.rho_v * pr.cp_v)
    return pr, beta, alpha


def stefan_case(nx, ny=4, dt=0.01):
    """The layer on nx x ny cells of side 10 mm / nx: heated wall at x = 0
    (T Dirichlet, p Neumann), outlet at x = l (T Neumann, p = 0), symmetry
    at the y sides; vapour T from the closed form at t0, liquid at T_sat."""
    pr, beta, alpha = stefan_constants()
    h = STEFAN_L / nx
    nn = (nx, ny, 1)
    ls = ei.Plane((1.0, 0.0, 0.0), (STEFAN_X0, 0.0, 0.0))
    vcol, ccol, markers = ei.colours_and_markers(2, nn, h, ls)
    cx = (np.arange(nx) + 0.5) * h
    Tv = closed.stefan_T(cx, STEFAN_T0, beta, alpha, STEFAN_TW, pr.T_sat)
    T = np.where(ccol[0] == 0, Tv[None, :], pr.T_sat).reshape(1, ny, nx).astype(np.float64)
    T_bc = [(ei.DIRICHLET, STEFAN_TW), (ei.NEUMANN, 0.0), (ei.NEUMANN, 0.0), (ei.NEUMANN, 0.0)]
    p_bc = [(ei.NEUMANN, 0.0), (ei.DIRICHLET, 0.0), (ei.NEUMANN, 0.0), (ei.NEUMANN, 0.0)]
    z = [np.zeros(ei.face_shape(2, nn, a)) for a in range(2)]
    return ei.Case(f"stefan_thin_{nx}", 2, nn, h, pr, dt, T_bc, p_bc, markers, vcol, ccol, T, z,
                   [x.copy() for x in z])


def interface_x(case):
    """Mean x of the markers on the x-edges (the planar front)."""
    mx = np.asarray(case.markers[0])[0]
    jj, ii = np.nonzero(~np.isnan(mx))
    return float(np.mean((ii + mx[jj, ii]) * case.h))


def oracle_time_loop(case, t_end, t0=STEFAN_T0, on_step=None, energy_advection=False):
    """Sec. 2.5 on the oracle:
      (with energy_advection) the advection step of the energy equation:
      T* from each phase's field carried across the interface (Eq.
      extrapolation) and that phase's velocity u^n (Eq. energy_advection),
      then T* carried across again; without it T* = T^n (exact for the
      Stefan problem, whose vapour is at rest and liquid uniform);
      the interfacial velocity from u^n and the band-extended mdot^n moves
      the markers; cells that change phase take the other phase's value
      carried across by Eq. extrapolation; the diffusion step on the new
      geometry; mdot and its band extension; the ghost velocities on the
      band faces from the extended mdot (Eq. ghost_velocity); the
      projection.
    The first mdot and velocities come from the initial T."""
    dt = case.dt
    geo = geometry.build(case)
    T = case.T0.ravel().copy()
    mdot, _ = flux.mass_flux(case, geo, T)
    mb = extend.extend(case, geo, mdot, extend.IFACE_TO_BAND, EXT_ITERS)
    ul, uv = project.ghost_velocities_band(case, geo, mb, case.u_l, case.u_v)
    pr = project.project(case, geo, mdot, ul, uv, solve.direct)
    ul, uv = pr["u_l"], pr["u_v"]
    nsteps = int(round((t_end - t0) / dt))
    t = t0
    for s in range(nsteps):
        Tl = extend.extend(case, geo, T, extend.LIQ_TO_VAP, EXT_ITERS)
        Tv = extend.extend(case, geo, T, extend.VAP_TO_LIQ, EXT_ITERS)
        if energy_advection:
            T = energy.advect_energy(case, Tl, Tv, ul, uv, dt)
            Tl = extend.extend(case, geo, T, extend.LIQ_TO_VAP, EXT_ITERS)
            Tv = extend.extend(case, geo, T, extend.VAP_TO_LIQ, EXT_ITERS)
        mk, vc, cc = advect.advect(case, geo, ul, uv, mb, dt)
        old = case.ccol.ravel()
        new = cc.ravel()
        Ts = np.where(new == old, T, np.where(new == 1, Tl, Tv))
        case = dataclasses.replace(case, markers=list(mk), vcol=vc, ccol=cc, T0=Ts.reshape(case.T0.shape))
        geo = geometry.build(case)
        A, b = heat.assemble(case, geo, Ts)
        T = solve.direct(A, b, heat.operator(case, geo))
        mdot, _ = flux.mass_flux(case, geo, T)
        mb = extend.extend(case, geo, mdot, extend.IFACE_TO_BAND, EXT_ITERS)
        ul, uv = project.ghost_velocities_band(case, geo, mb, ul, uv)
        pr = project.project(case, geo, mdot, ul, uv, solve.direct)
        ul, uv = pr["u_l"], pr["u_v"]
        t += dt
        if on_step is not None:
            on_step(s, t, case, T, mdot)
    return case, T, t


# ----------------------------------------------------------------------------
# exact markers of simple interfaces
# ----------------------------------------------------------------------------

def line_case(n, normal, point, periodic=(False, False), seed=0, rho=(1.0, 1.0)):
    """A straight interface {x : normal . (x - point) = 0} (liquid on the
    +normal side) on an n x n grid of side 1, exact markers."""
    m = np.array([normal[0], normal[1], 0.0], dtype=float)
    m /= np.linalg.norm(m)
    h = 1.0 / n
    nn = (n, n, 1)
    ls = ei.Plane(m, (point[0], point[1], 0.0))
    vcol, ccol, markers = ei.colours_and_markers(2, nn, h, ls)
    return _case_from(n, h, nn, vcol, ccol, markers, periodic, rho)


def _case_from(n, h, nn, vcol, ccol, markers, periodic, rho):
    """Walls: T Neumann, p Dirichlet (an outflow); periodic axes: both periodic."""
    pr = ei.Props(rho_l=rho[0], rho_v=rho[1])
    T_bc, p_bc = [], []
    for a in range(2):
        for _ in range(2):
            T_bc.append((ei.PERIODIC, 0.0) if periodic[a] else (ei.NEUMANN, 0.0))
            p_bc.append((ei.PERIODIC, 0.0) if periodic[a] else (ei.DIRICHLET, 0.0))
    z = [np.zeros(ei.face_shape(2, nn, a)) for a in range(2)]
    T0 = np.zeros(ei.cell_shape(2, nn))
    return ei.Case(f"line{n}", 2, nn, h, pr, 1e-3, T_bc, p_bc, markers, vcol, ccol, T0, z,
                   [x.copy() for x in z])


def translating_bubble_case(n, U, dt, dT=0.2):
    """The translating vapour disc of ebit_inputs (a uniform flow U along x,
    periodic in x, walls in y)."""
    return ei.translating_bubble(n, U, dt, dT)


def circle_case(n, centre, R, inside_vapour=True, rho=(1.0, 1.0)):
    h = 1.0 / n
    nn = (n, n, 1)
    ls = ei.Ball((centre[0], centre[1], 0.0), R, 1.0 if inside_vapour else -1.0, 2)
    vcol, ccol, markers = ei.colours_and_markers(2, nn, h, ls)
    return _case_from(n, h, nn, vcol, ccol, markers, (False, False), rho)


def stripe_case(n, c1, c2, periodic=(True, True)):
    """A unit square crossed by two lines of slope 1, x - y = c1 and
    x - y = c2 (mod 1); liquid where (x - y - c1) mod 1 lies in
    (0, (c2 - c1) mod 1).  Periodic axes store their seam line as a copy of
    line 0; a wall axis cuts the stripe."""
    h = 1.0 / n
    nn = (n, n, 1)
    w = (c2 - c1) % 1.0

    def liquid(x, y):
        return ((x - y - c1) % 1.0) < w

    vx, vy = np.meshgrid(np.arange(n + 1) * h, np.arange(n + 1) * h)
    vcol = liquid(vx, vy).astype(np.uint8)
    if periodic[0]:
        vcol[:, n] = vcol[:, 0]
    if periodic[1]:
        vcol[n, :] = vcol[0, :]
    vcol = vcol[None]
    cx, cy = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h)
    ccol = liquid(cx, cy).astype(np.uint8)[None]
    mx = np.full(ei.edge_shape(2, nn, 0), np.nan)
    my = np.full(ei.edge_shape(2, nn, 1), np.nan)
    for c in (c1, c2):
        for j in range(n + 1):
            for i in range(n):
                # x-edge at height y = j h: the crossing x = y + c (mod 1)
                if vcol[0, j, i] != vcol[0, j, i + 1]:
                    x = (j * h + c) % 1.0
                    s = x / h - i
                    if -1e-12 <= s <= 1 + 1e-12:
                        mx[0, j, i] = min(max(s, 0.0), 1.0)
        for j in range(n):
            for i in range(n + 1):
                if vcol[0, j, i] != vcol[0, j + 1, i]:
                    y = (i * h - c) % 1.0
                    s = y / h - j
                    if -1e-12 <= s <= 1 + 1e-12:
                        my[0, j, i] = min(max(s, 0.0), 1.0)
    if periodic[0]:
        my[0, :, n] = my[0, :, 0]
    if periodic[1]:
        mx[0, n, :] = mx[0, 0, :]
    return _case_from(n, h, nn, vcol, ccol, [mx, my], periodic, (1.0, 1.0))


# ----------------------------------------------------------------------------
# comparisons
# ----------------------------------------------------------------------------

def line_coordinates(markers, a):
    """Per grid line of the axis-a edges, the sorted marker coordinates
    (edge index + s) along the line: a marker on a vertex reads the same
    from either edge that holds it."""
    m = np.asarray(markers[a])[0]
    out = []
    lines = m.shape[0] if a == 0 else m.shape[1]
    for line in range(lines):
        row = m[line, :] if a == 0 else m[:, line]
        k = np.nonzero(~np.isnan(row))[0]
        out.append(np.sort(k + row[k]))
    return out


def compare_markers(got, ref, tol):
    """Largest difference of the marker coordinates line by line (in cells);
    raises if a line holds a different number of markers."""
    worst = 0.0
    for a in range(2):
        for line, (g, r) in enumerate(zip(line_coordinates(got, a), line_coordinates(ref, a))):
            assert g.size == r.size, (a, line, g, r)
            if g.size:
                worst = max(worst, float(np.max(np.abs(g - r))))
    assert worst <= tol, worst
    return worst


def near_marker_vertices(markers, n, tol):
    """Boolean [ny+1, nx+1]: vertices within tol (cells) of a marker on one
    of their two lines, where the colour of the vertex is a matter of
    rounding."""
    nx, ny = n
    near = np.zeros((ny + 1, nx + 1), bool)
    for a in range(2):
        for line, cs in enumerate(line_coordinates(markers, a)):
            for c in cs:
                v = int(round(c))
                if abs(c - v) <= tol:
                    if a == 0:
                        near[line, v] = True
                    else:
                        near[v, line] = True
    return near
