"""Pins of the marker-motion oracle (oracle/advect.py).

* bilinear interpolation reproduces linear fields exactly, inside and
  (extrapolating) next to walls, and wraps on periodic axes;
* Eq. jump_interfacial_vel: phase fields that satisfy the velocity jump
  (Eq. velocity_jump) give one interfacial velocity from either phase,
  u_v + mdot/rho_v n;
* straight interfaces translate exactly (markers, vertex and cell colours
  against the exact markers of the moved line), on walls and on a doubly
  periodic grid;
* a circle growing with a constant normal speed keeps its markers on the
  circle of radius R0 + V t (Sec. 3.3, R(t) = R0 + mdot t / rho_v), within
  what explicit Euler in time allows, and the result is always a
  consistent EBIT geometry;
* the time loop on the Stefan problem (Sec. 3.1) follows X(t) of
  Eq. stefan_interface_position at grid levels 4 and 5;
* saddles are rejected, zero velocity leaves the interface in place.
"""
import dataclasses
import math

import numpy as np
import pytest

import ebit_inputs as ei
from advect_util import (circle_case, compare_markers, interface_x, line_case, near_marker_vertices,
                         oracle_time_loop, stefan_case, stefan_constants, stripe_case, STEFAN_T0)
from oracle import advect, closed, extend, geometry
from oracle.geometry import GeometryError


def _field(case, f):
    nx, ny, _ = case.n
    h = case.h
    x, y = np.meshgrid((np.arange(nx) + 0.5) * h, (np.arange(ny) + 0.5) * h)
    return np.stack([f(x, y)[0].ravel(), f(x, y)[1].ravel()], axis=1)


def test_bilinear_is_exact_for_linear_fields():
    rng = np.random.Generator(np.random.PCG64(11))
    case = line_case(16, (1.0, 0.3), (0.5, 0.5))
    A = rng.normal(size=(2, 3))
    f = lambda x, y: (A[0, 0] * x + A[0, 1] * y + A[0, 2], A[1, 0] * x + A[1, 1] * y + A[1, 2])
    ug = _field(case, f)
    # interior points, points in the half cell next to each wall, corners
    P = np.concatenate([rng.uniform(0.05, 0.95, (200, 2)), rng.uniform(0.0, 1.0 / 32, (20, 2)),
                        1.0 - rng.uniform(0.0, 1.0 / 32, (20, 2)), [[0.0, 0.0], [1.0, 1.0], [0.0, 1.0]]])
    got = advect.interpolate(case, ug, P)
    ex = np.stack(f(P[:, 0], P[:, 1]), axis=1)
    assert np.max(np.abs(got - ex)) < 1e-13


def test_bilinear_wraps_on_periodic_axes():
    """On a periodic grid the stencil of a point near x = 0 takes the last
    column: the value equals that of the same point seen one period on."""
    rng = np.random.Generator(np.random.PCG64(12))
    case = stripe_case(16, 0.2, 0.6)
    ug = rng.normal(size=(256, 2))
    P = rng.uniform(0.0, 1.0 / 32, (50, 2))
    got = advect.interpolate(case, ug, P)
    # the same points on the grid rolled by one cell (cell i -> i + 1)
    rolled = np.roll(ug.reshape(16, 16, 2), (1, 1), axis=(0, 1)).reshape(-1, 2)
    got2 = advect.interpolate(case, rolled, P + 1.0 / 16)
    assert np.max(np.abs(got - got2)) < 1e-15
    # and the weights of a point half a cell from the seam are 1/2, 1/2
    q = advect.interpolate(case, ug, np.array([[0.0, 1.0 / 32]]))
    g = ug.reshape(16, 16, 2)
    assert np.allclose(q[0], 0.5 * (g[0, 0] + g[0, 15]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("normal", [(1.0, 0.0), (1.0, 0.4), (-0.3, 1.0)])
def test_interface_velocity_is_one_value_across_the_jump(normal):
    """u_v = U, u_l = U + mdot (1/rho_v - 1/rho_l) n (Eq. velocity_jump) with
    a planar interface: every band cell, liquid or vapour, gets U + mdot/rho_v n."""
    case = line_case(24, normal, (0.52, 0.47), rho=(1000.0, 1.0))
    geo = geometry.build(case)
    n = np.array(normal) / np.linalg.norm(normal)
    U = np.array([0.3, -0.2])
    mdot = 0.7
    jump = mdot * (1.0 / case.props.rho_v - 1.0 / case.props.rho_l)
    nn = case.n
    uv = [np.full(ei.face_shape(2, nn, a), U[a]) for a in range(2)]
    ul = [np.full(ei.face_shape(2, nn, a), U[a] + jump * n[a]) for a in range(2)]
    inb, _ = extend.band(case, geo)
    m = np.where(inb, mdot, 0.0)
    ug = advect.cell_interface_velocity(case, geo, ul, uv, m)
    ex = U + mdot / case.props.rho_v * n
    assert np.max(np.abs(ug[inb] - ex)) < 1e-12 * np.max(np.abs(ex))
    # off the band each cell keeps its own phase's velocity
    col = case.ccol.ravel().astype(bool)
    off = ~inb
    assert np.allclose(ug[off & col], U + jump * n, rtol=0, atol=1e-15)
    assert np.allclose(ug[off & ~col], U, rtol=0, atol=1e-15)


def test_interface_velocity_3d_band_cells():
    """The cell-centre velocity in 3D: the same closed form for a tilted plane."""
    rng_case = ei.random_case(3, 16, 3, kind="plane")
    case = dataclasses.replace(rng_case, props=ei.Props(rho_l=500.0, rho_v=2.0))
    geo = geometry.build(case)
    inb, nb = extend.band(case, geo)
    nF = geo["nF"].reshape(-1, 3)[geo["is_if"]][0]
    U = np.array([0.1, 0.2, -0.3])
    mdot = -0.4
    jump = mdot * (1.0 / 2.0 - 1.0 / 500.0)
    uv = [np.full(ei.face_shape(3, case.n, a), U[a]) for a in range(3)]
    ul = [np.full(ei.face_shape(3, case.n, a), U[a] + jump * nF[a]) for a in range(3)]
    ug = advect.cell_interface_velocity(case, geo, ul, uv, np.where(inb, mdot, 0.0))
    assert np.max(np.abs(ug[inb] - (U + mdot / 2.0 * nF))) < 1e-12


def _translate(case, u, dt):
    ug = np.tile(np.asarray(u, float), (case.ncells, 1))
    mk, vc = case.markers, case.vcol
    for a in range(2):
        mk, vc = advect.advect_pass(case, mk, vc, ug, dt, a)
    return mk, vc, advect.cell_colours(case, mk, vc)


def _check_against(case, mk, vc, cc, ref, tol=1e-11):
    compare_markers(mk, ref.markers, tol)
    near = near_marker_vertices(ref.markers, case.n[:2], 1e-9)
    assert np.array_equal(vc[0][~near], ref.vcol[0][~near])
    assert np.array_equal(cc, ref.ccol)


@pytest.mark.parametrize("normal,point,u", [
    ((1.0, 0.35), (0.43, 0.5), (0.7, 0.0)),     # steep line, moved along x
    ((1.0, -0.2), (0.61, 0.5), (-0.9, 0.0)),
    ((0.3, 1.0), (0.5, 0.45), (0.0, 0.8)),      # flat line, moved along y
    ((-0.25, 1.0), (0.5, 0.55), (0.0, -0.6)),
])
def test_straight_line_translates_exactly(normal, point, u):
    """A line that touches only the walls parallel to the motion moves
    exactly: both passes rebuild the markers of the moved line."""
    n = 32
    case = line_case(n, normal, point)
    dt = 0.6 / n
    mk, vc, cc = _translate(case, u, dt)
    moved = line_case(n, normal, (point[0] + u[0] * dt, point[1] + u[1] * dt))
    _check_against(case, mk, vc, cc, moved)
    geometry.check_markers(dataclasses.replace(case, markers=list(mk), vcol=vc))


@pytest.mark.parametrize("u", [(0.8, 0.0), (0.0, -0.7), (0.5, 0.45), (-0.6, 0.3)])
def test_periodic_stripe_translates_exactly(u):
    """Two lines of slope 1 on a doubly periodic grid: any translation moves
    them exactly, across the seams too."""
    n = 24
    c1, c2 = 0.137, 0.583
    case = stripe_case(n, c1, c2)
    dt = 0.9 / n
    mk, vc, cc = _translate(case, u, dt)
    shift = u[0] * dt - u[1] * dt                   # x - y of a moved point
    moved = stripe_case(n, c1 + shift, c2 + shift)
    _check_against(case, mk, vc, cc, moved)
    # each seam line is one grid line stored twice: the copies agree bit for bit
    assert np.array_equal(mk[0][0][n, :], mk[0][0][0, :], equal_nan=True)
    assert np.array_equal(mk[1][0][:, n], mk[1][0][:, 0], equal_nan=True)
    assert np.array_equal(vc[0][n, :], vc[0][0, :]) and np.array_equal(vc[0][:, n], vc[0][:, 0])


def _grow(case, V, steps, dt):
    """Advect with the interfacial velocity V n_band (rho_l = rho_v = 1,
    u = 0, mdot = V in the band): the band normal points out of the vapour."""
    for _ in range(steps):
        geo = geometry.build(case)
        inb, _ = extend.band(case, geo)
        z = [np.zeros(ei.face_shape(2, case.n, a)) for a in range(2)]
        mk, vc, cc = advect.advect(case, geo, z, z, np.where(inb, V, 0.0), dt)
        case = dataclasses.replace(case, markers=list(mk), vcol=vc, ccol=cc)
    return case


def _radius_error(case, centre, R):
    err = 0.0
    for a in range(2):
        jj, ii, P = advect.marker_points(case, case.markers, a)
        r = np.hypot(P[:, 0] - centre[0], P[:, 1] - centre[1])
        err = max(err, float(np.max(np.abs(r - R))))
    return err


def test_growing_circle_follows_the_closed_form():
    """A vapour disc growing at the constant speed V = mdot/rho_v (Sec. 3.3):
    R(t) = R0 + V t.  Explicit Euler in split passes is first order in dt,
    so with dt = 0.4 h / V the markers stay within 0.05 h of that circle at
    two resolutions (a chord re-intersection instead of the circle fit
    drifts 0.15 h inwards), the error shrinks with dt, and the colours agree
    with the exact disc away from the interface."""
    centre, R0, V, T = (0.5, 0.5), 0.2, 1.0, 0.08
    errs = {}
    for n, c in ((32, 0.4), (64, 0.4), (32, 0.1)):
        dt = c / n / V
        steps = int(round(T / dt))
        case = _grow(circle_case(n, centre, R0), V, steps, dt)
        geometry.check_markers(case)
        R = R0 + V * steps * dt
        errs[(n, c)] = _radius_error(case, centre, R) / case.h
        ex = circle_case(n, centre, R)
        # vertices and cells more than one cell from the circle
        h = case.h
        vx, vy = np.meshgrid(np.arange(n + 1) * h, np.arange(n + 1) * h)
        far_v = np.abs(np.hypot(vx - centre[0], vy - centre[1]) - R) > h
        assert np.array_equal(case.vcol[0][far_v], ex.vcol[0][far_v])
        cx, cy = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h)
        far_c = np.abs(np.hypot(cx - centre[0], cy - centre[1]) - R) > h
        assert np.array_equal(case.ccol[0][far_c], ex.ccol[0][far_c])
    assert errs[(32, 0.4)] < 0.05 and errs[(64, 0.4)] < 0.05, errs
    assert errs[(32, 0.1)] < 0.5 * errs[(32, 0.4)], errs


def test_random_motions_keep_a_consistent_geometry():
    """Random smooth velocity fields (CFL up to 0.9) on random discs and
    lines: the markers stay consistent with the vertex colours (one marker
    on every edge whose ends differ and nowhere else) and inside [0, 1]."""
    for seed in range(6):
        rng = np.random.Generator(np.random.PCG64(100 + seed))
        n = 24
        if seed % 2 == 0:
            case = circle_case(n, rng.uniform(0.35, 0.65, 2), rng.uniform(0.15, 0.3), bool(seed % 4))
        else:
            case = line_case(n, rng.normal(size=2), rng.uniform(0.4, 0.6, 2))
        k = rng.normal(size=(2, 3))
        f = lambda x, y: (k[0, 0] + k[0, 1] * np.sin(3 * y) + k[0, 2] * x,
                          k[1, 0] + k[1, 1] * np.cos(2 * x) + k[1, 2] * y)
        ug = _field(case, f)
        dt = 0.9 * case.h / np.max(np.abs(ug))
        mk, vc = case.markers, case.vcol
        for a in range(2):
            mk, vc = advect.advect_pass(case, mk, vc, ug, dt, a)
        cc = advect.cell_colours(case, mk, vc)
        moved = dataclasses.replace(case, markers=list(mk), vcol=vc, ccol=cc)
        geometry.check_markers(moved)
        for m in mk:
            v = m[~np.isnan(m)]
            assert np.all((v >= 0) & (v <= 1))


def test_zero_velocity_leaves_the_interface():
    case = circle_case(32, (0.47, 0.52), 0.21)
    ug = np.zeros((case.ncells, 2))
    mk, vc = case.markers, case.vcol
    for a in range(2):
        mk, vc = advect.advect_pass(case, mk, vc, ug, 1e-3, a)
    compare_markers(mk, case.markers, 1e-14)
    assert np.array_equal(vc, case.vcol)
    assert np.array_equal(advect.cell_colours(case, mk, vc), advect.cell_colours(case, case.markers, case.vcol))


def test_saddle_cells_are_rejected():
    """Two liquid vertices on a diagonal of cell (3, 3), vapour elsewhere:
    that cell holds four markers."""
    case = line_case(8, (1.0, 0.0), (2.0, 0.5))          # all vapour
    vcol = case.vcol.copy()
    mx, my = (m.copy() for m in case.markers)
    for (vi, vj) in ((3, 3), (4, 4)):
        vcol[0, vj, vi] = 1
        mx[0, vj, vi - 1] = 0.5
        mx[0, vj, vi] = 0.5
        my[0, vj - 1, vi] = 0.5
        my[0, vj, vi] = 0.5
    bad = dataclasses.replace(case, markers=[mx, my], vcol=vcol)
    geometry.check_markers(bad)                          # consistent, but a saddle
    with pytest.raises(GeometryError):
        advect.advect_pass(bad, bad.markers, bad.vcol, np.zeros((64, 2)), 1e-3, 0)


def test_stefan_front_follows_the_closed_form():
    """Sec. 3.1 (Ja = 29.84): from t = 0.282 s to t = 5.282 s with dt = 0.01 s
    the front of the full loop (interfacial velocity, marker motion, sharp
    diffusion, mass flux, projection) follows X(t) = 2 beta sqrt(alpha_v t)
    within 5e-3 all along at grid levels 4 and 5 (the largest excursions
    come early, while the layer is one or two cells thick), ends within 2e-3
    and 1e-3, and the finer level ends the closer."""
    pr, beta, alpha = stefan_constants()
    t1 = 5.282
    final = []
    for nx, bound in ((16, 2e-3), (32, 1e-3)):
        worst = [0.0]

        def watch(s, t, case, T, mdot):
            Xt = closed.stefan_position(t, beta, alpha)
            worst[0] = max(worst[0], abs(interface_x(case) - Xt) / Xt)

        case = stefan_case(nx, dt=0.01)
        case, T, t = oracle_time_loop(case, t1, on_step=watch)
        assert abs(t - t1) < 1e-9
        Xt = closed.stefan_position(t, beta, alpha)
        final.append(abs(interface_x(case) - Xt) / Xt)
        assert worst[0] < 5e-3, (nx, worst[0])
        assert final[-1] < bound, (nx, final[-1])
    assert final[1] < final[0], final
