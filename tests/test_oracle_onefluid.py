"""Pins for the oracle's one-fluid projection (Eq. pc_source).

Independent references:
  * the interface area of a planar facet in a cell: the derivative of the
    exact volume of a unit cube cut by a plane (inclusion-exclusion over the
    cube's corners), times |m|: A = |m| sum_v (-1)^|v| (alpha - m.v)_+^(d-1)
    / ((d-1)! prod m_i), exact for tilted planes in 2D and 3D;
  * an axis-aligned plane cuts every interface cell in a full face (h^(d-1));
  * in 2D the facet is the chord between the cell's two markers;
  * the facet areas of a circle / sphere add up to its perimeter / area, the
    error falling at second order;
  * with no mass flux the one-fluid projection is the ghost-fluid one on a
    single field, and with a constant mass flux on an evaporating bubble both
    push out the same volume, mdot (1/rho_v - 1/rho_l) |Gamma|, as h -> 0;
  * after the update the divergence equals the source (discrete Gauss: the
    net outflow through the outflow walls is sum S h^d).
"""
import itertools
import math

import numpy as np
import pytest

import ebit_inputs as ei
from oracle import geometry, onefluid, project, solve


def plane_case(dim, n, m, p):
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    ls = ei.Plane(np.asarray(m, float), np.asarray(p, float))
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    bc = [(0, 0.0)] * (2 * dim)
    return ei.Case("plane", dim, nn, h, ei.Props(), 1e-4, bc, [(1, 0.0)] * (2 * dim), mk, vcol, ccol,
                   np.zeros(ei.cell_shape(dim, nn)), [], [])


def ball_case(dim, n, R, props=None):
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    ls = ei.Ball((0.5, 0.5, 0.5), R, 1.0, dim)   # vapour inside
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    zero = [np.zeros(ei.face_shape(dim, nn, a)) for a in range(dim)]
    return ei.Case("ball", dim, nn, h, props or ei.Props(), 1e-4, [(0, 0.0)] * (2 * dim),
                   [(1, 0.0)] * (2 * dim), mk, vcol, ccol, np.zeros(ei.cell_shape(dim, nn)),
                   zero, [z.copy() for z in zero])


def unit_cell_area(m, alpha, dim):
    """Area (3D) / length (2D) of {m.x = alpha} inside the unit cube / square,
    from the derivative of the cut volume (all m_i != 0)."""
    m = np.asarray(m[:dim], float)
    # reflect the axes with negative m_i: x_i -> 1 - x_i
    alpha = alpha - sum(mi for mi in m if mi < 0)
    m = np.abs(m)
    tot = 0.0
    for v in itertools.product((0, 1), repeat=dim):
        d = alpha - float(np.dot(m, v))
        if d > 0:
            tot += (-1) ** sum(v) * d ** (dim - 1)
    return np.linalg.norm(m) * tot / (math.factorial(dim - 1) * np.prod(m))


@pytest.mark.parametrize("dim,n,seed", [(2, 17, 1), (2, 30, 2), (3, 9, 3), (3, 12, 4), (3, 15, 5)])
def test_tilted_plane_area_closed_form(dim, n, seed):
    rng = np.random.default_rng(seed)
    m = rng.normal(size=3)
    if dim == 2:
        m[2] = 0.0
    m /= np.linalg.norm(m)
    p = 0.5 + rng.uniform(-0.1, 0.1, 3)
    case = plane_case(dim, n, m, p)
    g = geometry.build(case)
    S = onefluid.facet_area(case, g)
    cells = np.nonzero(g["is_if"])[0]
    assert cells.size > 0 and np.all(S[~g["is_if"]] == 0.0)
    h = case.h
    for c in cells:
        i, j, k = c % n, (c // n) % n, c // (n * n)
        base = np.array([i * h, j * h, k * h if dim == 3 else 0.0])
        alpha = float(np.dot(m, p - base)) / h
        ref = unit_cell_area(m, alpha, dim) * h ** (dim - 1)
        assert abs(S[c] - ref) <= 1e-10 * h ** (dim - 1), (c, S[c], ref)


@pytest.mark.parametrize("dim,n", [(2, 20), (3, 10)])
def test_axis_plane_full_face(dim, n):
    case = plane_case(dim, n, (1.0, 0.0, 0.0), (0.437, 0.5, 0.5))
    g = geometry.build(case)
    S = onefluid.facet_area(case, g)
    assert np.allclose(S[g["is_if"]], case.h ** (dim - 1), rtol=1e-14, atol=0)


def test_2d_facet_is_the_marker_chord():
    case = ball_case(2, 48, 0.23)
    g = geometry.build(case)
    S = onefluid.facet_area(case, g)
    cells = np.nonzero(g["is_if"])[0]
    slots = geometry._edge_marker_positions(case, cells)
    P = np.stack([p for p, _ in slots], axis=1)
    M = np.stack([q for _, q in slots], axis=1)
    two = M.sum(axis=1) == 2
    d = []
    for r in np.nonzero(two)[0]:
        a, b = P[r][M[r]]
        d.append(np.linalg.norm(a - b))
    # a corner clip a few percent of h long carries the rounding of its
    # crossings: the bound is on the scale of the cell
    assert np.allclose(S[cells[two]], d, rtol=0, atol=1e-13 * case.h)


@pytest.mark.parametrize("dim,R,sizes", [(2, 0.27, (32, 64, 128)), (3, 0.3, (16, 24, 32))])
def test_total_area_converges(dim, R, sizes):
    exact = 2 * math.pi * R if dim == 2 else 4 * math.pi * R * R
    errs = []
    for n in sizes:
        case = ball_case(dim, n, R)
        g = geometry.build(case)
        errs.append(abs(onefluid.facet_area(case, g).sum() - exact) / exact)
    assert errs[-1] < (2e-4 if dim == 2 else 5e-3)
    rate = math.log(errs[0] / errs[-1]) / math.log(sizes[-1] / sizes[0])
    assert rate > 1.6, (errs, rate)


def test_no_mass_flux_equals_ghost_fluid():
    case = ei.random_case(2, 32, 5)
    g = geometry.build(case)
    u = case.u_l
    mdot = np.zeros(case.ncells)
    one = onefluid.project_one_fluid(case, g, mdot, u, solve.direct)
    gfm = project.project(case, g, mdot, u, u, solve.direct)
    assert np.allclose(one["p"], gfm["p"], rtol=0, atol=1e-14 * np.max(np.abs(gfm["p"])))
    for a in range(case.dim):
        assert np.allclose(one["u"][a], gfm["u_l"][a], rtol=0, atol=1e-14)


def _outflow(case, u):
    """Net volume flux out through the domain walls."""
    h = case.h
    tot = 0.0
    for a in range(case.dim):
        ax = 2 - a
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = 0
        hi[ax] = -1
        tot += (u[a][tuple(hi)].sum() - u[a][tuple(lo)].sum()) * h ** (case.dim - 1)
    return tot


@pytest.mark.parametrize("n", [32, 64])
def test_evaporating_bubble_volume_source(n):
    """Constant mdot on the interface cells of a vapour bubble, u* = 0: the
    divergence equals S after the update, the outflow is sum S h^d, and it
    approaches both mdot (1/rho_v - 1/rho_l) 2 pi R and the ghost-fluid
    projection's outflow."""
    R, md = 0.21, 0.5
    props = ei.Props(rho_l=1.0, rho_v=0.05)
    case = ball_case(2, n, R, props)
    g = geometry.build(case)
    mdot = np.where(g["is_if"], md, 0.0)
    one = onefluid.project_one_fluid(case, g, mdot, case.u_l, solve.direct)
    S = one["S"]
    assert np.all(S[g["is_if"]] > 0) and np.all(S[~g["is_if"]] == 0)
    assert np.max(np.abs(one["div"] - S)) <= 1e-9 * np.max(S)
    out1 = _outflow(case, one["u"])
    assert abs(out1 - S.sum() * case.h ** 2) <= 1e-10 * abs(out1)
    exact = md * (1 / props.rho_v - 1 / props.rho_l) * 2 * math.pi * R
    assert abs(out1 - exact) / exact < (2e-3 if n == 32 else 5e-4)
    gfm = project.project(case, g, mdot, case.u_l, case.u_v, solve.direct)
    outg = _outflow(case, gfm["u_l"])
    assert abs(out1 - outg) / exact < 0.05
