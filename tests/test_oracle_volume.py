"""Pins for the oracle's liquid volume fraction (oracle/volume.py, 2D).

Independent references:
  * a straight interface: each cell's fraction equals the area of the cell
    on the liquid side of the exact line, integrated column by column with
    scipy's quad (the liquid height of each column is a clamped linear
    function of x; its kinks are given to quad);
  * a disc: the fractions summed over the grid give the area of the polygon
    through the markers taken in angular order (the reconstruction is that
    polygon), and approach pi R^2 at second order;
  * a horizontal line: the cut row holds the closed-form fraction;
  * no interface: every cell takes the common colour; saddles and colours
    inconsistent with the markers are rejected.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import ebit_inputs as ei
from oracle import volume
from oracle.geometry import GeometryError


def _case(n, ls):
    nn = (n, n, 1)
    h = 1.0 / n
    vcol, ccol, mk = ei.colours_and_markers(2, nn, h, ls)
    zero = [np.zeros(ei.face_shape(2, nn, a)) for a in range(2)]
    return ei.Case("vf", 2, nn, h, ei.Props(), 1e-4, [(0, 0.0)] * 4, [(1, 0.0)] * 4, mk, vcol, ccol,
                   np.zeros(ei.cell_shape(2, nn)), zero, [z.copy() for z in zero])


def _exact_line_fraction(i, j, h, m, p):
    """Area fraction of cell (i, j) where m . (x - p) >= 0 (m_y != 0)."""
    def vstar(u):  # local height of the line above the cell's bottom
        return (p[1] - m[0] * ((i + u) * h - p[0]) / m[1]) / h - j

    def length(u):
        v = vstar(u)
        return min(max(1.0 - v, 0.0), 1.0) if m[1] > 0 else min(max(v, 0.0), 1.0)

    kinks = []
    for target in (0.0, 1.0):
        # vstar(u) = target, solved for u (vstar is linear in u)
        a, b = vstar(0.0), vstar(1.0)
        if a != b:
            u = (target - a) / (b - a)
            if 0.0 < u < 1.0:
                kinks.append(u)
    val, _ = quad(length, 0.0, 1.0, points=kinks or None, epsabs=1e-14, epsrel=1e-14, limit=200)
    return val


@pytest.mark.parametrize("m,p", [((0.8, 0.6), (0.52, 0.47)), ((-0.28, 0.96), (0.41, 0.55)),
                                 ((0.6, -0.8), (0.37, 0.61)), ((-0.95, -0.31), (0.58, 0.44))])
def test_straight_line_cells_match_exact_integral(m, p):
    n = 16
    mv = np.array([m[0], m[1], 0.0])
    mv /= np.linalg.norm(mv)
    case = _case(n, ei.Plane(mv, (p[0], p[1], 0.0)))
    vf = volume.volume_fraction(case)
    h = 1.0 / n
    cut = 0
    for j in range(n):
        for i in range(n):
            ex = _exact_line_fraction(i, j, h, mv, p)
            assert abs(vf[j, i] - ex) <= 1e-12, (i, j, vf[j, i], ex)
            cut += 0.0 < ex < 1.0
    assert cut > n


def _marker_points(case):
    n, h = case.n[0], case.h
    pts = []
    mx = np.asarray(case.markers[0]).reshape(n + 1, n)
    my = np.asarray(case.markers[1]).reshape(n, n + 1)
    for j, i in zip(*np.nonzero(~np.isnan(mx))):
        pts.append(((i + mx[j, i]) * h, j * h))
    for j, i in zip(*np.nonzero(~np.isnan(my))):
        pts.append((i * h, (j + my[j, i]) * h))
    return np.asarray(pts)


@pytest.mark.parametrize("n,c,R,sign", [(32, (0.51, 0.47), 0.23, 1.0), (64, (0.5, 0.5), 0.3, -1.0),
                                        (48, (0.43, 0.56), 0.17, 1.0)])
def test_disc_total_is_marker_polygon_area(n, c, R, sign):
    case = _case(n, ei.Ball((c[0], c[1], 0.0), R, sign, 2))
    vf = volume.volume_fraction(case)
    h = 1.0 / n
    P = _marker_points(case)
    ang = np.arctan2(P[:, 1] - c[1], P[:, 0] - c[0])
    Q = P[np.argsort(ang)]
    poly = 0.5 * abs(np.sum(Q[:, 0] * np.roll(Q[:, 1], -1) - np.roll(Q[:, 0], -1) * Q[:, 1]))
    liquid = vf.sum() * h * h
    expect = 1.0 - poly if sign > 0 else poly       # sign +1: a vapour bubble
    assert abs(liquid - expect) <= 1e-12
    # the inscribed polygon's deficit: sum over chords of R^2 (t - sin t) / 2
    # ~ R^2 t^3 / 12 with chord angles t <= sqrt(2) h / R, so at most
    # pi R^2 t^2 / 6 <= pi R^2 (h / R)^2 / 3: second order in h
    assert 0.0 < math.pi * R * R - poly <= math.pi * R * R * (h / R) ** 2 / 3.0


def test_horizontal_line_row_fraction():
    n = 20
    y0 = 0.4137
    case = _case(n, ei.Plane((0.0, 1.0, 0.0), (0.5, y0, 0.0)))    # liquid above y0
    vf = volume.volume_fraction(case)
    jr = int(y0 * n)
    assert np.all(vf[:jr] == 0.0) and np.all(vf[jr + 1:] == 1.0)
    assert np.allclose(vf[jr], (jr + 1) - y0 * n, rtol=0, atol=1e-13)


def test_no_interface_and_rejections():
    case = _case(8, ei.Plane((0.0, 1.0, 0.0), (0.5, -0.5, 0.0)))  # all liquid
    assert np.all(volume.volume_fraction(case) == 1.0)
    assert volume.cell_fraction((0, 0, 0, 0), (np.nan,) * 4) == 0.0
    # a saddle: opposite corners liquid, a marker on every edge
    with pytest.raises(GeometryError):
        volume.cell_fraction((1, 0, 1, 0), (0.5, 0.5, 0.5, 0.5))
    # colours that change where there is no marker
    with pytest.raises(GeometryError):
        volume.cell_fraction((1, 0, 0, 0), (np.nan, np.nan, np.nan, 0.5))
    # a triangle: one liquid corner, markers at 0.25 (bottom) and 0.5 (left)
    assert abs(volume.cell_fraction((1, 0, 0, 0), (0.25, np.nan, np.nan, 0.5)) - 0.0625) < 1e-15
