"""Liquid volume fraction of each cell from the EBIT interface (oracle, 2D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 (Eq. property_average and the text after it) and Sec. 3.1: the
volume fraction is the integral of the Heaviside function H (1 in the
liquid) over a cell, and in 2D the paper takes it from the piecewise-linear
reconstruction of the interface by the EBIT segments.

Readings:
  * the reconstruction in a cell is the segment joining its two markers
    (the cell's facet); the liquid part of the cell is the polygon whose
    vertices are, in counter-clockwise order round the cell's boundary, its
    liquid corners (colour vertices equal to 1) and its two markers; the
    fraction is that polygon's area (shoelace formula) over h^2;
  * a cell with no marker takes the common colour of its corners (1 or 0);
  * a cell with other than 0 or 2 markers (a saddle), or whose corner
    colours do not change exactly at its markers, is rejected
    (GeometryError): the segment does not define the liquid region there.

Cell-local coordinates (x, y) in [0, 1]^2, corners counter-clockwise
(0,0), (1,0), (1,1), (0,1); the bottom edge is the x-edge of row j, the
top edge that of row j+1, the left edge the y-edge of column i, the right
edge that of column i+1; a marker s on an edge sits at fraction s from its
lower vertex.
"""
from __future__ import annotations

import numpy as np

from .geometry import GeometryError


def _polygon_area(P):
    """Shoelace area of the polygon P (k x 2, vertices in order)."""
    x, y = P[:, 0], P[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def cell_fraction(colours, marks):
    """Liquid fraction of one cell.

    colours: the corner colours in counter-clockwise order from (0,0);
    marks: the marker fractions (NaN = none) on the bottom, right, top and
    left edges, each measured from the edge's lower vertex."""
    corners = ((0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0))
    s_b, s_r, s_t, s_l = marks
    # the marker point on the edge after each corner, walking counter-clockwise
    after = ((s_b, 0.0) if not np.isnan(s_b) else None,
             (1.0, s_r) if not np.isnan(s_r) else None,
             (s_t, 1.0) if not np.isnan(s_t) else None,
             (0.0, s_l) if not np.isnan(s_l) else None)
    nm = sum(p is not None for p in after)
    for e in range(4):
        if (colours[e] != colours[(e + 1) % 4]) != (after[e] is not None):
            raise GeometryError("corner colours do not change at the cell's markers")
    if nm == 0:
        return float(colours[0])
    if nm != 2:
        raise GeometryError("a cell holds other than 0 or 2 markers")
    poly = []
    for e in range(4):
        if colours[e] == 1:
            poly.append(corners[e])
        if after[e] is not None:
            poly.append(after[e])
    return _polygon_area(np.asarray(poly, dtype=float))


def volume_fraction(case):
    """[ny, nx] liquid volume fraction of every cell of a 2D case."""
    if case.dim != 2:
        raise ValueError("the volume fraction is two-dimensional")
    nx, ny = case.n[0], case.n[1]
    vc = np.asarray(case.vcol).reshape(ny + 1, nx + 1)
    mx = np.asarray(case.markers[0]).reshape(ny + 1, nx)      # x-edges: row j, from vertex i to i+1
    my = np.asarray(case.markers[1]).reshape(ny, nx + 1)      # y-edges: column i, from vertex j to j+1
    out = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            colours = (vc[j, i], vc[j, i + 1], vc[j + 1, i + 1], vc[j + 1, i])
            # each point sits at its fraction from the edge's lower vertex
            marks = (mx[j, i], my[j, i + 1], mx[j + 1, i], my[j, i])
            out[j, i] = cell_fraction(colours, marks)
    return out
