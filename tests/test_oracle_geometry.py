"""Pins for the oracle's marker -> facet -> cut-fraction pass.

Independent references: exact plane crossings (closed form), exact circle /
sphere crossings (closed form) with the O(h) convergence in cell units that
a chord / planar facet through exact markers gives, and the flag layout.
"""
import math

import numpy as np
import pytest

import ebit_inputs as ei
from oracle import geometry


def exact_theta_linear(case, phi):
    """theta from the lower cell on every cut link of a linear level set."""
    out = []
    h = case.h
    for a in range(case.dim):
        th = np.full(ei.face_shape(case.dim, case.n, a), np.nan)
        nz, ny, nx = ei.cell_shape(case.dim, case.n)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    c = np.array([(i + .5) * h, (j + .5) * h, (k + .5) * h if case.dim == 3 else 0.0])
                    d = c.copy()
                    d[a] += h
                    idx = [k, j, i]
                    idx[2 - a] += 1
                    if [i, j, k][a] + 1 >= case.n[a]:
                        continue
                    f0, f1 = phi(*c), phi(*d)
                    if (f0 >= 0) != (f1 >= 0):
                        th[tuple(idx)] = f0 / (f0 - f1)
        out.append(th)
    return out


def test_stefan_theta_and_facets():
    """C1: x_Gamma = 19.2 h -> theta = 0.7 from vapour cell 18 on every row."""
    c = ei.config(0)
    g = geometry.build(c)
    th = g["theta"][0]
    cut = ~np.isnan(th)
    assert cut.sum() == 64
    assert np.all(np.argwhere(cut)[:, 2] == 19)
    assert np.allclose(th[cut], 0.7, rtol=0, atol=1e-15)
    assert np.all(np.isnan(g["theta"][1]))
    iface = np.nonzero(g["is_if"])[0]
    assert np.all(iface % 64 == 19) and len(iface) == 64
    assert np.allclose(g["nF"][iface], [1.0, 0.0, 0.0], atol=0)
    assert np.allclose(g["cF"][iface][:, 0], 19.2 / 64, atol=1e-16)


@pytest.mark.parametrize("dim,n,seed", [(2, 16, 1), (2, 23, 2), (2, 40, 3), (3, 8, 4), (3, 11, 5), (3, 14, 6)])
def test_tilted_plane_theta_exact(dim, n, seed):
    """A plane is reproduced exactly by every facet, so theta is exact."""
    rng = np.random.default_rng(seed)
    m = rng.normal(size=3)
    if dim == 2:
        m[2] = 0
    m /= np.linalg.norm(m)
    p = 0.5 + rng.uniform(-0.1, 0.1, 3)
    ls = ei.Plane(m, p)
    nn = (n, n, n if dim == 3 else 1)
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, 1.0 / n, ls)
    case = ei.Case("plane", dim, nn, 1.0 / n, ei.Props(), 1e-4, [(0, 0.0)] * (2 * dim),
                   [(1, 0.0)] * (2 * dim), mk, vcol, ccol, np.zeros(ei.cell_shape(dim, nn)), [], [])
    g = geometry.build(case)
    ref = exact_theta_linear(case, lambda x, y, z: ls.phi(x, y, z))
    for a in range(dim):
        assert np.array_equal(np.isnan(g["theta"][a]), np.isnan(ref[a]))
        ok = ~np.isnan(ref[a])
        assert np.max(np.abs(g["theta"][a][ok] - ref[a][ok]), initial=0) < 1e-12
    # normals: the plane normal (unit, into the liquid) in every interface cell;
    # a facet through three markers a few 1e-4 h apart is conditioned ~1e-12
    iface = g["is_if"]
    assert np.max(np.abs(g["nF"][iface] - m[None, :]), initial=0) < 1e-10


def _ball_theta_error(dim, n):
    ls = ei.Ball((0.5, 0.5, 0.5), 0.3 if dim == 2 else 0.3, +1.0, dim)
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    case = ei.Case("ball", dim, nn, h, ei.Props(), 1e-4, [(0, 0.0)] * (2 * dim),
                   [(1, 0.0)] * (2 * dim), mk, vcol, ccol, np.zeros(ei.cell_shape(dim, nn)), [], [])
    g = geometry.build(case)
    err = 0.0
    for a in range(dim):
        th = g["theta"][a]
        for idx in np.argwhere(~np.isnan(th)):
            k, j, i = idx
            ci = [i, j, k]
            ci[a] -= 1
            x0 = np.array([(ci[0] + .5) * h, (ci[1] + .5) * h, (ci[2] + .5) * h if dim == 3 else 0.0])
            q = sum((x0[b] - 0.5) ** 2 for b in range(dim) if b != a)
            root = math.sqrt(0.09 - q)
            cand = [0.5 - root, 0.5 + root]
            t = [(x - x0[a]) / h for x in cand]
            t = [v for v in t if -1e-12 <= v <= 1 + 1e-12]
            assert len(t) == 1
            X = x0.copy()
            X[a] += t[0] * h
            nrm = (X - 0.5)[:dim]
            nrm /= np.linalg.norm(nrm)
            # distance error along the normal, in cells (a link almost tangent
            # to the circle turns an O(h^2) offset into a large theta error)
            err = max(err, abs(th[tuple(idx)] - t[0]) * abs(nrm[a]))
    return err


@pytest.mark.parametrize("dim,ns", [(2, (64, 128, 256)), (3, (24, 48))])
def test_ball_theta_converges_first_order_in_cells(dim, ns):
    """Crossing error along the normal is O(h) in cells, O(h^2) in position."""
    errs = [_ball_theta_error(dim, n) for n in ns]
    assert errs[0] < 0.05
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.55 * e0, errs


def test_marker_colour_mismatch_raises():
    c = ei.config(0, 16)
    c.markers[0][0, 3, 2] = 0.5       # marker on an edge whose ends agree
    with pytest.raises(geometry.GeometryError):
        geometry.link_theta(c)


def test_marker_out_of_range_raises():
    c = ei.config(0, 16)
    cut = np.argwhere(~np.isnan(c.markers[0]))[0]
    c.markers[0][tuple(cut)] = 1.5
    with pytest.raises(geometry.GeometryError):
        geometry.link_theta(c)


def test_flags_layout():
    c = ei.config(0, 16)            # x_Gamma = 4.8 cells: inside vapour cell 4
    g = geometry.build(c)
    f = g["flags"][0]
    assert np.all(f[:, 4] == 0x80 | 0b00000010)    # vapour, +x link cut, interface cell
    assert np.all(f[:, 5] == 0b01000001)           # liquid, -x link cut
    assert np.all(f[:, 6] == 0b01000000)
    assert np.all(f[:, 0] == 0)


class _Slab(ei.LevelSet):
    """Liquid within w of x0 along x, measured on the unit circle (periodic)."""

    def __init__(self, x0, w):
        self.x0, self.w = x0, w

    def phi(self, x, y, z):
        d = np.abs(np.mod(x - self.x0 + 0.5, 1.0) - 0.5)
        return self.w - d

    def root(self, a, x0, y0, z0, h, start_liquid):
        best = np.full(np.shape(x0), np.nan)
        for c in (self.x0 - self.w, self.x0 + self.w):
            for shift in (-1.0, 0.0, 1.0):
                t = (c + shift - x0) / h
                best = np.where((t >= 0) & (t <= 1), t, best)
        return best


def test_periodic_wrap_link():
    """A liquid strip whose edge sits across the periodic seam: the wrap link
    (cell n-1 -> cell 0) is cut and stored on both copies of the seam face."""
    dim, n = 2, 16
    h = 1.0 / n
    nn = (n, n, 1)
    ls = _Slab(0.2, 0.18)             # liquid on [0.02, 0.38]
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    assert np.array_equal(vcol[:, :, 0], vcol[:, :, n])
    case = ei.Case("wrap", dim, nn, h, ei.Props(), 1e-4, [(2, 0.0), (2, 0.0), (0, 0.0), (0, 0.0)],
                   [(2, 0.0), (2, 0.0), (1, 0.0), (1, 0.0)], mk, vcol, ccol,
                   np.zeros(ei.cell_shape(dim, nn)), [], [])
    g = geometry.build(case)
    th = g["theta"][0]
    assert case.ccol[0, 0, n - 1] == 0 and case.ccol[0, 0, 0] == 1
    exact = (1.02 - (n - 0.5) * h) / h       # from cell n-1 to x = 0.02 + 1
    assert np.allclose(th[:, :, 0], exact, atol=1e-12)
    assert np.array_equal(th[:, :, 0], th[:, :, n])
    exact2 = (0.38 - 5.5 * h) / h             # cells 5 (0.344) liquid, 6 (0.406) vapour
    assert np.allclose(th[:, :, 6], exact2, atol=1e-12)
    assert np.sum(~np.isnan(th)) == 3 * n
