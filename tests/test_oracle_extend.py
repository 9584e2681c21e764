"""Pins for the oracle's narrow-band extension (Eq. extrapolation).

Independent references:
  * an axis-aligned plane: the band normal is exactly the axis, so every row
    of cells is a one-dimensional upwind chain whose iterates have a closed
    form (geometric decay mu^t, mu = 1 - 1/d, of the head's deviation from
    its upwind data value; mu^t e2 + t (1 - mu) mu^(t-1) e1 for the cell
    behind it), and the band is exactly the three columns around the cut
    cells;
  * a field that is constant along the normal of a straight interface is a
    fixed point of the transport equation (its steady state), so the
    iteration must leave it unchanged;
  * the scheme is monotone, and a constant carried from the cut cells fills
    the band with that constant;
  * band membership and band normals by brute force (plain loops over every
    cell's 3^d block) on tiny grids.
"""
import math

import numpy as np
import pytest

import ebit_inputs as ei
from oracle import extend, geometry


def plane_case(dim, n, m, p, periodic=False):
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    ls = ei.Plane(np.asarray(m, float), np.asarray(p, float))
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    bc = [(2 if periodic else 0, 0.0)] * (2 * dim)
    # periodic only across the axes the interface does not cut
    if periodic:
        bc[0] = bc[1] = (0, 0.0)
    return ei.Case("plane", dim, nn, h, ei.Props(), 1e-4, bc, bc, mk, vcol, ccol,
                   np.zeros(ei.cell_shape(dim, nn)), [], []), ls


def ball_case(dim, n, c, R, sign, periodic=False):
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    ls = ei.Ball(np.asarray(c, float), R, sign, dim)
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    bc = [(2 if periodic else 0, 0.0)] * (2 * dim)
    return ei.Case("ball", dim, nn, h, ei.Props(), 1e-4, bc, bc, mk, vcol, ccol,
                   np.zeros(ei.cell_shape(dim, nn)), [], [])


def chain_value(mu, t, e_head0, e_tail0=None):
    """Deviation after t steps of the head of an upwind chain (data ahead of
    it) and, if given, of the cell behind the head."""
    head = mu ** t * e_head0
    if e_tail0 is None:
        return head
    tail = mu ** t * e_tail0 + (t * (1 - mu) * mu ** (t - 1) * e_head0 if t > 0 else 0.0)
    return head, tail


@pytest.mark.parametrize("dim,n,xg,periodic", [(2, 32, 0.3, False), (2, 20, 0.52, True),
                                               (3, 12, 0.37, False), (3, 10, 0.64, True)])
@pytest.mark.parametrize("t", [0, 1, 2, 5, 17])
def test_axis_plane_closed_form(dim, n, xg, periodic, t):
    case, _ = plane_case(dim, n, (1.0, 0.0, 0.0), (xg, 0.0, 0.0), periodic)
    g = geometry.build(case)
    shape = ei.cell_shape(dim, case.n)
    N = int(np.prod(shape))
    col = np.arange(N) % n
    iface_cols = np.unique(col[g["is_if"]])
    assert iface_cols.size == 1
    ig = int(iface_cols[0])
    inb, nb = extend.band(case, g)
    assert np.array_equal(inb, np.isin(col, [ig - 1, ig, ig + 1]))
    assert np.array_equal(nb[inb], np.tile([1.0, 0.0, 0.0], (inb.sum(), 1)))
    liquid_ig = (ig + 0.5) * case.h >= xg
    rng = np.random.default_rng(7 + t)
    q0 = rng.uniform(-2.0, 3.0, N)
    mu = 1.0 - 1.0 / dim

    def at(f, c):
        return f[col == c]

    for mode in (extend.LIQ_TO_VAP, extend.VAP_TO_LIQ, extend.IFACE_TO_BAND):
        q = extend.extend(case, g, q0, mode, t)
        # expected: (target columns -> (data column it chains from), head first)
        if mode == extend.IFACE_TO_BAND:
            chains = [([ig - 1], ig), ([ig + 1], ig)]
        elif (mode == extend.LIQ_TO_VAP) == liquid_ig:
            # the cut column holds data: one target column on the far side
            chains = [([ig - 1], ig)] if mode == extend.LIQ_TO_VAP else [([ig + 1], ig)]
        else:
            # the cut column is a target: a chain of two from the data beyond it
            chains = [([ig, ig - 1], ig + 1)] if mode == extend.LIQ_TO_VAP else [([ig, ig + 1], ig - 1)]
        touched = set()
        for cols, src in chains:
            ref = at(q0, src)
            assert np.array_equal(at(q, src), ref)
            e_head = at(q0, cols[0]) - ref
            if len(cols) == 1:
                exp = ref + chain_value(mu, t, e_head)
                assert np.allclose(at(q, cols[0]), exp, rtol=0, atol=1e-13)
            else:
                eh, et = chain_value(mu, t, e_head, at(q0, cols[1]) - ref)
                assert np.allclose(at(q, cols[0]), ref + eh, rtol=0, atol=1e-13)
                assert np.allclose(at(q, cols[1]), ref + et, rtol=0, atol=1e-13)
            touched |= set(cols)
        rest = ~np.isin(col, sorted(touched))
        assert np.array_equal(q[rest], q0[rest])


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 14)])
def test_field_constant_along_normal_is_fixed(dim, n):
    """A straight interface with normal (1,1[,1])/sqrt(d): q = x - y (2D) or
    x - z plus y - z (3D) does not vary along the normal."""
    m = np.array([1.0, 1.0, 1.0 if dim == 3 else 0.0])
    m /= np.linalg.norm(m)
    case, _ = plane_case(dim, n, m, (0.513, 0.5, 0.5))
    g = geometry.build(case)
    shape = ei.cell_shape(dim, case.n)
    N = int(np.prod(shape))
    idx = np.arange(N)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    h = case.h
    x, y, z = (i + .5) * h, (j + .5) * h, (k + .5) * h
    q0 = 3.0 * (x - y) + 0.25 if dim == 2 else 2.0 * (x - z) - (y - z) + 0.25
    inb, nb = extend.band(case, g)
    # every band normal is the plane normal (to rounding)
    assert np.max(np.abs(nb[inb] - m[None, :])) < 1e-13
    # away from the walls (where terms drop out) nothing moves
    inner = np.ones(N, bool)
    for c in (i, j, k)[:dim]:
        inner &= (c >= 4) & (c < n - 4)
    for mode in (extend.LIQ_TO_VAP, extend.VAP_TO_LIQ, extend.IFACE_TO_BAND):
        q = extend.extend(case, g, q0, mode, 30)
        assert np.max(np.abs(q - q0)[inner & inb]) < 1e-12
    # and a field that varies along the normal does move
    q = extend.extend(case, g, x + y, extend.LIQ_TO_VAP, 3)
    assert np.max(np.abs(q - (x + y))[inner & inb]) > 1e-3


@pytest.mark.parametrize("dim,n,periodic", [(2, 40, False), (2, 33, True), (3, 16, False), (3, 15, True)])
def test_monotone_and_constant_fill(dim, n, periodic):
    case = ball_case(dim, n, (0.47, 0.52, 0.5), 0.27, 1.0 if n % 2 else -1.0, periodic)
    g = geometry.build(case)
    N = int(np.prod(ei.cell_shape(dim, case.n)))
    rng = np.random.default_rng(n)
    q0 = rng.uniform(-1.0, 1.0, N)
    liquid = case.ccol.ravel().astype(bool)
    is_if = g["is_if"]
    inb, _ = extend.band(case, g)
    for mode, data in ((extend.LIQ_TO_VAP, liquid), (extend.VAP_TO_LIQ, ~liquid),
                       (extend.IFACE_TO_BAND, is_if)):
        known = data | inb
        q1 = extend.extend(case, g, q0, mode, 1)
        assert q1[known].max() <= q0[known].max() and q1[known].min() >= q0[known].min()
        assert np.array_equal(q1[data], q0[data])
        assert np.array_equal(q1[~known], q0[~known])
    # a constant on the cut cells fills the whole band
    q = np.where(is_if, 0.75, q0)
    out = extend.extend(case, g, q, extend.IFACE_TO_BAND, 200)
    assert np.max(np.abs(out[inb] - 0.75)) < 1e-12
    assert np.array_equal(out[~inb], q[~inb])


@pytest.mark.parametrize("dim,n,periodic", [(2, 11, False), (2, 9, True), (3, 7, False), (3, 6, True)])
def test_band_brute_force(dim, n, periodic):
    """Band membership and band normals by plain loops over cells and their
    3^d blocks on tiny grids (a tilted plane crosses the blocks diagonally)."""
    m = np.array([0.8, 0.5, 0.33 if dim == 3 else 0.0])
    m /= np.linalg.norm(m)
    case, _ = plane_case(dim, n, m, (0.47, 0.5, 0.5))
    if periodic:
        case = ball_case(dim, n, (0.5, 0.45, 0.5), 0.3, -1.0, True)
    g = geometry.build(case)
    is_if = g["is_if"]
    nF = g["nF"]
    inb, nb = extend.band(case, g)
    nz = n if dim == 3 else 1
    per = [case.T_bc[2 * a][0] == 2 for a in range(dim)]
    diag_only = 0
    for k in range(nz):
        for j in range(n):
            for i in range(n):
                c = i + n * (j + n * k)
                hit, face_hit = False, False
                s = [0.0, 0.0, 0.0]
                for dk in ((-1, 0, 1) if dim == 3 else (0,)):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            q = [i + di, j + dj, k + dk]
                            ok = True
                            for a in range(dim):
                                if per[a]:
                                    q[a] %= n
                                elif not 0 <= q[a] < n:
                                    ok = False
                            if not ok:
                                continue
                            mcell = q[0] + n * (q[1] + n * q[2])
                            if is_if[mcell]:
                                hit = True
                                face_hit |= abs(di) + abs(dj) + abs(dk) <= 1
                                for r in range(3):
                                    s[r] += nF[mcell][r]
                assert inb[c] == hit, (i, j, k)
                diag_only += hit and not face_hit
                L = math.sqrt(sum(v * v for v in s))
                if hit and L > 0:
                    assert np.allclose(nb[c], [v / L for v in s], rtol=0, atol=1e-15)
                else:
                    assert not np.any(nb[c])
    # the case really has cells reached only through a block corner or edge
    assert diag_only > 0
