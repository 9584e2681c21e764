"""EBIT markers -> interface facets -> link cut fractions (oracle).

Paper, Sec. 2.1: at most one marker per cell edge, markers move along grid
lines, colour vertices (corners + cell centre) give the phase (f = 1 liquid,
f = 0 vapour) and the reconstructed interface.  Sec. 2.4 (Eq. ghost_T) needs
theta = (x_Gamma - x_i)/dx along each grid link that crosses the interface,
and Eq. normal_gradient needs the interface centroid and normal per cut cell.

Readings (the paper gives theta, not its construction from markers):
  * a cell is an interface cell when its edges carry >= 2 markers (2D) or
    >= 3 markers (3D); its facet centroid is the mean of those markers;
  * the facet normal is the unit perpendicular of the two-marker segment
    (2D) or else the least-squares plane normal (eigenvector of the smallest
    eigenvalue of the marker covariance), oriented from vapour into liquid by
    the signed sum over the cell's corner colours (cell-centre colour on a
    tie); coinciding markers fall back to the corner-colour direction;
  * a link between cells of different colour is cut; its fraction theta is
    measured from the lower cell, from the candidates the two cells' facets
    give (windows [0, 1/2] from the lower cell's facet, [1/2, 1] from the
    upper cell's), averaged when both are valid, the clamped mean of the
    computable ones when none is, 1/2 when none is computable;
  * a marker must sit exactly on the edges whose end colours differ.
"""
from __future__ import annotations

import numpy as np

NORMAL_EPS = 1e-12


class GeometryError(ValueError):
    pass


def _edge_marker_positions(case):
    """List of (positions [ncell, 3], present [ncell]) per cell edge slot."""
    dim, h = case.dim, case.h
    nx, ny, nz = case.n
    nzc = nz if dim == 3 else 1
    k, j, i = np.meshgrid(np.arange(nzc), np.arange(ny), np.arange(nx), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    slots = []
    offs = [(0, 0), (1, 0), (0, 1), (1, 1)] if dim == 3 else [(0, 0), (1, 0)]
    for a in range(dim):
        m = case.markers[a]
        for (b, c) in offs:
            # transverse offsets: the two other axes (in increasing order)
            ii, jj, kk = i.copy(), j.copy(), k.copy()
            others = [x for x in range(dim) if x != a]
            idx = [ii, jj, kk]
            idx[others[0]] = idx[others[0]] + b
            if dim == 3:
                idx[others[1]] = idx[others[1]] + c
            ii, jj, kk = idx
            s = m[kk if dim == 3 else np.zeros_like(kk), jj, ii]
            pos = np.stack([ii * h, jj * h, kk * h], axis=1).astype(float)
            if dim == 2:
                pos[:, 2] = 0.0
            pos[:, a] = pos[:, a] + np.where(np.isnan(s), 0.0, s) * h
            slots.append((pos, ~np.isnan(s)))
    return slots


def check_markers(case):
    """Marker present on an edge  <=>  the edge's end colours differ."""
    for a in range(case.dim):
        v = case.vcol.astype(int)
        es = case.markers[a].shape
        lo = v[:es[0], :es[1], :es[2]]
        sl = [slice(0, es[0]), slice(0, es[1]), slice(0, es[2])]
        sl[2 - a] = slice(1, es[2 - a] + 1)
        hi = v[tuple(sl)]
        has = ~np.isnan(case.markers[a])
        if np.any(has != (lo != hi)):
            raise GeometryError(f"axis {a}: markers inconsistent with vertex colours")
        s = case.markers[a][has]
        if np.any((s < 0) | (s > 1)):
            raise GeometryError(f"axis {a}: marker outside [0, 1]")
    for a in range(case.dim):
        if case.T_bc[2 * a][0] != 2:
            continue
        # a periodic axis: the vertex layer at n_a is the layer at 0
        ax = 2 - a
        first = np.take(case.vcol, 0, axis=ax)
        last = np.take(case.vcol, case.vcol.shape[ax] - 1, axis=ax)
        if not np.array_equal(first, last):
            raise GeometryError(f"axis {a}: periodic vertex colours differ across the seam")
        for b in range(case.dim):
            if b == a:
                continue
            m = case.markers[b]
            m0 = np.take(m, 0, axis=ax)
            m1 = np.take(m, m.shape[ax] - 1, axis=ax)
            if not np.array_equal(m0, m1, equal_nan=True):
                raise GeometryError(f"axis {a}: periodic markers differ across the seam")


def facets(case):
    """Per-cell facet: (is_iface [N] bool, cF [N,3], nF [N,3]); N = cells.

    Sec. 2.1 (markers, colour vertices) and Sec. 2.4 (interface centroid and
    normal used by the normal-gradient stencil).  Normal from vapour into
    liquid.
    """
    dim, h = case.dim, case.h
    nx, ny, nz = case.n
    nzc = nz if dim == 3 else 1
    N = nx * ny * nzc
    slots = _edge_marker_positions(case)
    P = np.stack([p for p, _ in slots], axis=1)          # [N, S, 3]
    M = np.stack([m for _, m in slots], axis=1)          # [N, S]
    cnt = M.sum(axis=1)
    need = 2 if dim == 2 else 3
    is_if = cnt >= need
    cF = np.zeros((N, 3))
    nF = np.zeros((N, 3))
    Pm = np.where(M[:, :, None], P, 0.0)
    cF[is_if] = Pm[is_if].sum(axis=1) / cnt[is_if][:, None]

    # corner positions and colours of every cell
    k, j, i = np.meshgrid(np.arange(nzc), np.arange(ny), np.arange(nx), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    corners = []
    for dk in ((0, 1) if dim == 3 else (0,)):
        for dj in (0, 1):
            for di in (0, 1):
                col = case.vcol[k + dk if dim == 3 else np.zeros_like(k), j + dj, i + di].astype(float)
                pos = np.stack([(i + di) * h, (j + dj) * h, (k + dk) * h if dim == 3 else 0.0 * k], axis=1)
                corners.append((pos, col))
    xc = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h if dim == 3 else 0.0 * k], axis=1)
    fc = case.ccol.ravel().astype(float)

    for c in np.nonzero(is_if)[0]:
        pts = P[c][M[c]]
        cen = cF[c]
        n = None
        if dim == 2 and len(pts) == 2:
            d = pts[1] - pts[0]
            L = np.hypot(d[0], d[1])
            if L > 0:
                n = np.array([-d[1], d[0], 0.0]) / L
        else:
            X = pts - cen
            C = X.T @ X
            if dim == 2:
                C = C[:2, :2]
            if np.max(np.abs(C)) > 0:
                w, V = np.linalg.eigh(C)
                v = V[:, 0]
                n = np.array([v[0], v[1], 0.0]) if dim == 2 else v.copy()
                n /= np.linalg.norm(n)
        if n is None:
            # all markers coincide: direction of the corner-colour contrast
            g = sum((2 * col[c] - 1) * (pos[c] - cen) for pos, col in corners)
            n = g / np.linalg.norm(g)
        s = sum((2 * col[c] - 1) * np.dot(n, pos[c] - cen) for pos, col in corners)
        if s == 0:
            s = (2 * fc[c] - 1) * np.dot(n, xc[c] - cen)
        if s < 0:
            n = -n
        nF[c] = n
    return is_if, cF, nF


def _cell_index(case):
    nx, ny, nz = case.n
    nzc = nz if case.dim == 3 else 1
    return np.arange(nx * ny * nzc).reshape(nzc, ny, nx)


def link_theta(case, fac=None):
    """Cut fraction theta per face (measured from the lower cell), NaN if the
    link is not cut.  Returns list of dim face arrays.  Eq. ghost_T defines
    theta = (x_Gamma - x_i)/dx on the link."""
    check_markers(case)
    if fac is None:
        fac = facets(case)
    is_if, cF, nF = fac
    dim, h = case.dim, case.h
    ids = _cell_index(case)
    col = case.ccol
    out = []
    for a in range(dim):
        ax = 2 - a
        n_a = ids.shape[ax]
        fshape = list(ids.shape)
        fshape[ax] += 1
        th = np.full(fshape, np.nan)
        periodic = case.T_bc[2 * a][0] == 2
        # links (lower cell at index t, upper at t+1) ; wrap link when periodic
        lo_list = list(range(n_a - 1)) + ([n_a - 1] if periodic else [])
        for t in lo_list:
            up = (t + 1) % n_a
            c = np.take(ids, t, axis=ax).ravel()
            nb = np.take(ids, up, axis=ax).ravel()
            cc = np.take(col, t, axis=ax).ravel()
            cn = np.take(col, up, axis=ax).ravel()
            vals = np.full(c.shape, np.nan)
            for q in np.nonzero(cc != cn)[0]:
                vals[q] = _theta_one(case, a, c[q], nb[q], is_if, cF, nF, wrap=(up == 0))
            sl = [slice(None)] * 3
            sl[ax] = t + 1
            th[tuple(sl)] = vals.reshape(np.take(th, t + 1, axis=ax).shape)
            if periodic and up == 0:
                sl[ax] = 0
                th[tuple(sl)] = vals.reshape(np.take(th, 0, axis=ax).shape)
        out.append(th)
    return out


def _centre(case, c):
    nx, ny, nz = case.n
    i = c % nx
    j = (c // nx) % ny
    k = c // (nx * ny)
    h = case.h
    return np.array([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h if case.dim == 3 else 0.0])


def _theta_one(case, a, c, nb, is_if, cF, nF, wrap=False):
    h = case.h
    xc = _centre(case, c)
    cands = []    # (value, valid)
    for cell, lo_hi in ((c, 0), (nb, 1)):
        if not is_if[cell]:
            continue
        n = nF[cell]
        if abs(n[a]) < NORMAL_EPS:
            cands.append((None, False, True))
            continue
        cen = cF[cell].copy()
        if lo_hi == 1 and wrap:
            cen[a] += case.n[a] * h
        t = np.dot(cen - xc, n) / (h * n[a])
        ok = (0.0 <= t <= 0.5) if lo_hi == 0 else (0.5 <= t <= 1.0)
        cands.append((t, ok, True))
    if not cands:
        raise GeometryError("cut link with no interface cell on either side")
    valid = [t for t, ok, _ in cands if ok]
    if len(valid) == 1:
        return valid[0]
    if len(valid) == 2:
        return 0.5 * (valid[0] + valid[1])
    exist = [t for t, _, _ in cands if t is not None]
    if exist:
        return min(max(sum(exist) / len(exist), 0.0), 1.0)
    return 0.5


def flags(case, theta, is_if):
    """Cell flag byte: bits 0..5 = cut link on side (-x,+x,-y,+y,-z,+z),
    bit 6 = liquid, bit 7 = interface cell (carries a facet)."""
    dim = case.dim
    f = (case.ccol.astype(np.uint8) << 6) | (is_if.reshape(case.ccol.shape).astype(np.uint8) << 7)
    for a in range(dim):
        ax = 2 - a
        cut = ~np.isnan(theta[a])
        n_a = f.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n_a)
        hi[ax] = slice(1, n_a + 1)
        f |= (cut[tuple(lo)].astype(np.uint8) << (2 * a))
        f |= (cut[tuple(hi)].astype(np.uint8) << (2 * a + 1))
    return f


def build(case):
    """All geometry for one case: dict with is_if, cF, nF, theta, flags."""
    fac = facets(case)
    th = link_theta(case, fac)
    fl = flags(case, th, fac[0])
    return dict(is_if=fac[0], cF=fac[1], nF=fac[2], theta=th, flags=fl)
