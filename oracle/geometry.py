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


def _edge_marker_positions(case, cells):
    """For the given cells: list over the cell's edge slots (axis-major, then
    transverse offsets) of (positions [n, 3], present [n])."""
    dim, h = case.dim, case.h
    nx, ny, _ = case.n
    i, j, k = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    slots = []
    offs = [(0, 0), (1, 0), (0, 1), (1, 1)] if dim == 3 else [(0, 0), (1, 0)]
    for a in range(dim):
        m = case.markers[a]
        others = [x for x in range(dim) if x != a]
        for (b, c) in offs:
            idx = [i.copy(), j.copy(), k.copy()]
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


def _marker_count(case):
    """Number of markers on the edges of every cell (uint8, cell layout)."""
    dim = case.dim
    nz = case.n[2] if dim == 3 else 1
    cnt = np.zeros((nz, case.n[1], case.n[0]), np.uint8)
    for a in range(dim):
        has = (~np.isnan(case.markers[a])).astype(np.uint8)
        others = [x for x in range(dim) if x != a]
        offs = [(0, 0), (1, 0), (0, 1), (1, 1)] if dim == 3 else [(0, 0), (1, 0)]
        for (b, c) in offs:
            sl = [slice(0, nz), slice(0, case.n[1]), slice(0, case.n[0])]
            o = [0, 0, 0]
            o[others[0]] = b
            if dim == 3:
                o[others[1]] = c
            sl = [slice(o[2], o[2] + nz), slice(o[1], o[1] + case.n[1]), slice(o[0], o[0] + case.n[0])]
            cnt += has[tuple(sl)]
    return cnt.ravel()


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
    need = 2 if dim == 2 else 3
    is_if = _marker_count(case) >= need
    cells = np.nonzero(is_if)[0]
    cF = np.zeros((N, 3))
    nF = np.zeros((N, 3))
    slots = _edge_marker_positions(case, cells)
    P = np.stack([p for p, _ in slots], axis=1)          # [n, S, 3]
    M = np.stack([m for _, m in slots], axis=1)          # [n, S]
    cnt = M.sum(axis=1)
    Pm = np.where(M[:, :, None], P, 0.0)
    cen = Pm.sum(axis=1) / cnt[:, None]
    cF[cells] = cen
    # corners of each interface cell, in the order (dk, dj, di), and colours
    i, j, k = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    corners = []
    for dk in ((0, 1) if dim == 3 else (0,)):
        for dj in (0, 1):
            for di in (0, 1):
                col = case.vcol[k + dk if dim == 3 else np.zeros_like(k), j + dj, i + di].astype(float)
                pos = np.stack([(i + di) * h, (j + dj) * h, (k + dk) * h if dim == 3 else 0.0 * k], axis=1)
                corners.append((pos, col))
    xc = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h if dim == 3 else 0.0 * k], axis=1)
    fc = case.ccol.ravel().astype(float)[cells]

    idx = np.arange(cells.size)
    n_all = np.full((idx.size, 3), np.nan)
    # 2D cells with two markers: unit perpendicular of the segment P1 -> P2
    if dim == 2:
        two = cnt == 2
        sel = idx[two]
        # the two present slots, in slot order
        order = np.argsort(~M[sel], axis=1, kind="stable")[:, :2]
        p1 = P[sel, order[:, 0]]
        p2 = P[sel, order[:, 1]]
        d = p2 - p1
        L = np.hypot(d[:, 0], d[:, 1])
        ok = L > 0
        nn = np.full((sel.size, 3), np.nan)
        nn[ok, 0] = -d[ok, 1] / L[ok]
        nn[ok, 1] = d[ok, 0] / L[ok]
        nn[ok, 2] = 0.0
        n_all[two] = nn
        rest = ~two
    else:
        rest = np.ones(idx.size, bool)
    # otherwise: least-squares plane, eigenvector of the smallest eigenvalue
    sel = idx[rest]
    if sel.size:
        X = np.where(M[sel][:, :, None], P[sel] - cen[sel][:, None, :], 0.0)
        C = np.einsum("nsi,nsj->nij", X, X)
        if dim == 2:
            C = C[:, :2, :2]
        good = np.max(np.abs(C.reshape(sel.size, -1)), axis=1) > 0
        nn = np.full((sel.size, 3), np.nan)
        if good.any():
            w, V = np.linalg.eigh(C[good])
            v = V[:, :, 0]
            if dim == 2:
                v = np.concatenate([v, np.zeros((v.shape[0], 1))], axis=1)
            nn[good] = v / np.linalg.norm(v, axis=1)[:, None]
        n_all[rest] = nn
    # coinciding markers: direction of the corner-colour contrast
    for q in np.nonzero(np.isnan(n_all[:, 0]))[0]:
        g = sum((2 * col[q] - 1) * (pos[q] - cen[q]) for pos, col in corners)
        n_all[q] = g / np.linalg.norm(g)
    # orientation from vapour into liquid: corner colours, then the centre colour
    s = np.zeros(idx.size)
    for pos, col in corners:
        s = s + (2 * col - 1) * np.einsum("ni,ni->n", n_all, pos - cen)
    tie = s == 0
    s[tie] = (2 * fc[tie] - 1) * np.einsum("ni,ni->n", n_all[tie], xc[tie] - cen[tie])
    n_all[s < 0] *= -1
    nF[cells] = n_all
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
    ids = _cell_index(case)
    col = case.ccol
    out = []
    for a in range(case.dim):
        ax = 2 - a
        n_a = ids.shape[ax]
        fshape = list(ids.shape)
        fshape[ax] += 1
        th = np.full(fshape, np.nan)
        periodic = case.T_bc[2 * a][0] == 2
        if periodic:
            lo = ids.ravel()
            up = np.roll(ids, -1, axis=ax).ravel()
        else:
            lo = np.take(ids, np.arange(n_a - 1), axis=ax).ravel()
            up = np.take(ids, np.arange(1, n_a), axis=ax).ravel()
        cut = col.ravel()[lo] != col.ravel()[up]
        lo, up = lo[cut], up[cut]
        t_lo = (lo // _stride(case, a)) % n_a
        wrap = t_lo == n_a - 1            # the upper cell sits across the seam
        theta = _theta_links(case, a, lo, up, wrap, is_if, cF, nF)
        # the face between lower index t and t + 1; the seam also fills face 0
        th.ravel()[_face_index(case, a, lo, t_lo + 1)] = theta
        if wrap.any():
            th.ravel()[_face_index(case, a, lo[wrap], np.zeros(int(wrap.sum()), int))] = theta[wrap]
        out.append(th)
    return out


def _stride(case, a):
    nx, ny, _ = case.n
    return (1, nx, nx * ny)[a]


def _face_index(case, a, cells, t_face):
    """Flat index, in the axis-a face array, of the face at position t_face
    along a in the row of each given cell."""
    nx, ny, nz = case.n
    nzc = nz if case.dim == 3 else 1
    q = [cells % nx, (cells // nx) % ny, cells // (nx * ny)]
    q[a] = t_face
    dims = [nx, ny, nzc]
    dims[a] += 1
    return q[0] + dims[0] * (q[1] + dims[1] * q[2])


def _centres(case, cells):
    nx, ny, _ = case.n
    h = case.h
    i = cells % nx
    j = (cells // nx) % ny
    k = cells // (nx * ny)
    return np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h if case.dim == 3 else 0.0 * k], axis=1)


def _theta_links(case, a, lo, up, wrap, is_if, cF, nF):
    """theta of each cut link from the two cells' facets: candidate t from
    the lower cell's facet valid in [0, 1/2], from the upper cell's in
    [1/2, 1]; the mean of the valid ones, else the clamped mean of the
    computable ones, else 1/2.  No facet on either side: geometry error."""
    h = case.h
    if np.any(~is_if[lo] & ~is_if[up]):
        raise GeometryError("cut link with no interface cell on either side")
    xc = _centres(case, lo)
    t = np.full((lo.size, 2), np.nan)
    for side, cell in ((0, lo), (1, up)):
        n = nF[cell]
        cen = cF[cell].copy()
        if side == 1:
            cen[wrap, a] += case.n[a] * h
        ok = is_if[cell] & (np.abs(n[:, a]) >= NORMAL_EPS)
        dot = (cen[:, 0] - xc[:, 0]) * n[:, 0] + (cen[:, 1] - xc[:, 1]) * n[:, 1] + (cen[:, 2] - xc[:, 2]) * n[:, 2]
        t[ok, side] = dot[ok] / (h * n[ok, a])
    v0 = (t[:, 0] >= 0.0) & (t[:, 0] <= 0.5)
    v1 = (t[:, 1] >= 0.5) & (t[:, 1] <= 1.0)
    theta = np.full(lo.size, 0.5)
    both = v0 & v1
    theta[both] = 0.5 * (t[both, 0] + t[both, 1])
    only0 = v0 & ~v1
    theta[only0] = t[only0, 0]
    only1 = v1 & ~v0
    theta[only1] = t[only1, 1]
    none = ~v0 & ~v1
    ex = ~np.isnan(t)
    cnt = ex.sum(axis=1)
    some = none & (cnt > 0)
    mean = np.where(ex, t, 0.0).sum(axis=1)[some] / cnt[some]
    theta[some] = np.minimum(np.maximum(mean, 0.0), 1.0)
    return theta


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
