"""EBIT marker motion and the interfacial velocity (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1, Eqs. marker_motion and discrete_marker_motion: each marker moves
with the interfacial velocity by an explicit Euler step, one dimension after
the other (x, then y).  In a 1D pass along axis a the aligned markers (on
the grid lines along a) move along their line; the unaligned ones (on lines
across a) leave their lines, and the interface they carry is cut again by
the unaligned grid edges.  The colour vertices follow the interface.
Sec. 2.3, Eq. jump_interfacial_vel: the interfacial velocity at a cell
centre is the velocity of the cell's own phase less the mass flux over that
phase's density times the normal; at a marker it is the bilinear
interpolation of the four nearest cell centres.  The cell-centre field is
computed in 2D and 3D; the marker motion is two-dimensional (the EBIT
method of the paper is).

Readings (the paper defers the re-intersection to the EBIT papers):
  * R21 re-intersection: each interface cell's segment joins its two
    markers, and every marker of the pass moves by its own displacement.
    An unaligned edge holds a marker after the pass when its end vertices
    differ in colour (the colour vertices decide the topology).  The marker
    sits where the moved interface meets the edge's line: for each moved
    segment that reaches the line (an end point on the line counts for each
    segment that holds it), the circles through the segment and the far end
    of each neighbouring segment are met with the line on the arc between
    the segment's ends, and their mean is taken (the chord where the
    interface has no neighbour); several segments give the mean of theirs,
    none the edge's midpoint.  Straight lines and circles are moved exactly.
    Cells with other than 0 or 2 markers (saddles) are rejected.
  * R22 the cell-centred velocity of phase k is the mean of the cell's two
    faces per axis in the phase-k face field (the cell's own colour).
  * R23 at a cell centre, the normal is the band normal of the extension
    (normalised sum of the facet normals of the 3^d block) and the mass
    flux the caller's cell field (the interface cells' value carried into
    the band by Eq. extrapolation).
  * R24 sign: with n from vapour into liquid (R1), u_G = u_k + (mdot/rho_k) n;
    the paper's n in Eq. jump_interfacial_vel points into the vapour, as in
    Eq. mass_flux.
  * R25 an aligned marker at x1 = x0 + u_G dt lands on the edge of its line
    that holds x1 (the last edge for a point on the far wall; walls clamp
    x1 to the domain, periodic axes wrap it); two markers landing on one
    edge cancel (one marker per edge at most).  The vertices after the old
    edge up to the new one (or after the new one up to the old one) change
    colour, once per marker.
  * R26 the second pass interpolates the same cell-centre field (the flow
    at time level n) at the markers' new positions.
  * R28 a marker on a wall across the pass axis (x_a = 0 or x_a = n_a h on
    a non-periodic axis) keeps x_a: no flow crosses a wall, while the
    interpolated velocity there need not vanish.
  * R27 a cell whose corners agree takes their colour; a cell with two
    markers takes, at its centre, the side of its segment's line that the
    corner colours mark as liquid (a centre on the line is liquid).

Bilinear stencil: the four centres around the point, kept inside
non-periodic walls (the point is then extrapolated linearly from the
nearest centres); periodic axes wrap.
"""
from __future__ import annotations

import math

import numpy as np

from . import extend
from .geometry import GeometryError


def _dims(case):
    if case.dim != 2:
        raise ValueError("EBIT marker motion is two-dimensional")
    nx, ny, _ = case.n
    return nx, ny


def _periodic(case):
    return [case.T_bc[2 * a][0] == 2 for a in range(2)]


def cell_velocity(case, u_l, u_v):
    """[N, dim]: each cell's velocity in its own phase field, the mean of
    its two faces per axis (R22)."""
    dim = case.dim
    shp = tuple(int(x) for x in np.asarray(case.ccol).shape)
    col = np.asarray(case.ccol).reshape(shp).astype(bool)
    out = np.zeros((col.size, dim))
    for a in range(dim):
        ax = 2 - a                       # numpy axis of grid axis a
        lo = [slice(None)] * 3
        up = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        up[ax] = slice(1, None)
        fl = np.asarray(u_l[a]).reshape(shp[:ax] + (shp[ax] + 1,) + shp[ax + 1:])
        fv = np.asarray(u_v[a]).reshape(fl.shape)
        cl = 0.5 * (fl[tuple(lo)] + fl[tuple(up)])
        cv = 0.5 * (fv[tuple(lo)] + fv[tuple(up)])
        out[:, a] = np.where(col, cl, cv).ravel()
    return out


def cell_interface_velocity(case, geo, u_l, u_v, mdot):
    """[N, dim]: Eq. jump_interfacial_vel at every cell centre (R22-R24);
    off the band the normal is zero and the cell keeps its own velocity."""
    pr = case.props
    u = cell_velocity(case, u_l, u_v)
    _, n = extend.band(case, geo)
    col = np.asarray(case.ccol).ravel().astype(bool)
    rho = np.where(col, pr.rho_l, pr.rho_v)
    m = np.asarray(mdot, dtype=float).ravel()
    return u + (m / rho)[:, None] * n[:, :case.dim]


def interpolate(case, ug, P):
    """Bilinear interpolation of the cell-centre field ug [N, 2] at points
    P [m, 2] from the four nearest centres (the paper's cells 1-4)."""
    nx, ny = _dims(case)
    h = case.h
    per = _periodic(case)
    P = np.atleast_2d(np.asarray(P, dtype=float))
    idx, w = [], []
    for a, n_a in ((0, nx), (1, ny)):
        t = P[:, a] / h - 0.5
        c0 = np.floor(t).astype(int)
        f = t - c0
        if per[a]:
            c1 = np.mod(c0 + 1, n_a)
            c0 = np.mod(c0, n_a)
        else:
            lo = c0 < 0
            c0 = np.where(lo, 0, c0)
            f = np.where(lo, t, f)
            hi = c0 > n_a - 2
            f = np.where(hi, t - (n_a - 2), f)
            c0 = np.where(hi, n_a - 2, c0)
            c1 = c0 + 1
        idx.append((c0, c1))
        w.append(f)
    (i0, i1), (j0, j1) = idx
    fx, fy = w
    g = ug.reshape(ny, nx, 2)
    return ((1 - fx)[:, None] * (1 - fy)[:, None] * g[j0, i0] + (1 - fx)[:, None] * fy[:, None] * g[j1, i0]
            + fx[:, None] * (1 - fy)[:, None] * g[j0, i1] + (fx * fy)[:, None] * g[j1, i1])


def marker_points(case, markers, a):
    """(rows, cols, positions [m, 2]) of the markers on the axis-a edges."""
    h = case.h
    m = np.asarray(markers[a])[0]
    jj, ii = np.nonzero(~np.isnan(m))
    s = m[jj, ii]
    if a == 0:
        P = np.stack([(ii + s) * h, jj * h], axis=1)
    else:
        P = np.stack([ii * h, (jj + s) * h], axis=1)
    return jj, ii, P


def marker_velocities(case, geo, u_l, u_v, mdot):
    """Eq. jump_interfacial_vel at the cell centres, interpolated to every
    marker: list over the edge axes of [m, 2] (markers in np.nonzero order)."""
    ug = cell_interface_velocity(case, geo, u_l, u_v, mdot)
    return [interpolate(case, ug, marker_points(case, case.markers, a)[2]) for a in range(2)], ug


def _cell_segments(case, markers):
    """Per interface cell (0 or 2 markers): its two markers as
    (edge axis, row, col) pairs; raises for other counts (saddles)."""
    nx, ny = _dims(case)
    mx = np.asarray(markers[0])[0]
    my = np.asarray(markers[1])[0]
    segs = {}
    for j in range(ny):
        for i in range(nx):
            ends = []
            for (a, r, c) in ((0, j, i), (0, j + 1, i), (1, j, i), (1, j, i + 1)):
                m = mx if a == 0 else my
                if not np.isnan(m[r, c]):
                    ends.append((a, r, c))
            if len(ends) == 2:
                segs[(j, i)] = ends
            elif len(ends) != 0:
                raise GeometryError(f"cell ({i}, {j}) holds {len(ends)} markers")
    return segs


def _neighbour_end(case, segs, moved, cell, key):
    """The far end of the segment that continues the cell's segment through
    its marker `key` (the other marker of the cell across that marker's
    edge), in the cell's own frame; None where the interface ends on a wall
    or the neighbour holds no segment."""
    nx, ny = _dims(case)
    per = _periodic(case)
    h = case.h
    j, i = cell
    e, r, c = key
    if e == 0:
        dj, di = (-1, 0) if r == j else (1, 0)
    else:
        dj, di = (0, -1) if c == i else (0, 1)
    jn, in_ = j + dj, i + di
    shift = np.zeros(2)
    if not 0 <= in_ < nx:
        if not per[0]:
            return None
        shift[0] = (in_ - in_ % nx) * h
        in_ %= nx
    if not 0 <= jn < ny:
        if not per[1]:
            return None
        shift[1] = (jn - jn % ny) * h
        jn %= ny
    other = segs.get((jn, in_))
    if other is None:
        return None
    # the shared edge as the neighbour indexes it
    if dj == -1:
        shared = (0, jn + 1, in_)
    elif dj == 1:
        shared = (0, jn, in_)
    elif di == -1:
        shared = (1, jn, in_ + 1)
    else:
        shared = (1, jn, in_)
    far = [k for k in other if k != shared]
    if len(far) != 1:
        return None
    return moved[far[0]] + shift


def _arc_point(A, B, C, a, xg):
    """Where the arc from A to B of the circle through A, B and C meets the
    line x_a = xg (A and B on either side of it, or on it).

    In the chord frame (u along A->B, w across it) the arc is
    w(u) = -2 k q / (1 + sqrt(1 + 4 k^2 q)),  q = u (L - u),  k = w_C / D,
    D = w_C^2 + u_C (u_C - L), which stays finite as C approaches the chord
    (k -> 0 is the chord itself).  The chord crossing starts four Newton
    steps on x_a(u) = xg."""
    dx, dy = B[0] - A[0], B[1] - A[1]
    L = math.sqrt(dx * dx + dy * dy)
    tx, ty = dx / L, dy / L
    nx_, ny_ = -ty, tx
    cx, cy = C[0] - A[0], C[1] - A[1]
    uc = cx * tx + cy * ty
    wc = cx * nx_ + cy * ny_
    D = wc * wc + uc * (uc - L)
    k = wc / D if D != 0.0 else 0.0
    ta = tx if a == 0 else ty
    na = nx_ if a == 0 else ny_
    Aa = A[0] if a == 0 else A[1]
    u = (xg - Aa) / ta
    u = min(max(u, 0.0), L)
    w = 0.0
    for _ in range(4):
        q = u * (L - u)
        S = math.sqrt(1.0 + 4.0 * k * k * q)
        w = -2.0 * k * q / (1.0 + S)
        dwdq = -2.0 * k / (1.0 + S) * (1.0 - 2.0 * k * k * q / (S * (1.0 + S)))
        f = Aa + u * ta + w * na - xg
        fp = ta + dwdq * (L - 2.0 * u) * na
        if fp != 0.0:
            u = min(max(u - f / fp, 0.0), L)
    q = u * (L - u)
    w = -2.0 * k * q / (1.0 + math.sqrt(1.0 + 4.0 * k * k * q))
    return (A[1] + u * ty + w * ny_) if a == 0 else (A[0] + u * tx + w * nx_)


def _crossing(p1, p2, q1, q2, a, xg):
    """The coordinate across a of the interface between p1 and p2 on the
    line x_a = xg: the mean over the circles through (q1, p1, p2) and
    (p1, p2, q2) that exist, else the chord."""
    vals = []
    if q1 is not None:
        vals.append(_arc_point(p1, p2, q1, a, xg))
    if q2 is not None:
        vals.append(_arc_point(p1, p2, q2, a, xg))
    if not vals:
        b = 1 - a
        return p1[b] + (xg - p1[a]) * (p2[b] - p1[b]) / (p2[a] - p1[a])
    return vals[0] if len(vals) == 1 else 0.5 * (vals[0] + vals[1])


def _wrap(x, L):
    """A coordinate moved by less than one period, wrapped into [0, L)."""
    if x < 0.0:
        return x + L
    if x >= L:
        return x - L
    return x


def _landing(x1, n_a, h, per):
    """Edge index (unwrapped on a periodic axis) and fraction of an aligned
    marker at the new coordinate x1 (R25)."""
    L = n_a * h
    if per:
        xw = _wrap(x1, L)
        k = min(int(np.floor(xw / h)), n_a - 1)
        shift = int(round((x1 - xw) / L)) * n_a
        return k + shift, xw / h - k
    xc = min(max(x1, 0.0), L)
    k = min(int(np.floor(xc / h)), n_a - 1)
    return k, xc / h - k


def advect_pass(case, markers, vcol, ug, dt, a):
    """One 1D pass along axis a (R21, R25, R26): returns the new marker
    arrays and vertex colours."""
    nx, ny = _dims(case)
    h = case.h
    n = (nx, ny)
    per = _periodic(case)[a]
    b = 1 - a
    old = [np.asarray(m)[0] for m in markers]
    vc = np.asarray(vcol)[0].astype(int).copy()
    segs = _cell_segments(case, markers)
    # every marker of both families moves along a by u_G,a dt (R26); one on
    # a wall across a stays on it (R28)
    L = n[a] * h
    moved = {}
    for e in range(2):
        jj, ii, P = marker_points(case, markers, e)
        u = interpolate(case, ug, P)[:, a]
        for r, c, uu, p in zip(jj, ii, u, P):
            q = p.copy()
            if per or (p[a] != 0.0 and p[a] != L):
                q[a] = p[a] + uu * dt
            moved[(e, r, c)] = q
    new = [np.full_like(old[0], np.nan), np.full_like(old[1], np.nan)]
    # aligned markers: along their own line (R25)
    al = old[a]
    nlines = al.shape[0] if a == 0 else al.shape[1]
    per_b = _periodic(case)[b]
    for line in range(nlines):
        if per_b and line == n[b]:
            continue                         # the seam line: a copy of line 0, below
        land = {}
        for e_idx in range(n[a]):
            r, c = (line, e_idx) if a == 0 else (e_idx, line)
            if np.isnan(al[r, c]):
                continue
            k, s = _landing(moved[(a, r, c)][a], n[a], h, per)
            # the vertices between the old edge and the new one change colour
            passed = range(e_idx + 1, k + 1) if k > e_idx else range(k + 1, e_idx + 1)
            for v in passed:
                vv = v % n[a] if per else v
                rv, cv = (line, vv) if a == 0 else (vv, line)
                vc[rv, cv] ^= 1
                if per and vv == 0:          # the seam vertex is stored twice
                    rv2, cv2 = (line, n[a]) if a == 0 else (n[a], line)
                    vc[rv2, cv2] ^= 1
            land.setdefault(k % n[a] if per else k, []).append(s)
        for k, ss in land.items():
            if len(ss) == 1:                 # two markers on one edge cancel
                r, c = (line, k) if a == 0 else (k, line)
                new[a][r, c] = ss[0]
    if per_b:
        # the seam line across b is line 0 stored twice
        if a == 0:
            new[a][n[b], :] = new[a][0, :]
            vc[n[b], :] = vc[0, :]
        else:
            new[a][:, n[b]] = new[a][:, 0]
            vc[:, n[b]] = vc[:, 0]
    # unaligned markers (R21): an unaligned edge holds a marker when its end
    # vertices (on aligned lines) now differ in colour; the marker sits at
    # the mean of the crossings of the moved interface with the edge's line,
    # each found on the arcs fitted through a moved segment and its
    # neighbours
    cross = {}
    for (j, i), ends in segs.items():
        p1, p2 = (moved[key] for key in ends)
        if p1[a] == p2[a]:
            continue
        lo, hi = min(p1[a], p2[a]), max(p1[a], p2[a])
        row = j if a == 0 else i             # the cell's index across a
        q1 = _neighbour_end(case, segs, moved, (j, i), ends[0])
        q2 = _neighbour_end(case, segs, moved, (j, i), ends[1])
        for g in range(int(np.floor(lo / h)), int(np.ceil(hi / h)) + 1):
            xg = g * h
            if not (lo <= xg <= hi):
                continue
            if per:
                gg = g % n[a]
            elif 0 <= g <= n[a]:
                gg = g
            else:
                continue
            yb = _crossing(p1, p2, q1, q2, a, xg)
            cross.setdefault((row, gg), []).append(yb / h - row)
    nrows = n[b]
    for row in range(nrows):
        for g in range(n[a] + 1):
            if a == 0:
                r, c = row, g
                differ = vc[row, g] != vc[row + 1, g]
            else:
                r, c = g, row
                differ = vc[g, row] != vc[g, row + 1]
            if not differ:
                continue
            ss = cross.get((row, g % n[a] if per else g), [])
            sb = sum(ss) / len(ss) if ss else 0.5   # no crossing found: the edge's midpoint
            new[b][r, c] = min(max(sb, 0.0), 1.0)
    if per:
        # the seam edges repeat the first ones
        if a == 0:
            new[b][:, n[a]] = new[b][:, 0]
        else:
            new[b][n[a], :] = new[b][0, :]
    return [x[None] for x in new], vc[None].astype(np.uint8)


def cell_colours(case, markers, vcol):
    """Cell-centre colours from the markers and corner colours (R27)."""
    nx, ny = _dims(case)
    h = case.h
    vc = np.asarray(vcol)[0].astype(int)
    cc = np.zeros((ny, nx), np.uint8)
    segs = _cell_segments(case, markers)
    for j in range(ny):
        for i in range(nx):
            corners = [vc[j, i], vc[j, i + 1], vc[j + 1, i], vc[j + 1, i + 1]]
            if (j, i) not in segs:
                cc[j, i] = corners[0]
                continue
            pts = []
            for (e, r, c) in segs[(j, i)]:
                s = float(np.asarray(markers[e])[0][r, c])
                pts.append(((c + s) * h, r * h) if e == 0 else (c * h, (r + s) * h))
            (x1, y1), (x2, y2) = pts
            # the segment's normal, turned towards the liquid corners
            nxs, nys = -(y2 - y1), x2 - x1
            side = 0.0
            for (dx, dy), col in zip(((0, 0), (1, 0), (0, 1), (1, 1)), corners):
                side += (2 * col - 1) * (nxs * ((i + dx) * h - x1) + nys * ((j + dy) * h - y1))
            if side < 0:
                nxs, nys = -nxs, -nys
            centre = nxs * ((i + 0.5) * h - x1) + nys * ((j + 0.5) * h - y1)
            cc[j, i] = 1 if centre >= 0 else 0
    return cc[None]


def advect(case, geo, u_l, u_v, mdot, dt):
    """One time step of the interface (Eq. discrete_marker_motion, x pass
    then y pass): returns (markers, vertex colours, cell colours)."""
    ug = cell_interface_velocity(case, geo, u_l, u_v, mdot)
    mk, vc = case.markers, case.vcol
    for a in range(2):
        mk, vc = advect_pass(case, mk, vc, ug, dt, a)
    return mk, vc, cell_colours(case, mk, vc)
