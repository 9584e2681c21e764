"""One-fluid projection with the phase-change source term (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper Sec. 2.3: the alternative to the ghost-fluid projection keeps one face
velocity field and puts the phase change into the continuity equation of the
interface cells, div u^{n+1} = S_pc, with S_pc = mdot S_Gamma / V [1/rho]
(Eq. pc_source): the Poisson problem of Eq. Poisson_equation gets the source
on its right-hand side, and the face update is the one of the ghost-fluid
projection.

Readings:
  * S_Gamma, the interface area inside the cell: the area (3D) or length (2D)
    of the cell's facet plane (through the facet centroid, with the facet
    normal) clipped to the cell; V = h^d;
  * the sign: S_pc = mdot S_Gamma / V (1/rho_v - 1/rho_l), so that an
    evaporating cell (mdot > 0) is a volume source: the net outflow the
    ghost-fluid jump of Eq. ghost_velocity puts through the facet;
  * face densities, walls, outflow and periodic faces as in project.py.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import project

CORNERS = np.array(list(itertools.product((0, 1), repeat=3)))[:, ::-1]   # (x, y, z), x fastest
EDGES = [(a, b) for a in range(8) for b in range(a + 1, 8)
         if np.abs(CORNERS[a] - CORNERS[b]).sum() == 1]


def facet_area(case, geo):
    """S_Gamma per cell [N] (zero off the interface): the cell's facet plane
    clipped to the cell.  The clipped polygon's corners are the plane's
    crossings of the cell's edges (and the cell corners on the plane); they
    are ordered by angle about their mean and the area is the shoelace sum
    (2D: the distance between the two extreme crossings along the facet)."""
    dim, h = case.dim, case.h
    nx, ny, _ = case.n
    is_if = np.asarray(geo["is_if"]).ravel().astype(bool)
    cells = np.nonzero(is_if)[0]
    cF = np.asarray(geo["cF"]).reshape(-1, 3)[cells]
    nF = np.asarray(geo["nF"]).reshape(-1, 3)[cells]
    i, j, k = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    base = np.stack([i * h, j * h, (k * h) if dim == 3 else np.zeros_like(i, dtype=float)], axis=1)
    corners = CORNERS if dim == 3 else CORNERS[:4]
    edges = [(a, b) for (a, b) in EDGES if a < len(corners) and b < len(corners)]
    V = base[:, None, :] + h * corners[None, :, :].astype(float)            # [n, 8|4, 3]
    if dim == 2:
        V[:, :, 2] = 0.0
    s = np.einsum("nvi,ni->nv", V - cF[:, None, :], nF)                    # signed distances
    pts, ok = [], []
    for q in range(len(corners)):
        pts.append(V[:, q])
        ok.append(s[:, q] == 0.0)
    for a, b in edges:
        sa, sb = s[:, a], s[:, b]
        cross = sa * sb < 0
        t = np.where(cross, sa / np.where(cross, sa - sb, 1.0), 0.0)
        pts.append(V[:, a] + t[:, None] * (V[:, b] - V[:, a]))
        ok.append(cross)
    P = np.stack(pts, axis=1)                                               # [n, m, 3]
    M = np.stack(ok, axis=1)
    cnt = M.sum(axis=1)
    o = np.where(M[:, :, None], P, 0.0).sum(axis=1) / np.maximum(cnt, 1)[:, None]
    area = np.zeros(cells.size)
    if dim == 2:
        tau = np.stack([-nF[:, 1], nF[:, 0], np.zeros(cells.size)], axis=1)
        t = np.einsum("nmi,ni->nm", P - o[:, None, :], tau)
        tmax = np.where(M, t, -np.inf).max(axis=1)
        tmin = np.where(M, t, np.inf).min(axis=1)
        area = np.where(cnt >= 2, tmax - tmin, 0.0)
    else:
        # in-plane basis e1, e2 (e1 from the axis least aligned with n)
        ax = np.argmin(np.abs(nF), axis=1)
        e = np.zeros((cells.size, 3))
        e[np.arange(cells.size), ax] = 1.0
        e1 = np.cross(nF, e)
        e1 /= np.linalg.norm(e1, axis=1)[:, None]
        e2 = np.cross(nF, e1)
        R = P - o[:, None, :]
        ang = np.arctan2(np.einsum("nmi,ni->nm", R, e2), np.einsum("nmi,ni->nm", R, e1))
        ang = np.where(M, ang, np.inf)
        order = np.argsort(ang, axis=1, kind="stable")
        Rs = np.take_along_axis(R, order[:, :, None], axis=1)
        Ms = np.take_along_axis(M, order, axis=1)
        # close the loop: unused trailing slots repeat the first corner
        Rs = np.where(Ms[:, :, None], Rs, Rs[:, :1, :])
        nxt = np.roll(Rs, -1, axis=1)
        cr = np.einsum("nmi,ni->nm", np.cross(Rs, nxt), nF)
        area = np.where(cnt >= 3, 0.5 * np.abs(cr.sum(axis=1)), 0.0)
    out = np.zeros(is_if.size)
    out[cells] = area
    return out


def source(case, geo, mdot):
    """S_pc per cell (Eq. pc_source, sign as read above)."""
    pr = case.props
    return (np.asarray(mdot).ravel() * facet_area(case, geo) / case.h ** case.dim
            * (1.0 / pr.rho_v - 1.0 / pr.rho_l))


def project_one_fluid(case, geo, mdot, u, solver):
    """div_c(beta grad p) = div_c u* - S_pc, then u = u* - beta grad p.

    Returns dict(p, u, b, S, div) with div the post-update divergence."""
    S = source(case, geo, mdot)
    div0 = project.divergence(case, u, u)
    L, bc = project.assemble(case, geo)
    rhs = div0 - S - bc
    p = solver(-L, -rhs, project.operator(case, geo))
    u1, _ = project.face_update(case, geo, p, u, u)
    div1 = project.divergence(case, u1, u1)
    return dict(p=p, u=u1, b=rhs, S=S, div=div1)
