"""Ghost temperatures and the interfacial mass flux (oracle).

Paper Sec. 2.4:
  * Eq. ghost_T: across a cut link from a phase-k cell c, the other cell g
    gets T_k(g) = T_Gamma + (T_Gamma - T_c)(1 - theta)/theta, theta measured
    from c (clamped below like the operator).  A cell with several cut links
    to phase-k cells takes the mean of the extrapolations.
  * Eq. normal_gradient: two points along the normal at d1, d2 from the
    interface centroid, T there by bi-/tri-quadratic interpolation, and
    dT/ds = [d2/d1 (T1 - T_G) - d1/d2 (T2 - T_G)]/(d2 - d1), s the distance
    into the phase (sign reading: with d1, d2 measured into the phase this
    is the derivative along the outward direction of the interface into the
    phase, exact for quadratic profiles).
  * Eq. mass_flux_computation: mdot = (lam_l dT_l/ds_l + lam_v dT_v/ds_v)/h_lg
    with the normal read as pointing into the liquid on the liquid side, so
    mdot > 0 is evaporation.

Stencil reading: d1 = h, d2 = 2h; the 3^d Lagrange block is centred on the
cell containing the point (moved inward to stay inside non-periodic walls),
values come from phase-k cells or the ghost
layer; when one is missing the block moves one cell along the dominant axis
of the direction into the phase; when still missing the gradient falls back
to the first-order difference from the nearest phase-k centre (counted).
"""
from __future__ import annotations

import numpy as np

from .heat import side_neighbours, theta_from_cell


def ghost_fill(case, geo, T, theta_min=1e-3):
    """Ghost value of the *other* phase in every cell (NaN where none)."""
    pr = case.props
    col = case.ccol.ravel().astype(int)
    Tf = T.ravel()
    acc = np.zeros(col.size)
    cnt = np.zeros(col.size)
    for a in range(case.dim):
        for sgn in (-1, +1):
            ids, nb = side_neighbours(case, a, sgn)
            # link seen from cell ids (the ghost cell g) towards nb (= c, the phase-k cell)
            inner = nb >= 0
            cut = np.zeros_like(inner)
            cut[inner] = col[nb[inner]] != col[inner]
            th_g = theta_from_cell(geo["theta"], case, a, sgn)   # from g's centre
            th_c = np.maximum(1.0 - th_g[cut], theta_min)        # from c's centre
            Tc = Tf[nb[cut]]
            val = pr.T_sat + (pr.T_sat - Tc) * (1.0 - th_c) / th_c
            np.add.at(acc, ids[cut], val)
            np.add.at(cnt, ids[cut], 1.0)
    g = np.full(col.size, np.nan)
    m = cnt > 0
    g[m] = acc[m] / cnt[m]
    return g


def _lagrange3(t):
    return np.array([0.5 * t * (t - 1.0), (1.0 - t) * (1.0 + t), 0.5 * t * (t + 1.0)])


def _value(case, k, T, ghost, idx3):
    """T_k at cell (i, j, k) with wrap on periodic axes; None if unavailable."""
    n = case.n
    ii = list(idx3)
    for a in range(case.dim):
        if not (0 <= ii[a] < n[a]):
            if case.T_bc[2 * a][0] == 2:
                ii[a] %= n[a]
            else:
                return None
    c = ii[0] + n[0] * (ii[1] + n[1] * (ii[2] if case.dim == 3 else 0))
    if case.ccol.ravel()[c] == k:
        return T.ravel()[c]
    g = ghost[c]
    return None if np.isnan(g) else g


def _interp(case, k, T, ghost, P, centre):
    h, dim = case.h, case.dim
    w = []
    for a in range(3):
        if a < dim:
            t = (P[a] - (centre[a] + 0.5) * h) / h
            w.append(_lagrange3(t))
        else:
            w.append(np.array([0.0, 1.0, 0.0]))
    tot = 0.0
    for dk in ((-1, 0, 1) if dim == 3 else (0,)):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                v = _value(case, k, T, ghost, (centre[0] + di, centre[1] + dj, centre[2] + dk))
                if v is None:
                    return None
                tot += w[0][di + 1] * w[1][dj + 1] * w[2][dk + 1] * v
    return tot


def _clamp_block(case, centre):
    """Keep a 3-wide block inside the domain along non-periodic axes."""
    for a in range(case.dim):
        if case.T_bc[2 * a][0] != 2:
            centre[a] = min(max(centre[a], 1), case.n[a] - 2)
    return centre


def _point_value(case, k, T, ghost, P, s_dir):
    h, dim = case.h, case.dim
    centre = _clamp_block(case, [int(np.floor(P[a] / h)) if a < dim else 0 for a in range(3)])
    v = _interp(case, k, T, ghost, P, centre)
    if v is not None:
        return v
    a_dom = int(np.argmax(np.abs(s_dir[:dim])))
    centre[a_dom] += 1 if s_dir[a_dom] > 0 else -1
    centre = _clamp_block(case, centre)
    return _interp(case, k, T, ghost, P, centre)


def mass_flux(case, geo, T, theta_min=1e-3, cells=None):
    """Per-cell mdot (0 off the interface) and the number of fallbacks;
    ``cells`` restricts the evaluation to a sample of interface cells."""
    pr, h, dim = case.props, case.h, case.dim
    ghost = ghost_fill(case, geo, T, theta_min)
    N = case.ccol.size
    mdot = np.zeros(N)
    fallbacks = 0
    d1, d2 = h, 2.0 * h
    todo = np.nonzero(geo["is_if"])[0] if cells is None else np.asarray(cells)
    for c in todo:
        cF, nF = geo["cF"][c], geo["nF"][c]
        D = {}
        for k, sgn in ((1, 1.0), (0, -1.0)):
            s_dir = sgn * nF
            P1 = cF + d1 * s_dir
            P2 = cF + d2 * s_dir
            T1 = _point_value(case, k, T, ghost, P1, s_dir)
            T2 = _point_value(case, k, T, ghost, P2, s_dir)
            if T1 is not None and T2 is not None:
                D[k] = (d2 / d1 * (T1 - pr.T_sat) - d1 / d2 * (T2 - pr.T_sat)) / (d2 - d1)
            else:
                fallbacks += 1
                D[k] = _fallback(case, k, T, cF, s_dir, P1)
        mdot[c] = (pr.lam_l * D[1] + pr.lam_v * D[0]) / pr.h_lg
    return mdot, fallbacks


def _fallback(case, k, T, cF, s_dir, P1):
    h, dim, n = case.h, case.dim, case.n
    centre = [int(np.floor(P1[a] / h)) if a < dim else 0 for a in range(3)]
    best = None
    for dk in ((-1, 0, 1) if dim == 3 else (0,)):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                q = [centre[0] + di, centre[1] + dj, centre[2] + dk]
                ok = True
                for a in range(dim):
                    if not (0 <= q[a] < n[a]):
                        if case.T_bc[2 * a][0] == 2:
                            q[a] %= n[a]
                        else:
                            ok = False
                if not ok:
                    continue
                c = q[0] + n[0] * (q[1] + n[1] * q[2])
                if case.ccol.ravel()[c] != k:
                    continue
                x = np.array([(centre[0] + di + 0.5) * h, (centre[1] + dj + 0.5) * h,
                              (centre[2] + dk + 0.5) * h if dim == 3 else 0.0])
                proj = np.dot(x - cF, s_dir)
                if proj <= 0:
                    continue
                dist = np.sum((x - P1) ** 2)
                if best is None or dist < best[0] or (dist == best[0] and c < best[1]):
                    best = (dist, c, proj)
    if best is None:
        return 0.0
    return (T.ravel()[best[1]] - case.props.T_sat) / best[2]


def face_holder(theta_face):
    """For a cut link, which cell holds the crossing: 0 = lower, 1 = upper."""
    return np.where(theta_face <= 0.5, 0, 1)


def mass_flux_faces(case, geo, mdot):
    """mdot on each cut face: the value of the cell holding the crossing
    (the other cell if that one carries no facet); NaN on uncut faces."""
    out = []
    is_if = geo["is_if"]
    for a in range(case.dim):
        th = geo["theta"][a]
        mf = np.full(th.shape, np.nan)
        lo_c, up_c = _face_cells(case, a)
        cut = ~np.isnan(th)
        for fidx in zip(*np.nonzero(cut)):
            lo, up = lo_c[fidx], up_c[fidx]
            hold = lo if th[fidx] <= 0.5 else up
            if not is_if[hold]:
                hold = up if hold == lo else lo
            mf[fidx] = mdot[hold]
        out.append(mf)
    return out


def _face_cells(case, a):
    """Lower / upper cell id of every face of axis a (-1 where none)."""
    from .geometry import _cell_index
    ids = _cell_index(case)
    ax = 2 - a
    n_a = ids.shape[ax]
    fshape = list(ids.shape)
    fshape[ax] += 1
    lo = np.full(fshape, -1)
    up = np.full(fshape, -1)
    sl = [slice(None)] * 3
    sl[ax] = slice(1, n_a + 1)
    lo[tuple(sl)] = ids
    sl[ax] = slice(0, n_a)
    up[tuple(sl)] = ids
    if case.T_bc[2 * a][0] == 2:
        s0 = [slice(None)] * 3
        s0[ax] = 0
        sl_last = [slice(None)] * 3
        sl_last[ax] = n_a - 1
        lo[tuple(s0)] = ids[tuple(sl_last)]
        sN = [slice(None)] * 3
        sN[ax] = n_a
        s_first = [slice(None)] * 3
        s_first[ax] = 0
        up[tuple(sN)] = ids[tuple(s_first)]
    return lo, up
