"""Ghost-fluid projection with phase change (oracle).

Paper Sec. 2.3:
  * Eq. ghost_velocity: in the band, each phase's velocity gets a ghost
    value from the other phase's real velocity and the jump of Eq.
    velocity_jump, [u] = mdot [1/rho] n, [phi] = phi_liq - phi_vap.
    Sign reading: with n the unit normal from vapour into liquid,
    u_liq^g = u_vap - mdot [1/rho] n and u_vap^g = u_liq + mdot [1/rho] n, so
    an evaporating front (mdot > 0) pushes the liquid away from the vapour.
  * Eq. poisson_ghost_fluid: div_c(dt/rho_f grad p) = div_c u*_{f,k(c)} with
    the velocity field of the cell's own phase; no pressure jump is imposed.
  * Face update: u_{f,k} = u*_{f,k} - dt/rho_f grad p, applied to both phase
    fields on every face.
Face density reading: rho_f = rho of the common phase on an uncut link, the
property average of Eq. property_average along a cut link otherwise
(rho_f = theta rho_k(lower) + (1 - theta) rho_k(upper)).  Wall faces:
Neumann (no flux, the face velocity is left as given); outflow faces:
p = p_w on the face (ghost 2 p_w - p_c).  Periodic faces wrap.
A face is owned by the phase on its side of the crossing: the lower cell's
colour if theta > 1/2, the upper cell's if theta < 1/2, liquid at 1/2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .flux import _face_cells
from .heat import side_neighbours, face_of_side, grid_shape

NEUMANN, DIRICHLET, PERIODIC = 0, 1, 2


def face_beta(case, geo, a):
    """beta_f = dt / rho_f on every face of axis a (interior and periodic
    links; wall faces get the adjacent cell's dt/rho)."""
    pr = case.props
    col = case.ccol.ravel().astype(int)
    rho_c = np.where(col == 1, pr.rho_l, pr.rho_v)
    lo, up = _face_cells(case, a)
    th = geo["theta"][a]
    beta = np.full(th.shape, np.nan)
    both = (lo >= 0) & (up >= 0)
    cut = both & ~np.isnan(th)
    unc = both & np.isnan(th)
    beta[unc] = case.dt / rho_c[lo[unc]]
    rf = th[cut] * rho_c[lo[cut]] + (1.0 - th[cut]) * rho_c[up[cut]]
    beta[cut] = case.dt / rf
    only_lo = (lo >= 0) & (up < 0)
    only_up = (up >= 0) & (lo < 0)
    beta[only_lo] = case.dt / rho_c[lo[only_lo]]
    beta[only_up] = case.dt / rho_c[up[only_up]]
    return beta


def ghost_velocities(case, geo, mdot, u_l, u_v):
    """Set the ghost value on every cut face (copies returned)."""
    pr = case.props
    col = case.ccol.ravel().astype(int)
    jump_coef = 1.0 / pr.rho_l - 1.0 / pr.rho_v      # [1/rho]
    ul = [x.copy() for x in u_l]
    uv = [x.copy() for x in u_v]
    is_if = geo["is_if"]
    for a in range(case.dim):
        th = geo["theta"][a]
        lo, up = _face_cells(case, a)
        for fidx in zip(*np.nonzero(~np.isnan(th))):
            t = th[fidx]
            c, n = lo[fidx], up[fidx]
            kf = col[c] if t > 0.5 else (col[n] if t < 0.5 else 1)
            hold = c if t <= 0.5 else n
            if not is_if[hold]:
                hold = n if hold == c else c
            jump = mdot[hold] * jump_coef * geo["nF"][hold][a]
            if kf == 1:
                uv[a][fidx] = ul[a][fidx] + jump
            else:
                ul[a][fidx] = uv[a][fidx] - jump
    return ul, uv


def ghost_velocities_band(case, geo, mdot_band, u_l, u_v):
    """Eq. ghost_velocity over the whole narrow band (Sec. 2.3, used only in
    the band; Sec. 2.4, the mass flux carried to the band by Eq.
    extrapolation for this purpose; step 4 of the time iteration of Sec.
    2.5).  mdot_band: the mass flux after extension to the band.  Copies
    returned.

    Readings (the paper names the band and the jump, not the face rule):
      * a face is in the band when both its cells are band cells (those of
        extend.band); a cut link always is (its holder is an interface cell
        and the other cell lies in that cell's block);
      * a cut face takes the ghost of ghost_velocities (face owner, the
        holder's mdot and facet normal); the holder is an interface cell,
        whose extended value is its own mass flux;
      * an uncut face belongs to the common phase of its two cells; mdot_f
        and n_f are the means of the two cells' extended mdot and unit band
        normals (a zero band normal counts as zero), and the other phase's
        field takes the jump with the sign of ghost_velocities (u_v - u_l =
        mdot_f [1/rho] n_f on every band face)."""
    from .extend import band
    pr = case.props
    col = case.ccol.ravel().astype(int)
    jump_coef = 1.0 / pr.rho_l - 1.0 / pr.rho_v      # [1/rho]
    m = np.asarray(mdot_band, dtype=np.float64).ravel()
    inb, nrm = band(case, geo)
    ul, uv = ghost_velocities(case, geo, m, u_l, u_v)
    for a in range(case.dim):
        th = geo["theta"][a]
        lo, up = _face_cells(case, a)
        sel = (lo >= 0) & (up >= 0) & np.isnan(th)
        sel[sel] = inb[lo[sel]] & inb[up[sel]]
        c, n = lo[sel], up[sel]
        mf = 0.5 * (m[c] + m[n])
        nf = 0.5 * (nrm[c, a] + nrm[n, a])
        jump = mf * jump_coef * nf
        liq = col[c] == 1
        ua, va = ul[a][sel], uv[a][sel]
        uv[a][sel] = np.where(liq, ua + jump, va)
        ul[a][sel] = np.where(liq, ua, va - jump)
    return ul, uv


def divergence(case, u_l, u_v):
    """div_c of the cell's own phase field (Eq. poisson_ghost_fluid RHS)."""
    col = case.ccol.astype(int)
    div = np.zeros(col.shape)
    for a in range(case.dim):
        ax = 2 - a
        n_a = col.shape[ax]
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[ax] = slice(1, n_a + 1)
        lo[ax] = slice(0, n_a)
        dl = u_l[a][tuple(hi)] - u_l[a][tuple(lo)]
        dv = u_v[a][tuple(hi)] - u_v[a][tuple(lo)]
        div += np.where(col == 1, dl, dv)
    return (div / case.h).ravel()


def operator(case, geo):
    """The SPD form A = -L as link fluxes (solve.FluxOp): w = beta_f/h^2 on
    every interior or periodic link, m_c = 2 beta/h^2 per outflow face."""
    from .solve import FluxOp
    dim, h = case.dim, case.h
    N = case.ccol.size
    mexc = np.zeros(N)
    rows, cols, w = [], [], []
    plus = []
    for a in range(dim):
        beta = face_beta(case, geo, a)
        for sgn, side in ((-1, 2 * a), (+1, 2 * a + 1)):
            ids, nb = side_neighbours(case, a, sgn)
            bf = face_of_side(beta, case, a, sgn)
            wall = nb < 0
            kind, _ = case.p_bc[side]
            if kind == DIRICHLET:
                mexc[wall] += 2 * bf[wall] / h ** 2
            inner = ~wall
            rows.append(ids[inner])
            cols.append(nb[inner])
            w.append(bf[inner] / h ** 2)
            if sgn > 0:
                wp = np.zeros(N)
                wp[ids[inner]] = bf[inner] / h ** 2
                plus.append(wp)
    return FluxOp(mexc, np.concatenate(rows), np.concatenate(cols), np.concatenate(w),
                  plus, grid_shape(case))


def bc_rhs(case, geo):
    """Boundary part of the Poisson right-hand side: 2 beta p_w/h^2 on every
    outflow face (L p = div - bc_rhs)."""
    h = case.h
    out = np.zeros(case.ccol.size)
    for a in range(case.dim):
        beta = face_beta(case, geo, a)
        for sgn, side in ((-1, 2 * a), (+1, 2 * a + 1)):
            ids, nb = side_neighbours(case, a, sgn)
            bf = face_of_side(beta, case, a, sgn)
            wall = nb < 0
            kind, val = case.p_bc[side]
            if kind == DIRICHLET:
                out[wall] += 2 * bf[wall] * val / h ** 2
    return out


def assemble(case, geo):
    """(L csr, bc_rhs): L p = div - bc_rhs is the discrete Eq. Poisson_equation,
    L p = sum_a [beta_+ (p_+ - p_c) - beta_- (p_c - p_-)] / h^2."""
    return -operator(case, geo).to_csr(), bc_rhs(case, geo)


def face_update(case, geo, p, u_l, u_v):
    """u <- u - beta_f grad p on every face, both phase fields (copies)."""
    dim, h = case.dim, case.h
    ul = [x.copy() for x in u_l]
    uv = [x.copy() for x in u_v]
    pf = p.ravel()
    for a in range(dim):
        beta = face_beta(case, geo, a)
        lo, up = _face_cells(case, a)
        g = np.zeros(beta.shape)
        both = (lo >= 0) & (up >= 0)
        g[both] = (pf[up[both]] - pf[lo[both]]) / h
        ax = 2 - a
        n_a = beta.shape[ax] - 1
        for end, side in ((0, 2 * a), (n_a, 2 * a + 1)):
            kind, val = case.p_bc[side]
            if kind != DIRICHLET:
                continue
            sl = [slice(None)] * 3
            sl[ax] = end
            sl = tuple(sl)
            if end == 0:
                g[sl] = 2.0 * (pf[up[sl]] - val) / h
            else:
                g[sl] = 2.0 * (val - pf[lo[sl]]) / h
        upd = np.where(np.isnan(beta), 0.0, beta) * g
        ul[a] = ul[a] - upd
        uv[a] = uv[a] - upd
    return ul, uv


def project(case, geo, mdot, u_l, u_v, solver):
    """Full projection: ghosts -> RHS -> Poisson solve -> update.

    Returns dict(p, u_l, u_v, b, div) with div the post-update divergence."""
    ulg, uvg = ghost_velocities(case, geo, mdot, u_l, u_v)
    div0 = divergence(case, ulg, uvg)
    L, bc = assemble(case, geo)
    rhs = div0 - bc
    p = solver(-L, -rhs, operator(case, geo))
    ul1, uv1 = face_update(case, geo, p, ulg, uvg)
    div1 = divergence(case, ul1, uv1)
    return dict(p=p, u_l=ul1, u_v=uv1, b=rhs, div=div1, L=L, u_l_ghost=ulg, u_v_ghost=uvg)
