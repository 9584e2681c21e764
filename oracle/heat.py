"""Implicit per-phase heat diffusion with T = T_sat imposed sharply (oracle).

Paper Sec. 2.4, Eq. energy_diffusion (backward Euler for the diffusion part,
T* is the advected field), Eq. temp_bc_interface (T_Gamma = T_sat) imposed by
the ghost value of Eq. ghost_T, which turns the stencil into Eq. Txx_ghost.

Row of cell c of phase k (assembled, one matrix for both phases; a cut link
couples nothing, so the matrix is block diagonal by phase):

  (rho_k cp_k/dt + sum_links lam_k w / h^2) T_c - sum_{same-phase nb} lam_k/h^2 T_nb
      = rho_k cp_k/dt T*_c + sum_cut lam_k T_sat/(theta' h^2) + sum_Dirichlet 2 lam_k T_w/h^2

w = 1 for a same-phase neighbour, 1/theta' for a cut link (theta' = fraction
from c's centre to the interface, clamped below at theta_min), 2 for a
Dirichlet wall face (ghost 2 T_w - T_c, i.e. a cut at theta = 1/2), 0 for a
Neumann face; periodic faces wrap.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import _cell_index

NEUMANN, DIRICHLET, PERIODIC = 0, 1, 2


def side_neighbours(case, a, sgn):
    """(cell ids, neighbour ids or -1 at a non-periodic wall, theta' from the
    cell, cut mask) for side (a, sgn) of every cell, using the face arrays."""
    ids = _cell_index(case)
    ax = 2 - a
    n_a = ids.shape[ax]
    nb = np.roll(ids, -sgn, axis=ax)
    periodic = case.T_bc[2 * a][0] == PERIODIC
    if not periodic:
        sl = [slice(None)] * 3
        sl[ax] = n_a - 1 if sgn > 0 else 0
        nb[tuple(sl)] = -1
    return ids.ravel(), nb.ravel()


def face_of_side(theta_a, case, a, sgn):
    """Face value on side (a, sgn) of every cell (face arrays have n_a + 1)."""
    ax = 2 - a
    n_a = theta_a.shape[ax] - 1
    sl = [slice(None)] * 3
    sl[ax] = slice(1, n_a + 1) if sgn > 0 else slice(0, n_a)
    return theta_a[tuple(sl)].ravel()


def theta_from_cell(theta, case, a, sgn):
    """Fraction of the link from the cell's own centre to the interface."""
    t = face_of_side(theta[a], case, a, sgn)
    return t if sgn > 0 else 1.0 - t


def operator(case, geo, theta_min=1e-3):
    """The heat operator as link fluxes (solve.FluxOp): m_c = rho cp/dt plus
    the wall (2 lam/h^2) and cut-link (lam/(theta' h^2)) terms; w = lam/h^2
    on every same-phase link."""
    from .solve import FluxOp
    pr = case.props
    dim, h, dt = case.dim, case.h, case.dt
    col = case.ccol.ravel().astype(int)
    rho = np.where(col == 1, pr.rho_l, pr.rho_v)
    cp = np.where(col == 1, pr.cp_l, pr.cp_v)
    lam = np.where(col == 1, pr.lam_l, pr.lam_v)
    mexc = rho * cp / dt
    rows, cols, w = [], [], []
    plus = []
    for a in range(dim):
        for sgn, side in ((-1, 2 * a), (+1, 2 * a + 1)):
            ids, nb = side_neighbours(case, a, sgn)
            kind, _ = case.T_bc[side]
            wall = nb < 0
            if kind == DIRICHLET:
                mexc[wall] += 2 * lam[wall] / h ** 2
            inner = ~wall
            same = inner.copy()
            same[inner] = col[nb[inner]] == col[inner]
            cut = inner & ~same
            rows.append(ids[same])
            cols.append(nb[same])
            w.append(lam[same] / h ** 2)
            if sgn > 0:
                wp = np.zeros(col.size)
                wp[ids[same]] = lam[same] / h ** 2
                plus.append(wp)
            th = theta_from_cell(geo["theta"], case, a, sgn)
            if np.any(np.isnan(th[cut])):
                raise ValueError("cut link without theta")
            tc = np.maximum(th[cut], theta_min)
            mexc[cut] += lam[cut] / (tc * h ** 2)
    return FluxOp(mexc, np.concatenate(rows), np.concatenate(cols), np.concatenate(w),
                  plus, grid_shape(case))


def grid_shape(case):
    """(cells per axis, periodic flag per axis) of the case's grid."""
    return (tuple(case.n), tuple(case.T_bc[2 * a][0] == PERIODIC if a < case.dim else False
                                 for a in range(3)))


def rhs(case, geo, T_star, theta_min=1e-3):
    """Right-hand side of the heat system: rho cp/dt T* plus the interface
    (lam T_sat/(theta' h^2)) and wall (2 lam T_w/h^2) terms."""
    pr = case.props
    dim, h, dt = case.dim, case.h, case.dt
    col = case.ccol.ravel().astype(int)
    rho = np.where(col == 1, pr.rho_l, pr.rho_v)
    cp = np.where(col == 1, pr.cp_l, pr.cp_v)
    lam = np.where(col == 1, pr.lam_l, pr.lam_v)
    b = rho * cp / dt * T_star.ravel()
    for a in range(dim):
        for sgn, side in ((-1, 2 * a), (+1, 2 * a + 1)):
            ids, nb = side_neighbours(case, a, sgn)
            kind, val = case.T_bc[side]
            wall = nb < 0
            if kind == DIRICHLET:
                b[wall] += 2 * lam[wall] * val / h ** 2
            inner = ~wall
            cut = inner.copy()
            cut[inner] = col[nb[inner]] != col[inner]
            th = theta_from_cell(geo["theta"], case, a, sgn)
            tc = np.maximum(th[cut], theta_min)
            b[cut] += lam[cut] * pr.T_sat / (tc * h ** 2)
    return b


def assemble(case, geo, T_star, theta_min=1e-3):
    """Return (A csr, b) of the heat system (Eqs. energy_diffusion, Txx_ghost)."""
    return operator(case, geo, theta_min).to_csr(), rhs(case, geo, T_star, theta_min)
