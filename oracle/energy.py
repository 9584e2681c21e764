"""The advection part of the energy equation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.4, Eq. energy_advection: in each phase k the intermediate
temperature T*_k follows from T_k by one explicit Euler step of
rho_k cp_k (dT/dt + u_k . grad T) = 0, i.e.

    T*_k = T_k - dt * sum_a u_{k,a} dT_k/dx_a,

with the derivative taken by the third-order WENO scheme of Jiang & Shu
(1996).  Each cell takes the value of its own phase; the other phase's
values near the interface are those the caller extended across it (Eq.
extrapolation), so that every stencil reads one phase only.

Readings (the paper names the scheme and nothing more):
  * R30 the derivative along axis a is the difference of two face values
    over h, each reconstructed from the upwind side by the Jiang & Shu
    third-order WENO reconstruction (the point values playing the part of
    cell averages, as in their finite-difference form): with the upwind
    cells (m, 0) and the downwind cell p of the face,
        q0 = (3 T_0 - T_m) / 2,   q1 = (T_0 + T_p) / 2,
        beta0 = (T_0 - T_m)^2,    beta1 = (T_p - T_0)^2,
        alpha_r = d_r / (eps + beta_r)^2,  d = (1/3, 2/3),
        face = (alpha0 q0 + alpha1 q1) / (alpha0 + alpha1).
    The upwind side is given by the sign of the cell's velocity component
    (u > 0: the faces i - 1/2 and i + 1/2 seen from the left; u < 0: from
    the right); a zero component contributes nothing.
  * R31 eps is a caller's argument, 1e-6 by default (Jiang & Shu's value).
  * R32 the velocity of a cell is that of its own phase at the centre, the
    mean of the cell's two faces per axis in that phase's face field (R22).
  * R33 a stencil cell beyond a wall takes the value of the nearest cell
    inside (the stencil is clamped); periodic axes wrap.
  * R34 the sum over axes runs a = 0, 1, 2 and is multiplied by dt once:
    T* = T - dt * (u_0 D_0 + u_1 D_1 + u_2 D_2).
"""
from __future__ import annotations

import numpy as np

from . import advect

WENO_EPS = 1e-6
_D0, _D1 = 1.0 / 3.0, 2.0 / 3.0


def weno3_face(tm, t0, tp, eps=WENO_EPS):
    """Value at the face between cell 0 and its downwind neighbour p,
    reconstructed from the upwind cells m and 0 (R30)."""
    q0 = 0.5 * (3.0 * t0 - tm)
    q1 = 0.5 * (t0 + tp)
    b0 = (t0 - tm) ** 2
    b1 = (tp - t0) ** 2
    a0 = _D0 / (eps + b0) ** 2
    a1 = _D1 / (eps + b1) ** 2
    return (a0 * q0 + a1 * q1) / (a0 + a1)


def _periodic(case):
    return [case.T_bc[2 * a][0] == 2 for a in range(case.dim)]


def _ijk(case, cells):
    nx, ny, _ = case.n
    i = cells % nx
    j = (cells // nx) % ny
    k = cells // (nx * ny)
    return [i, j, k]


def _shift(case, ijk, a, off, per):
    """Flat indices of the cells off steps along axis a (wrapped on a
    periodic axis, clamped at a wall: R33)."""
    nx, ny, _ = case.n
    c = list(ijk)
    n_a = case.n[a]
    v = c[a] + off
    c[a] = np.mod(v, n_a) if per else np.clip(v, 0, n_a - 1)
    return c[0] + nx * (c[1] + ny * c[2])


def derivative(case, T, a, sign, cells, eps=WENO_EPS):
    """dT/dx_a at the given cells by WENO3 from the side given by sign
    (+1: the flow goes to +x_a, -1: to -x_a), R30."""
    T = np.asarray(T, dtype=float).ravel()
    per = _periodic(case)[a]
    ijk = _ijk(case, cells)
    t = {o: T[_shift(case, ijk, a, o, per)] for o in (-2, -1, 0, 1, 2)}
    h = case.h
    if sign > 0:
        # upwind cells on the left: face i+1/2 from (i-1, i | i+1), face
        # i-1/2 from (i-2, i-1 | i)
        up = weno3_face(t[-1], t[0], t[1], eps)
        lo = weno3_face(t[-2], t[-1], t[0], eps)
    else:
        # upwind cells on the right: face i+1/2 from (i+2, i+1 | i), face
        # i-1/2 from (i+1, i | i-1)
        up = weno3_face(t[2], t[1], t[0], eps)
        lo = weno3_face(t[1], t[0], t[-1], eps)
    return (up - lo) / h


def advect_energy(case, T_l, T_v, u_l, u_v, dt, eps=WENO_EPS, cells=None):
    """Eq. energy_advection: T* at the given flat cell indices (all cells by
    default).  case.ccol gives each cell's phase (1 liquid: T_l and u_l;
    0 vapour: T_v and u_v)."""
    N = int(np.prod(case.n))
    cells = np.arange(N) if cells is None else np.asarray(cells, dtype=np.int64)
    col = np.asarray(case.ccol).ravel()[cells].astype(bool)
    u = advect.cell_velocity(case, u_l, u_v)[cells]          # own phase, R32
    out = np.empty(cells.size)
    for liq, T in ((True, T_l), (False, T_v)):
        sel = col == liq
        if not np.any(sel):
            continue
        cs = cells[sel]
        Tc = np.asarray(T, dtype=float).ravel()[cs]
        acc = np.zeros(cs.size)
        for a in range(case.dim):
            ua = u[sel, a]
            dp = derivative(case, T, a, +1, cs, eps)
            dm = derivative(case, T, a, -1, cs, eps)
            d = np.where(ua > 0, dp, np.where(ua < 0, dm, 0.0))
            acc = acc + ua * d
        out[sel] = Tc - dt * acc
    return out
