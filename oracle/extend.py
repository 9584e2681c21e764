"""Narrow-band extension of a cell field across the interface (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.4, Eq. extrapolation: a field known in one region is carried into a
narrow band around the interface by marching, in a pseudo time tau, the
transport equation  df/dtau + a . grad f = 0  whose velocity a is the unit
interface normal pointing out of the region that holds the data.  The paper
uses it for the advected temperature of each phase (liquid -> vapour and
vapour -> liquid) and for the mass flux (from the cut cells to the band).

Readings (the paper gives the equation and the band, not the scheme):
  * a cell is in the band when it, or any cell of its 3^d block, is an
    interface cell (one that carries a facet);
  * the normal of a band cell is the normalised sum of the facet normals
    (vapour -> liquid) of the interface cells in its 3^d block, the cell
    itself included; a band cell whose sum vanishes keeps its value;
  * the transport velocity of a band cell points away from the interface into
    the cell's own phase: a = +n in liquid cells, a = -n in vapour cells (the
    paper's two equations, for a normal from vapour into liquid);
  * modes: LIQ_TO_VAP updates the vapour band cells (liquid cells hold the
    data), VAP_TO_LIQ the liquid band cells (vapour cells hold the data),
    IFACE_TO_BAND the band cells that are not interface cells (the interface
    cells hold the data); every other cell keeps its value;
  * first-order upwind differences, explicit Euler steps in tau with
    dtau = h / d, so that sum_d |a_d| dtau / h <= sqrt(d) / d <= 1 (the update
    is a convex combination: monotone), all target cells from the previous
    iterate (Jacobi);
  * along axis d the difference takes the upwind neighbour (c - e_d when
    a_d > 0, c + e_d when a_d < 0) only if that cell holds data or is itself
    a target; a neighbour beyond a wall, or outside the band on the far side,
    drops the term.  Periodic axes wrap.

The update of a target cell c is

    f(c) <- f(c) - (1/d) * sum_d |a_d| (f(c) - f(up_d(c))).
"""
from __future__ import annotations

import itertools

import numpy as np

LIQ_TO_VAP, VAP_TO_LIQ, IFACE_TO_BAND = 0, 1, 2


def _periodic(case):
    return [case.T_bc[2 * a][0] == 2 for a in range(case.dim)]


def _shape(case):
    nx, ny, nz = case.n
    return (nz if case.dim == 3 else 1, ny, nx)


def _neighbour(case, idx, off):
    """Flat index of the cell at integer offset `off` (per axis) from each
    cell of `idx`, and whether it exists (walls stop, periodic axes wrap)."""
    nx, ny, nz = case.n
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    per = _periodic(case)
    pos = [i, j, k]
    ok = np.ones(idx.shape, bool)
    for a in range(case.dim):
        p = pos[a] + off[a]
        n_a = case.n[a]
        if per[a]:
            p = np.mod(p, n_a)
        else:
            ok &= (p >= 0) & (p < n_a)
            p = np.clip(p, 0, n_a - 1)
        pos[a] = p
    return pos[0] + nx * (pos[1] + ny * pos[2]), ok


def band(case, geo):
    """Band membership [N] bool and band normals [N, 3] (zero where the sum
    of the block's facet normals vanishes or the cell is outside the band).

    Each interface cell is handed to every cell of its 3^d block: the cell c
    that sees interface cell m at offset o is c = m - o, so looping over the
    offsets o (x slowest) adds each cell's terms in its own block order."""
    dim = case.dim
    is_if = np.asarray(geo["is_if"]).ravel().astype(bool)
    nF = np.asarray(geo["nF"]).reshape(-1, 3)
    N = is_if.size
    src = np.nonzero(is_if)[0]
    inb = np.zeros(N, bool)
    s = np.zeros((N, 3))
    for off in itertools.product((-1, 0, 1), repeat=dim):
        back = [-o for o in off] + [0] * (3 - dim)
        c, ok = _neighbour(case, src, back)
        inb[c[ok]] = True
        np.add.at(s, c[ok], nF[src[ok]])
    L = np.sqrt((s * s).sum(axis=1))
    n = np.where((inb & (L > 0))[:, None], s / np.where(L > 0, L, 1.0)[:, None], 0.0)
    return inb, n


def extend(case, geo, q, mode, iters):
    """Apply `iters` pseudo-time steps of Eq. extrapolation to the cell field
    q (any shape with the case's cell count); returns a new array."""
    dim = case.dim
    f = np.asarray(q, dtype=np.float64).ravel().copy()
    N = f.size
    liquid = np.asarray(case.ccol).ravel().astype(bool)
    is_if = np.asarray(geo["is_if"]).ravel().astype(bool)
    inb, n = band(case, geo)
    if mode == LIQ_TO_VAP:
        data, target = liquid, inb & ~liquid
    elif mode == VAP_TO_LIQ:
        data, target = ~liquid, inb & liquid
    elif mode == IFACE_TO_BAND:
        data, target = is_if, inb & ~is_if
    else:
        raise ValueError(mode)
    target &= np.abs(n).sum(axis=1) > 0
    t = np.nonzero(target)[0]
    sgn = np.where(liquid[t], 1.0, -1.0)
    a = sgn[:, None] * n[t]
    known = data | target
    ups, ws = [], []
    for d in range(dim):
        off = [0, 0, 0]
        step = np.where(a[:, d] > 0, -1, 1)
        m = np.empty(t.size, dtype=np.int64)
        ok = np.empty(t.size, bool)
        for sv in (-1, 1):
            sel = step == sv
            off[d] = sv
            mm, oo = _neighbour(case, t[sel], off)
            m[sel] = mm
            ok[sel] = oo
        use = ok & (a[:, d] != 0) & known[m]
        ups.append(m)
        ws.append(np.where(use, np.abs(a[:, d]), 0.0))
    lam = 1.0 / dim
    for _ in range(iters):
        g = f.copy()
        acc = np.zeros(t.size)
        for d in range(dim):
            acc += ws[d] * (f[t] - f[ups[d]])
        g[t] = f[t] - lam * acc
        f = g
    return f.reshape(np.shape(q))
