"""Cases and fields of the energy-advection tests: grids of any shape with
walls or periodic axes, a plane interface splitting the phases, smooth or
rough per-phase temperatures and face velocities of both signs."""
import numpy as np

import ebit_inputs as ei


def energy_case(dim, n, periodic=(False, False, False), normal=(1.0, 0.4, 0.2), offset=0.5, h=None,
                name="energy"):
    """n = (nx, ny, nz) cells (nz = 1 in 2D); liquid where
    normal . (x - offset * extent) > 0; walls (T Neumann, p Dirichlet) or
    periodic axes (a library context needs a power-of-two length there and
    one wall axis)."""
    nn = (n[0], n[1], n[2] if dim == 3 else 1)
    h = h if h is not None else 1.0 / nn[0]
    m = np.array(normal, dtype=float)
    if dim == 2:
        m[2] = 0.0
    m /= np.linalg.norm(m)
    ext = np.array([nn[0] * h, nn[1] * h, nn[2] * h])
    ls = ei.Plane(m, tuple(offset * ext))
    vcol, ccol, markers = ei.colours_and_markers(dim, nn, h, ls)
    T_bc, p_bc = [], []
    for a in range(dim):
        for _ in range(2):
            T_bc.append((ei.PERIODIC, 0.0) if periodic[a] else (ei.NEUMANN, 0.0))
            p_bc.append((ei.PERIODIC, 0.0) if periodic[a] else (ei.DIRICHLET, 0.0))
    z = [np.zeros(ei.face_shape(dim, nn, a)) for a in range(dim)]
    T0 = np.zeros(ei.cell_shape(dim, nn))
    return ei.Case(name, dim, nn, h, ei.Props(), 1e-3, T_bc, p_bc, markers, vcol, ccol, T0, z,
                   [x.copy() for x in z])


def cell_centres(case):
    nx, ny, nz = case.n
    h = case.h
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h, (np.arange(nx) + 0.5) * h,
                          indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def smooth_field(case, rng, base=373.0, amp=2.0):
    """A sum of a few random sinusoids (periodic over the box) plus a slope
    along the wall axes."""
    x, y, z = cell_centres(case)
    L = [case.n[a] * case.h for a in range(3)]
    f = np.full(x.shape, base)
    for _ in range(4):
        k = rng.integers(1, 4, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        f += amp * rng.uniform(0.2, 1.0) * np.sin(2 * np.pi * k[0] * x / L[0] + ph[0]) * \
            np.cos(2 * np.pi * k[1] * y / L[1] + ph[1]) * np.cos(2 * np.pi * k[2] * z / L[2] + ph[2])
    return f


def rough_field(case, rng, base=373.0):
    """Smooth plus a step and cell-scale noise (exercises the nonlinear
    weights away from their linear values)."""
    x, _, _ = cell_centres(case)
    f = smooth_field(case, rng, base)
    f += np.where(x > 0.37 * case.n[0] * case.h, 3.0, 0.0)
    f += rng.normal(0.0, 0.05, f.shape)
    return f


def face_velocities(case, rng, scale, zero_frac=0.1):
    """Per-phase face fields of both signs; a share of the faces exactly 0
    (a zero cell component where both faces of a cell vanish).  On a
    periodic axis the last face layer is the copy of the first (the seam)."""
    ul, uv = [], []
    for a in range(case.dim):
        shp = ei.face_shape(case.dim, case.n, a)
        ax = len(shp) - 1 - a
        for out in (ul, uv):
            v = rng.normal(0.0, scale, shp)
            v[rng.uniform(size=shp) < zero_frac] = 0.0
            if case.T_bc[2 * a][0] == ei.PERIODIC:
                idx = [slice(None)] * len(shp)
                first = list(idx)
                idx[ax] = -1
                first[ax] = 0
                v[tuple(idx)] = v[tuple(first)]
            out.append(v)
    return ul, uv


def cfl_dt(case, ul, uv, cfl):
    """A time step with |u_a| dt / h <= cfl for every face speed."""
    vmax = max(float(np.max(np.abs(v))) for v in list(ul) + list(uv))
    return cfl * case.h / max(vmax, 1e-300)
