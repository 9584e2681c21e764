"""Pins for the oracle's multigrid solve (oracle/mg.c), the solve it uses on
grids too large for a sparse direct factorisation (the 128^3 sphere and the
256^3 film).

What fixes the answer independently of the multigrid code:
  * the refined sparse direct solve (SuperLU, itself pinned by dense LU and
    the closed forms in test_oracle_heat/test_oracle_project) on every kind
    of grid the workloads have: walls, outflow, periodic axes of even and odd
    length, 2D and 3D, heat and pressure systems;
  * the DCT-II (Neumann heat) and DST-II (Dirichlet Poisson) diagonalisations
    on grids larger than the direct-solve cases, with no interface;
  * the residual it reports, recomputed here in long double;
  * a zero right-hand side gives exactly zero; the thread count does not
    change a bit.
"""
import numpy as np
import pytest
import scipy.fft as fft

import ebit_inputs as ei
from oracle import flux, geometry, heat, mg, project, solve


@pytest.fixture(scope="module", autouse=True)
def _built():
    import os
    if not os.path.exists(mg.LIB_PATH) or os.path.getmtime(mg.LIB_PATH) < os.path.getmtime(mg.SRC_PATH):
        mg.build()


def _film_odd():
    return ei.film_3d(15, seed=3, name="film3d_15_odd_periodic")


CASES = {
    "stefan64": lambda: ei.config(0),
    "ball2d_37": lambda: ei.random_case(2, 37, 3),
    "plane2d_50_mixedbc": lambda: ei.random_case(2, 50, 4, kind="plane", bc="mixed"),
    "ball3d_13": lambda: ei.random_case(3, 13, 5),
    "plane3d_17_mixedbc": lambda: ei.random_case(3, 17, 6, kind="plane", bc="mixed"),
    "film3d_16_periodic": lambda: ei.film_3d(16),
    "film3d_15_odd_periodic": _film_odd,
    "bubble2d_128": lambda: ei.bubble(2, 128, 0.1, 1.0, 0.02, 1000.0, 0.1, sigma_u=1e-3, seed=2),
    "ball3d_32": lambda: ei.bubble(3, 32, 0.15, 2.0, 0.03, 1000.0, 0.05, name="ball3d_32"),
}


def _floor(op, x, b):
    """Representation floor of the relative residual of a double x:
    eps || |b| + |A| |x| || / ||b|| (|A| |x| in the flux form)."""
    ax = np.abs(op.mexc * x)
    np.add.at(ax, op.rows, np.abs(op.w) * (np.abs(x[op.rows]) + np.abs(x[op.cols])))
    return np.finfo(float).eps * np.linalg.norm(np.abs(b) + ax) / np.linalg.norm(b)


def _flux_residual_ld(op, x, b):
    """||b - A x|| / ||b|| with A x in the flux form, in long double."""
    xl = np.asarray(x, dtype=np.longdouble)
    r = np.asarray(b, dtype=np.longdouble) - op.matvec(xl, np.longdouble)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(np.asarray(b, np.longdouble) ** 2)))


@pytest.mark.parametrize("name", list(CASES))
def test_mg_equals_direct(name):
    c = CASES[name]()
    g = geometry.build(c)
    opH = heat.operator(c, g)
    bH = heat.rhs(c, g, c.T0)
    Td = solve.direct(opH.to_csr(), bH, opH)
    info = {}
    Tm = mg.solve_op(opH, bH, info=info)
    assert np.max(np.abs(Tm - Td)) <= 1e-13 * np.max(np.abs(Td)), info
    # the rounded x: its residual sits at the double representation floor
    assert info["rel_res"] < 1e-15
    assert abs(_flux_residual_ld(opH, Tm, bH) - info["rel_res"]) <= 1e-6 * info["rel_res"]
    mdot, _ = flux.mass_flux(c, g, Td)
    ulg, uvg = project.ghost_velocities(c, g, mdot, c.u_l, c.u_v)
    rhs = -(project.divergence(c, ulg, uvg) - project.bc_rhs(c, g))
    opP = project.operator(c, g)
    pd = solve.direct(opP.to_csr(), rhs, opP)
    info = {}
    pm = mg.solve_op(opP, rhs, info=info)
    assert np.max(np.abs(pm - pd)) <= 1e-13 * np.max(np.abs(pd)), info
    # stiff vapour rows: the residual of a double x stagnates at its
    # representation floor, which the direct solve's x meets as well
    fl = _floor(opP, pm, rhs)
    assert info["rel_res"] <= max(1e-15, fl), (info, fl)
    assert _flux_residual_ld(opP, pd, rhs) <= max(1e-15, 2 * fl)


def test_pipeline_with_mg_equals_direct():
    c = ei.random_case(3, 11, 8)
    a = __import__("oracle").pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    b = __import__("oracle").pipeline.run_step(c, c.T0, c.u_l, c.u_v, solver=mg.solver())
    for k in ("T", "mdot", "p"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * np.max(np.abs(a[k])), k
    for a_ in range(c.dim):
        assert np.max(np.abs(a["u_l"][a_] - b["u_l"][a_])) <= 1e-12 * np.max(np.abs(a["u_l"][a_]))


def _flat_case(dim, n, p_dirichlet):
    nn = (n, n, n if dim == 3 else 1)
    shp = ei.cell_shape(dim, nn)
    rng = np.random.default_rng(n + dim)
    props = ei.Props(rho_l=2.0, cp_l=3.0, lam_l=0.7)
    return ei.Case("flat", dim, nn, 1.0 / n, props, 1e-3, [(0, 0.0)] * (2 * dim),
                   [(1 if p_dirichlet else 0, 0.0)] * (2 * dim),
                   [np.full(ei.edge_shape(dim, nn, a), np.nan) for a in range(dim)],
                   np.ones(ei.vertex_shape(dim, nn), np.uint8), np.ones(shp, np.uint8),
                   rng.normal(size=shp), [], [])


def _eig(n, h, kind):
    k = np.arange(n)
    if kind == "dct":
        return (2 - 2 * np.cos(np.pi * k / n)) / h ** 2
    return (2 - 2 * np.cos(np.pi * (k + 1) / n)) / h ** 2


@pytest.mark.parametrize("dim,n", [(2, 256), (3, 48)])
def test_mg_heat_neumann_is_dct_diagonal(dim, n):
    """Interface-free heat step with Neumann walls: diagonal in DCT-II."""
    c = _flat_case(dim, n, False)
    g = geometry.build(c)
    op = heat.operator(c, g)
    T = mg.solve_op(op, heat.rhs(c, g, c.T0))
    sq = c.T0 if dim == 3 else c.T0[0]
    That = fft.dctn(sq, type=2, norm="ortho")
    lam = sum(_eig(n, c.h, "dct").reshape([-1 if ax == a else 1 for ax in range(That.ndim)])
              for a in range(That.ndim))
    m = c.props.rho_l * c.props.cp_l / c.dt
    ref = fft.idctn(m * That / (m + c.props.lam_l * lam), type=2, norm="ortho")
    assert np.max(np.abs(T - ref.ravel())) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim,n", [(2, 256), (3, 48)])
def test_mg_poisson_dirichlet_is_dst_diagonal(dim, n):
    """Uniform density, p = 0 on every wall face (ghost -p_c): the operator
    -div(beta grad) is diagonal in DST-II with eigenvalues beta (2 - 2 cos(pi
    (k+1)/n))/h^2 per axis."""
    c = _flat_case(dim, n, True)
    g = geometry.build(c)
    op = project.operator(c, g)
    rng = np.random.default_rng(5)
    b = rng.normal(size=c.ncells)
    p = mg.solve_op(op, b)
    shp = ei.cell_shape(dim, c.n)
    bq = b.reshape(shp) if dim == 3 else b.reshape(shp)[0]
    bhat = fft.dstn(bq, type=2, norm="ortho")
    lam = sum(_eig(n, c.h, "dst").reshape([-1 if ax == a else 1 for ax in range(bhat.ndim)])
              for a in range(bhat.ndim))
    beta = c.dt / c.props.rho_l
    ref = fft.idstn(bhat / (beta * lam), type=2, norm="ortho")
    assert np.max(np.abs(p - ref.ravel())) < 1e-12 * np.max(np.abs(ref))


def test_mg_zero_rhs_and_thread_independence():
    c = ei.film_3d(16)
    g = geometry.build(c)
    op = heat.operator(c, g)
    assert not np.any(mg.solve_op(op, np.zeros(c.ncells)))
    b = heat.rhs(c, g, c.T0)
    x1 = mg.solve_op(op, b, threads=1)
    x4 = mg.solve_op(op, b, threads=4)
    assert np.array_equal(x1, x4)


def test_mg_needs_structured_operator():
    c = ei.random_case(2, 9, 1)
    g = geometry.build(c)
    op = heat.operator(c, g)
    flat = solve.FluxOp(op.mexc, op.rows, op.cols, op.w)
    with pytest.raises(mg.MGError):
        mg.solve_op(flat, np.ones(c.ncells))
