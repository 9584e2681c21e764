"""Pins for the oracle's implicit heat operator with sharp T = T_sat.

Independent references: the linear Stefan steady state (Eq. ghost_T is exact
for linear profiles), the DCT-II diagonalisation of the interface-free
Neumann problem, a manufactured discontinuous solution converging at second
order (the accuracy the paper claims for Eq. Txx_ghost), the symmetry the
paper claims for the discretisation, and dense LU on tiny grids.
"""
import numpy as np
import pytest
import scipy.fft as fft

import ebit_inputs as ei
from oracle import geometry, heat, solve


def test_stefan_linear_profile_is_discrete_steady_state():
    c = ei.config(0)
    g = geometry.build(c)
    A, b = heat.assemble(c, g, c.T0)
    T = solve.direct(A, b)
    assert np.max(np.abs(T - c.T0.ravel())) < 1e-12
    assert np.all(T.reshape(c.T0.shape)[c.ccol == 1] == 0.0)


@pytest.mark.parametrize("dim,n", [(2, 24), (2, 37), (3, 10)])
def test_no_interface_neumann_is_dct_diagonal(dim, n):
    """All-liquid, Neumann walls: (rho cp/dt - lam Lap_h) T = rho cp/dt T*.
    The cell-centred Neumann Laplacian is diagonal in the DCT-II basis with
    eigenvalues (2 - 2 cos(pi k / n)) / h^2 per axis."""
    rng = np.random.default_rng(n)
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    shp = ei.cell_shape(dim, nn)
    props = ei.Props(rho_l=2.0, cp_l=3.0, lam_l=0.7)
    case = ei.Case("flat", dim, nn, h, props, 1e-3, [(0, 0.0)] * (2 * dim), [(1, 0.0)] * (2 * dim),
                   [np.full(ei.edge_shape(dim, nn, a), np.nan) for a in range(dim)],
                   np.ones(ei.vertex_shape(dim, nn), np.uint8), np.ones(shp, np.uint8),
                   rng.normal(size=shp), [], [])
    g = geometry.build(case)
    A, b = heat.assemble(case, g, case.T0)
    T = solve.direct(A, b)
    axes = tuple(range(3 - dim, 3))
    sq = case.T0 if dim == 3 else case.T0[0]
    That = fft.dctn(sq, type=2, norm="ortho")
    lam = np.zeros(That.shape)
    for ax in range(That.ndim):
        k = np.arange(That.shape[ax])
        ev = (2 - 2 * np.cos(np.pi * k / n)) / h ** 2
        shape = [1] * That.ndim
        shape[ax] = -1
        lam = lam + ev.reshape(shape)
    m = props.rho_l * props.cp_l / case.dt
    ref = fft.idctn(m * That / (m + props.lam_l * lam), type=2, norm="ortho")
    assert np.max(np.abs(T - ref.ravel())) < 1e-12 * np.max(np.abs(ref))
    del axes


@pytest.mark.parametrize("dim,n,seed", [(2, 20, 1), (2, 27, 2), (3, 9, 3)])
def test_operator_symmetric_positive_definite(dim, n, seed):
    """The paper calls the sharp treatment symmetric (Sec. 2.4, after Eq.
    Txx_ghost): the assembled matrix is
    symmetric with a positive diagonal dominating each row (SPD)."""
    c = ei.random_case(dim, n, seed)
    g = geometry.build(c)
    A, _ = heat.assemble(c, g, c.T0)
    assert abs(A - A.T).max() == 0.0
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    assert np.all(d > off)
    # phases decouple: no entry links a liquid to a vapour cell
    col = c.ccol.ravel()
    r, cc = A.nonzero()
    assert np.all(col[r] == col[cc])


@pytest.mark.parametrize("dim,n,seed", [(2, 8, 1), (2, 11, 4), (3, 5, 2), (3, 6, 7)])
def test_direct_matches_dense_lu(dim, n, seed):
    c = ei.random_case(dim, n, seed, bc="mixed")
    g = geometry.build(c)
    A, b = heat.assemble(c, g, c.T0)
    x1 = solve.direct(A, b)
    x2 = solve.dense(A, b)
    assert np.max(np.abs(x1 - x2)) <= 1e-13 * np.max(np.abs(x2))


def _manufactured_error(dim, n):
    """T_k = s_k (r^2 - R^2) prod sin(pi x_a): zero on the circle and the walls;
    T* = T - dt lam_k/(rho_k cp_k) Lap T_k makes T the exact solution of the
    backward-Euler step.  Returns the max-norm error at the cell centres."""
    R = 0.3
    ctr = 0.5 + 0.013
    props = ei.Props(rho_l=1.0, rho_v=0.5, lam_l=1.0, lam_v=0.1, cp_l=1.0, cp_v=2.0, T_sat=0.0)
    ls = ei.Ball((ctr, ctr, ctr), R, +1.0, dim)
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    shp = ei.cell_shape(dim, nn)
    z, y, x = np.meshgrid((np.arange(shp[0]) + .5) * h, (np.arange(shp[1]) + .5) * h,
                          (np.arange(shp[2]) + .5) * h, indexing="ij")
    X = [x, y, z][:dim]
    q = sum((X[a] - ctr) ** 2 for a in range(dim)) - R * R
    s = np.ones_like(x)
    for a in range(dim):
        s = s * np.sin(np.pi * X[a])
    grad_q = [2 * (X[a] - ctr) for a in range(dim)]
    grad_s = []
    for a in range(dim):
        g = np.pi * np.cos(np.pi * X[a])
        for b in range(dim):
            if b != a:
                g = g * np.sin(np.pi * X[b])
        grad_s.append(g)
    lap = 2 * dim * s + 2 * sum(grad_q[a] * grad_s[a] for a in range(dim)) + q * (-dim * np.pi ** 2 * s)
    sk = np.where(ccol == 1, 1.0, 3.0)
    Tex = sk * q * s
    lam = np.where(ccol == 1, props.lam_l, props.lam_v)
    rc = np.where(ccol == 1, props.rho_l * props.cp_l, props.rho_v * props.cp_v)
    dt = 1e-3
    Tstar = Tex - dt * lam / rc * sk * lap
    case = ei.Case("mms", dim, nn, h, props, dt, [(1, 0.0)] * (2 * dim), [(1, 0.0)] * (2 * dim),
                   mk, vcol, ccol, Tstar, [], [])
    g = geometry.build(case)
    A, b = heat.assemble(case, g, Tstar, theta_min=1e-12)
    T = solve.direct(A, b)
    return np.max(np.abs(T - Tex.ravel()))


def test_manufactured_second_order_2d():
    errs = [_manufactured_error(2, n) for n in (64, 128, 256)]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.36 * e0, errs     # ratio 1/4 expected for second order


def test_manufactured_converges_3d():
    # 16^3 -> 32^3 is still pre-asymptotic for this solution (the same ratio,
    # about 0.45, is seen with exact crossings in place of the facet ones)
    errs = [_manufactured_error(3, n) for n in (16, 32)]
    assert errs[1] < 0.5 * errs[0], errs


def test_planar_layer_reduces_to_tridiagonal_rows():
    """Input uniform in y with a planar interface (the Stefan layer, x_Gamma
    = 19.2 h): every row of the 2D system is the 1D system below, written
    here from Eqs. energy_diffusion and Txx_ghost (backward Euler, sharp
    T = T_sat through theta), and solved with scipy.linalg.solve_banded.
    Cells 0..18 are vapour, 19..63 liquid; the link 18-19 is cut at
    theta = 0.7 from cell 18 and 0.3 from cell 19; x = 0 is a wall at T_w
    (ghost 2 T_w - T_0), x = 1 a zero-flux wall."""
    from scipy.linalg import solve_banded
    c = ei.config(0)
    pr = c.props
    rng = np.random.default_rng(21)
    row = rng.uniform(-1.0, 1.0, 64)
    Tstar = np.repeat(row[None, :], 64, axis=0)[None]
    g = geometry.build(c)
    A, b = heat.assemble(c, g, Tstar)
    T = solve.direct(A, b, heat.operator(c, g)).reshape(64, 64)
    n, h, dt = 64, c.h, c.dt
    Tw = c.T_bc[0][1]
    ab = np.zeros((3, n))
    rhs = np.zeros(n)
    for i in range(n):
        liq = i >= 19
        lam = pr.lam_l if liq else pr.lam_v
        m = (pr.rho_l * pr.cp_l if liq else pr.rho_v * pr.cp_v) / dt
        d = m
        rhs[i] = m * row[i]
        # left side
        if i == 0:
            d += 2 * lam / h ** 2
            rhs[i] += 2 * lam * Tw / h ** 2
        elif i == 19:
            d += lam / (0.3 * h ** 2)
            rhs[i] += lam * pr.T_sat / (0.3 * h ** 2)
        else:
            d += lam / h ** 2
            ab[2, i - 1] = -lam / h ** 2
        # right side
        if i == n - 1:
            pass
        elif i == 18:
            d += lam / (0.7 * h ** 2)
            rhs[i] += lam * pr.T_sat / (0.7 * h ** 2)
        else:
            d += lam / h ** 2
            ab[0, i + 1] = -lam / h ** 2
        ab[1, i] = d
    ref = solve_banded((1, 1), ab, rhs)
    assert np.max(np.abs(T - ref[None, :])) <= 1e-13 * np.max(np.abs(ref))
