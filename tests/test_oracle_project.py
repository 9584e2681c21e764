"""Pins for the oracle's ghost-fluid projection.

Independent references: the Stefan outflow closed form after one projection
(liquid pushed out at mdot (1/rho_v - 1/rho_l), Sec. 3.1), the DST-II
diagonalisation of the uniform-density Dirichlet problem, exact
reproduction of a piecewise-linear pressure with continuous flux across a
planar interface at any theta, the discrete divergence constraint, the total
outflow of the constant-mdot bubble (Sec. 3.3) and reflection symmetry.
"""
import math

import numpy as np
import pytest
import scipy.fft as fft

import ebit_inputs as ei
from oracle import flux, geometry, pipeline, project, solve


def test_stefan_projection_closed_form():
    c = ei.config(0)
    r = pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    pr = c.props
    mdot = pr.lam_v / (0.3 * pr.h_lg)
    U = mdot * (1.0 / pr.rho_v - 1.0 / pr.rho_l)
    ul = r["u_l"][0][0]                 # [ny][nx+1]
    uv = r["u_v"][0][0]
    # exact up to rounding (the refined direct solve reaches the discrete solution)
    assert np.allclose(ul[:, 19:], U, rtol=1e-13, atol=0)
    # the vapour field is meaningful on faces touching a vapour cell (0..19)
    assert np.max(np.abs(uv[:, :20])) < 1e-12 * U
    assert np.max(np.abs(r["u_l"][1])) < 1e-12 * U
    x = (np.arange(64) + 0.5) / 64
    slope = pr.rho_l * U / c.dt
    pex = np.where(np.arange(64) >= 19, slope * (1 - x), slope * (1 - 19.5 / 64))
    p = r["p"].reshape(64, 64)
    assert np.max(np.abs(p - pex[None, :])) < 1e-14 * slope


@pytest.mark.parametrize("dim,n", [(2, 20), (2, 33), (3, 9)])
def test_uniform_dirichlet_is_dst_diagonal(dim, n):
    """No interface, p = 0 on every wall: the cell-centred Dirichlet
    Laplacian (ghost -p) is diagonal in the DST-II basis with eigenvalues
    -(2 - 2 cos(pi (k+1)/n)) / h^2 per axis."""
    rng = np.random.default_rng(n)
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    shp = ei.cell_shape(dim, nn)
    props = ei.Props(rho_l=3.0)
    case = ei.Case("flat", dim, nn, h, props, 2e-3, [(0, 0.0)] * (2 * dim), [(1, 0.0)] * (2 * dim),
                   [np.full(ei.edge_shape(dim, nn, a), np.nan) for a in range(dim)],
                   np.ones(ei.vertex_shape(dim, nn), np.uint8), np.ones(shp, np.uint8),
                   np.zeros(shp), [], [])
    g = geometry.build(case)
    L, bc = project.assemble(case, g)
    assert not np.any(bc)
    b = rng.normal(size=shp)
    p = solve.direct(L, b.ravel())
    sq = b if dim == 3 else b[0]
    bh = fft.dstn(sq, type=2, norm="ortho")
    lam = np.zeros(bh.shape)
    for ax in range(bh.ndim):
        k = np.arange(bh.shape[ax])
        ev = (2 - 2 * np.cos(np.pi * (k + 1) / n)) / h ** 2
        shape = [1] * bh.ndim
        shape[ax] = -1
        lam = lam + ev.reshape(shape)
    beta = case.dt / props.rho_l
    ref = fft.idstn(-bh / (beta * lam), type=2, norm="ortho")
    assert np.max(np.abs(p - ref.ravel())) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("xg_cells,rho_ratio", [(9.5, 1000.0), (9.03, 1000.0), (9.97, 50.0), (9.31, 7.0)])
def test_piecewise_linear_pressure_exact(xg_cells, rho_ratio):
    """Planar interface, Dirichlet p at both x walls, no sources: the exact
    solution is linear in each phase, continuous, with continuous dt/rho dp/dx.
    The link property average reproduces it exactly at any theta."""
    n = 24
    props = ei.Props(rho_l=1.0, rho_v=1.0 / rho_ratio)
    c = ei.stefan_2d(n, x_gamma_cells=xg_cells, props=props)
    p0, p1 = 2.0, -1.0
    c.p_bc = [(1, p0), (1, p1), (0, 0.0), (0, 0.0)]
    g = geometry.build(c)
    L, bc = project.assemble(c, g)
    p = solve.direct(L, -bc)
    xg = xg_cells / n
    # slopes: vapour s_v on [0, xg], liquid s_l on [xg, 1]; rho_l s_v... flux
    # continuity s_v / rho_v = s_l / rho_l; continuity p0 + s_v xg = p1 - s_l (1 - xg)
    rv, rl = props.rho_v, props.rho_l
    s_v = (p1 - p0) / (xg + (1 - xg) * rl / rv)
    s_l = s_v * rl / rv
    x = (np.arange(n) + 0.5) / n
    pex = np.where(x < xg, p0 + s_v * x, p1 - s_l * (1 - x))
    assert np.max(np.abs(p.reshape(n, n) - pex[None, :])) < 1e-11 * max(abs(p0), abs(p1))


@pytest.mark.parametrize("dim,n,seed", [(2, 24, 3), (2, 31, 5), (3, 10, 1)])
def test_divergence_free_after_projection(dim, n, seed):
    """Eq. Poisson_equation imposes div_c u^{n+1} = 0 per phase."""
    c = ei.random_case(dim, n, seed)
    r = pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    bnorm = np.linalg.norm(r["b"])
    assert np.max(np.abs(r["div"])) < 1e-11 * bnorm
    # both fields are updated with the same gradient on every face
    for a in range(dim):
        du_l = r["u_l"][a] - r["u_l_ghost"][a]
        du_v = r["u_v"][a] - r["u_v_ghost"][a]
        assert np.max(np.abs(du_l - du_v)) <= 1e-14 * np.max(np.abs(du_l))


def _bubble_outflow(n, mdot=0.1):
    R = 0.2
    rho_ratio = 1000.0
    c = ei.bubble(2, n, R, 1.0, 0.02, rho_ratio, 0.1)
    g = geometry.build(c)
    m = np.where(g["is_if"], mdot, 0.0)
    r = project.project(c, g, m, c.u_l, c.u_v, solve.direct)
    ul = r["u_l"]
    h = c.h
    out = (ul[0][0, :, -1].sum() - ul[0][0, :, 0].sum() + ul[1][0, -1, :].sum() - ul[1][0, 0, :].sum()) * h
    pr = c.props
    exact = mdot * (1.0 / pr.rho_v - 1.0 / pr.rho_l) * 2 * math.pi * R
    return abs(out - exact) / exact


def test_constant_mdot_bubble_outflow_converges():
    """Sec. 3.3 bubble with an imposed mdot: the liquid leaving the box per
    unit time equals mdot (1/rho_v - 1/rho_l) times the perimeter."""
    errs = [_bubble_outflow(n) for n in (64, 128, 256)]
    assert errs[-1] < 0.02, errs
    assert errs[2] < errs[0], errs


def test_reflection_symmetry_of_centred_bubble():
    c = ei.bubble(2, 48, 0.17, 1.0, 0.05, 100.0, 0.2)
    r = pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    n = 48
    T = r["T"].reshape(n, n)
    assert np.max(np.abs(T - T[:, ::-1])) < 1e-11
    assert np.max(np.abs(T - T.T)) < 1e-11
    m = r["mdot"].reshape(n, n)
    assert np.max(np.abs(m - m[::-1, :])) < 1e-11 * np.max(np.abs(m))
    p = r["p"].reshape(n, n)
    assert np.max(np.abs(p - p.T)) < 1e-9 * np.max(np.abs(p))
    assert np.max(np.abs(p - p[:, ::-1])) < 1e-9 * np.max(np.abs(p))
    ux = r["u_l"][0][0]          # [ny][nx+1]; x-reflection flips the sign
    assert np.max(np.abs(ux + ux[:, ::-1])) < 1e-9 * np.max(np.abs(ux))


@pytest.mark.parametrize("dim,mvec,pt", [
    (2, (0.8, 0.6, 0.0), (0.52, 0.47, 0.0)),
    (2, (-0.28, 0.96, 0.0), (0.41, 0.55, 0.0)),
    (3, (0.48, 0.6, 0.64), (0.49, 0.53, 0.51)),
])
def test_face_owner_and_mass_flux_holder_rule(dim, mvec, pt):
    """Which phase owns a cut face, which field gets the ghost, and which
    cell's mass flux and normal the ghost uses, worked out from the exact
    straight interface and the stated readings, not from the oracle's code.

    Readings: the crossing of a link lies in the cell holding it (the lower
    cell when the fraction from the lower centre is at most 1/2); the face
    takes the phase of the side it lies on (the lower cell's when the
    crossing is beyond the face); Eq. ghost_velocity with the jump of Eq.
    velocity_jump: u_vap^g = u_liq + mdot [1/rho] n and
    u_liq^g = u_vap - mdot [1/rho] n, n the unit normal from vapour into
    liquid.  Every cell gets a distinct mass flux, and the line is tilted so
    that both cells of many cut links carry a facet, with the crossing on
    either side of the face: a flipped holder or owner rule fails here."""
    n = 16 if dim == 2 else 10
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    mv = np.asarray(mvec, float)
    mv = mv / np.linalg.norm(mv)
    ls = ei.Plane(mv, pt)
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    rng = np.random.default_rng(3)
    props = ei.Props(rho_l=1.0, rho_v=0.02)
    u = [rng.normal(0, 1.0, ei.face_shape(dim, nn, a)) for a in range(dim)]
    uv = [rng.normal(0, 1.0, ei.face_shape(dim, nn, a)) for a in range(dim)]
    case = ei.Case("tilted", dim, nn, h, props, 1e-4, [(0, 0.0)] * (2 * dim), [(1, 0.0)] * (2 * dim),
                   mk, vcol, ccol, np.zeros(ei.cell_shape(dim, nn)), u, uv)
    g = geometry.build(case)
    N = case.ncells
    mdot = 1.0 + 0.001 * np.arange(N)
    ul_o, uv_o = project.ghost_velocities(case, g, mdot, case.u_l, case.u_v)
    mf_o = flux.mass_flux_faces(case, g, mdot)
    jump_coef = 1.0 / props.rho_l - 1.0 / props.rho_v
    col = ccol.ravel()
    both_if = {"below": 0, "beyond": 0}
    for a in range(dim):
        fs = ei.face_shape(dim, nn, a)
        exp_ul, exp_uv = u[a].copy(), uv[a].copy()
        exp_mf = np.full(fs, np.nan)
        for kk in range(nn[2] if dim == 3 else 1):
            for j in range(n):
                for i in range(n):
                    q = [i, j, kk]
                    q[a] += 1
                    if q[a] >= n:
                        continue
                    c = i + n * (j + n * kk)
                    up = q[0] + n * (q[1] + n * q[2])
                    if col[c] == col[up]:
                        continue
                    xc = np.array([(i + .5) * h, (j + .5) * h, (kk + .5) * h if dim == 3 else 0.0])
                    t = -float(np.dot(mv, xc - np.asarray(pt))) / (mv[a] * h)
                    assert 0.0 < t < 1.0 and abs(t - 0.5) > 1e-9
                    holder = c if t < 0.5 else up
                    owner = col[c] if t > 0.5 else col[up]
                    fidx = (kk, j, i + 1) if a == 0 else ((kk, j + 1, i) if a == 1 else (kk + 1, j, i))
                    if dim == 2:
                        fidx = (0,) + fidx[1:]
                    jump = mdot[holder] * jump_coef * mv[a]
                    if owner == 1:
                        exp_uv[fidx] = u[a][fidx] + jump
                    else:
                        exp_ul[fidx] = uv[a][fidx] - jump
                    exp_mf[fidx] = mdot[holder]
                    if g["is_if"][c] and g["is_if"][up]:
                        both_if["below" if t < 0.5 else "beyond"] += 1
        assert np.array_equal(np.isnan(exp_mf), np.isnan(mf_o[a]))
        ok = ~np.isnan(exp_mf)
        assert np.array_equal(exp_mf[ok], mf_o[a][ok])
        assert np.max(np.abs(ul_o[a] - exp_ul)) <= 1e-12 * np.max(np.abs(exp_ul))
        assert np.max(np.abs(uv_o[a] - exp_uv)) <= 1e-12 * np.max(np.abs(exp_uv))
    # the rule is exercised where it matters: both cells carry a facet, on both sides of 1/2
    assert both_if["below"] > 0 and both_if["beyond"] > 0, both_if


@pytest.mark.parametrize("dim,n,seed", [(2, 8, 1), (2, 13, 4), (3, 5, 2), (3, 6, 7)])
def test_pressure_direct_matches_dense_lu(dim, n, seed):
    """The assembled variable-density Poisson system on tiny random grids:
    the refined sparse direct solve equals dense LU (numpy.linalg.solve)."""
    c = ei.random_case(dim, n, seed, bc="mixed")
    g = geometry.build(c)
    L, bc = project.assemble(c, g)
    rng = np.random.default_rng(seed)
    b = rng.normal(size=c.ncells) - bc
    op = project.operator(c, g)
    x1 = solve.direct(-L, -b, op)
    x2 = solve.dense(L, b)
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x2))


@pytest.mark.parametrize("dim,mvec,pt", [
    (2, (0.8, 0.6, 0.0), (0.52, 0.47, 0.0)),
    (2, (-0.28, 0.96, 0.0), (0.41, 0.55, 0.0)),
    (3, (0.48, 0.6, 0.64), (0.49, 0.53, 0.51)),
])
def test_band_ghosts_planar_interface(dim, mvec, pt):
    """Ghost velocities over the narrow band (Eq. ghost_velocity, the mass
    flux carried to the band, step 4 of Sec. 2.5) on an exact straight
    interface, worked out from the definitions rather than the oracle's code.

    Every band normal of a plane is the plane's unit normal, and a mass flux
    linear in position has, as the mean of two neighbouring cells, its value
    at the face centre.  So on every face whose two cells are band cells
    (a cell is in the band when its 3^d block holds an interface cell):
      * a cut face follows the owner/holder rule (mdot of the cell holding
        the crossing);
      * an uncut face keeps the real field of its cells' common phase, and
        the other field takes u_vap - u_liq = mdot(x_face) [1/rho] n_a;
    every other face keeps both fields.  A flipped sign, a wrong axis of n,
    the wrong field, one cell's mdot in place of the mean, or a face with
    one cell outside the band taking a ghost fails here."""
    n = 16 if dim == 2 else 9
    nn = (n, n, n if dim == 3 else 1)
    h = 1.0 / n
    mv = np.asarray(mvec, float)
    mv = mv / np.linalg.norm(mv)
    ls = ei.Plane(mv, pt)
    vcol, ccol, mk = ei.colours_and_markers(dim, nn, h, ls)
    rng = np.random.default_rng(5)
    props = ei.Props(rho_l=1.0, rho_v=0.02)
    u = [rng.normal(0, 1.0, ei.face_shape(dim, nn, a)) for a in range(dim)]
    uv = [rng.normal(0, 1.0, ei.face_shape(dim, nn, a)) for a in range(dim)]
    case = ei.Case("tilted", dim, nn, h, props, 1e-4, [(0, 0.0)] * (2 * dim), [(1, 0.0)] * (2 * dim),
                   mk, vcol, ccol, np.zeros(ei.cell_shape(dim, nn)), u, uv)
    g = geometry.build(case)
    N = case.ncells
    nz = nn[2] if dim == 3 else 1
    alpha, beta = 0.7, np.array([0.3, -0.45, 0.2])

    def centre(i, j, kk):
        return np.array([(i + .5) * h, (j + .5) * h, (kk + .5) * h if dim == 3 else 0.0])

    mdot = np.zeros(N)
    for kk in range(nz):
        for j in range(n):
            for i in range(n):
                mdot[i + n * (j + n * kk)] = alpha + float(np.dot(beta, centre(i, j, kk)))
    ul_o, uv_o = project.ghost_velocities_band(case, g, mdot, case.u_l, case.u_v)
    # band membership from its definition
    is_if = np.asarray(g["is_if"]).ravel().astype(bool)
    inb = np.zeros(N, bool)
    rz = 1 if dim == 3 else 0
    for kk in range(nz):
        for j in range(n):
            for i in range(n):
                for dk in range(-rz, rz + 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            q = (i + di, j + dj, kk + dk)
                            if all(0 <= q[b] < nn[b] for b in range(3)) and is_if[q[0] + n * (q[1] + n * q[2])]:
                                inb[i + n * (j + n * kk)] = True
    jump_coef = 1.0 / props.rho_l - 1.0 / props.rho_v
    col = ccol.ravel()
    seen = {"cut": 0, "liq": 0, "vap": 0, "half_band": 0}
    for a in range(dim):
        exp_ul, exp_uv = u[a].copy(), uv[a].copy()
        for kk in range(nz):
            for j in range(n):
                for i in range(n):
                    q = [i, j, kk]
                    q[a] += 1
                    if q[a] >= n:
                        continue
                    c = i + n * (j + n * kk)
                    up = q[0] + n * (q[1] + n * q[2])
                    fidx = (kk, j, i + 1) if a == 0 else ((kk, j + 1, i) if a == 1 else (kk + 1, j, i))
                    if dim == 2:
                        fidx = (0,) + fidx[1:]
                    if not (inb[c] and inb[up]):
                        seen["half_band"] += int(inb[c] or inb[up])
                        continue
                    if col[c] != col[up]:
                        xc = centre(i, j, kk)
                        t = -float(np.dot(mv, xc - np.asarray(pt))) / (mv[a] * h)
                        holder = c if t < 0.5 else up
                        owner = col[c] if t > 0.5 else col[up]
                        jump = mdot[holder] * jump_coef * mv[a]
                        seen["cut"] += 1
                    else:
                        xf = centre(i, j, kk)
                        xf[a] += 0.5 * h
                        jump = (alpha + float(np.dot(beta, xf))) * jump_coef * mv[a]
                        owner = col[c]
                        seen["liq" if owner == 1 else "vap"] += 1
                    if owner == 1:
                        exp_uv[fidx] = u[a][fidx] + jump
                    else:
                        exp_ul[fidx] = uv[a][fidx] - jump
        scale = max(np.max(np.abs(exp_ul)), np.max(np.abs(exp_uv)))
        assert np.max(np.abs(ul_o[a] - exp_ul)) <= 1e-12 * scale
        assert np.max(np.abs(uv_o[a] - exp_uv)) <= 1e-12 * scale
    assert all(v > 0 for v in seen.values()), seen


def test_band_ghosts_reduce_to_cut_faces_off_the_band():
    """On the 2D bubble with a mass flux only in the interface cells (not
    extended): the cut faces take exactly the projection's ghosts, and an
    uncut band face whose two cells carry no mass flux gets a ghost equal to
    the real velocity of its phase (a zero jump)."""
    case = ei.config(0)
    g = geometry.build(case)
    rng = np.random.default_rng(9)
    mdot = rng.normal(0.0, 1.0, case.ncells) * np.asarray(g["is_if"]).ravel()
    ul_b, uv_b = project.ghost_velocities_band(case, g, mdot, case.u_l, case.u_v)
    ul_c, uv_c = project.ghost_velocities(case, g, mdot, case.u_l, case.u_v)
    col = case.ccol.ravel().astype(int)
    for a in range(case.dim):
        th = g["theta"][a]
        cut = ~np.isnan(th)
        assert np.array_equal(ul_b[a][cut], ul_c[a][cut]) and np.array_equal(uv_b[a][cut], uv_c[a][cut])
        # uncut faces: a zero mdot on both cells leaves u_v = u_l on liquid faces (ghost = real)
        lo, up = flux._face_cells(case, a)
        both = (lo >= 0) & (up >= 0) & ~cut
        changed = both & ((ul_b[a] != case.u_l[a]) | (uv_b[a] != case.u_v[a]))
        z = changed & (mdot[np.maximum(lo, 0)] == 0) & (mdot[np.maximum(up, 0)] == 0)
        liq = col[np.maximum(lo, 0)] == 1
        assert np.array_equal(uv_b[a][z & liq], ul_b[a][z & liq])
        assert np.array_equal(ul_b[a][z & ~liq], uv_b[a][z & ~liq])
