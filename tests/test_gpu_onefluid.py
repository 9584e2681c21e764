"""One-fluid projection (Eq. pc_source) through the C ABI against the oracle.

* The parity cases of the ghost-fluid tests (2D/3D, walls, outflow, mixed
  and periodic boundaries, ragged sizes), FP64 and mixed precision, driven
  by the oracle's mass flux of the input temperature: p to relative L2
  1e-12; u within what the face update, linear in p, makes of the measured
  difference dp of the two pressures (per face beta_f (|dp_lo| + |dp_up|)/h,
  2 beta_f |dp_c|/h on outflow walls), plus 1e-12 of the update for the face
  density on cut faces (theta agrees to ~1e-13), plus rounding; the reported
  max |div u - S_pc| at the solve's rounding level.
* No mass flux: the one-fluid call equals the ghost-fluid call on u_l = u_v
  bit for bit.
* Full sizes: the 256^2 bubble element by element against the direct
  solve; the 256^3 film element by element against the oracle's multigrid
  solve.
"""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
import oracle
from oracle import onefluid

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def _aniso():
    dim, n = 2, (45, 29, 1)
    h = 1.0 / 45
    ls = ei.Ball((0.5, 0.31, 0.0), 0.17, +1.0, dim)
    vcol, ccol, mk = ei.colours_and_markers(dim, n, h, ls)
    rng = np.random.default_rng(7)
    T0 = rng.uniform(-1, 1, ei.cell_shape(dim, n))
    u = [rng.normal(0, 1e-2, ei.face_shape(dim, n, a)) for a in range(dim)]
    return ei.Case("aniso", dim, n, h, ei.Props(rho_v=0.01, lam_v=0.3, h_lg=50.0), 2e-4,
                   [(0, 0.0)] * 4, [(1, 0.0)] * 4, mk, vcol, ccol, T0, u, [x.copy() for x in u])


def _aniso3d():
    """70 x 21 x 19 cells: two 64-wide tiles in x (the second ragged)."""
    dim, n = 3, (70, 21, 19)
    h = 1.0 / 70
    ls = ei.Ball((0.47, 0.151, 0.137), 0.095, -1.0, dim)
    vcol, ccol, mk = ei.colours_and_markers(dim, n, h, ls)
    rng = np.random.default_rng(11)
    T0 = rng.uniform(-1, 1, ei.cell_shape(dim, n))
    u = [rng.normal(0, 1e-2, ei.face_shape(dim, n, a)) for a in range(dim)]
    return ei.Case("aniso3d", dim, n, h, ei.Props(rho_v=0.02, lam_v=0.25, h_lg=40.0), 2e-4,
                   [(0, 0.0)] * 6, [(1, 0.0)] * 6, mk, vcol, ccol, T0, u, [x.copy() for x in u])


CASES = {
    "stefan64": lambda: ei.config(0),
    "ball2d_37": lambda: ei.random_case(2, 37, 3),
    "plane2d_50_mixedbc": lambda: ei.random_case(2, 50, 4, kind="plane", bc="mixed"),
    "ball2d_45x29": _aniso,
    "ball3d_13": lambda: ei.random_case(3, 13, 5),
    "plane3d_17_mixedbc": lambda: ei.random_case(3, 17, 6, kind="plane", bc="mixed"),
    "film3d_16_periodic": lambda: ei.film_3d(16),
    "bubble2d_40": lambda: ei.bubble(2, 40, 0.17, 1.0, 0.05, 1000.0, 0.1, sigma_u=1e-3, seed=9),
    "ball3d_70x21x19_aniso": _aniso3d,
}


def velocity_floor(case, geo, p, u):
    """Relative size on u of the eps-level rounding of p through the face
    update u -= beta_f (p_up - p_lo)/h."""
    eps = np.finfo(float).eps
    num = 0.0
    for a in range(case.dim):
        beta = oracle.project.face_beta(case, geo, a)
        lo, up = oracle.flux._face_cells(case, a)
        both = (lo >= 0) & (up >= 0)
        d = beta[both] * eps * (np.abs(p[lo[both]]) + np.abs(p[up[both]])) / case.h
        num += np.sum(d * d)
    return np.sqrt(num) / np.sqrt(sum(np.sum(x * x) for x in u))


def update_bound(case, geo, dp):
    """Per axis, the most the face update u -= beta_f grad p can move a face
    velocity for a pressure error dp."""
    out = []
    adp = np.abs(dp)
    for a in range(case.dim):
        beta = np.nan_to_num(oracle.project.face_beta(case, geo, a))
        lo, up = oracle.flux._face_cells(case, a)
        b = np.zeros(beta.shape)
        both = (lo >= 0) & (up >= 0)
        b[both] = beta[both] * (adp[lo[both]] + adp[up[both]]) / case.h
        only = (lo >= 0) ^ (up >= 0)
        cell = np.where(lo >= 0, lo, up)
        b[only] = 2.0 * beta[only] * adp[cell[only]] / case.h
        out.append(b)
    return out


def face_slack(bnd, u_ref, u_star):
    """Per-face allowance for |u_GPU - u_oracle|: what the pressure
    difference makes of it (bnd), plus the face density's own difference on
    cut faces (each side's theta agrees to ~1e-13, so beta_f to ~1e-12 of
    itself: that much of the update u_ref - u*), plus rounding."""
    return 1.001 * bnd + 1e-12 * np.abs(u_ref - u_star) + 4e-16 * (np.abs(u_ref) + np.max(np.abs(u_ref)))


def reference(case):
    geo = oracle.geometry.build(case)
    mdot, _ = oracle.flux.mass_flux(case, geo, case.T0)
    ref = onefluid.project_one_fluid(case, geo, mdot, case.u_l, oracle.solve.direct)
    return geo, mdot, ref


def gpu_one_fluid(case, mdot, opts):
    ebit = _ebit()
    ctx, dc = ebit.context_for(case, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    u = [x.clone() for x in dc.u_l]
    p = torch.zeros_like(dc.T0)
    st = ctx.project_one_fluid(u, torch.tensor(mdot, device="cuda"), p)
    out = p.cpu().numpy().ravel(), [x.cpu().numpy() for x in u], st
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_one_fluid_parity(name, precision):
    ebit = _ebit()
    say(f"[gpu] one-fluid {name} {precision}")
    case = CASES[name]()
    geo, mdot, ref = reference(case)
    opts = ebit.default_opts(rtol=1e-15, max_iters=400,
                             precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    p, u, st = gpu_one_fluid(case, mdot, opts)
    ep = rel(p, ref["p"])
    fl = velocity_floor(case, geo, ref["p"], ref["u"])
    eu = max(rel(u[a], ref["u"][a]) for a in range(case.dim))
    say(f"   p {ep:.1e}  u {eu:.1e} (floor {fl:.1e})  div_max {st['div_max']:.1e}  iters {st['iters']}")
    assert ep < 1e-12
    bnd = update_bound(case, geo, p - ref["p"])
    for a in range(case.dim):
        du = np.abs(u[a] - ref["u"][a])
        assert np.all(du <= face_slack(bnd[a], ref["u"][a], case.u_l[a])), a
    assert st["div_max"] <= 1e-9 * max(np.max(np.abs(ref["b"])), 1e-300)


def test_no_mass_flux_is_the_ghost_fluid_call():
    ebit = _ebit()
    case = ei.random_case(2, 40, 12)
    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    z = torch.zeros_like(dc.T0)
    u1 = [x.clone() for x in dc.u_l]
    p1 = torch.zeros_like(dc.T0)
    ctx.project_one_fluid(u1, z, p1)
    ul = [x.clone() for x in dc.u_l]
    uv = [x.clone() for x in dc.u_l]
    p2 = torch.zeros_like(dc.T0)
    ctx.project(ul, uv, z, p2)
    assert torch.equal(p1, p2)
    for a in range(case.dim):
        assert torch.equal(u1[a], ul[a])
    ctx.close()


def test_one_fluid_bubble2d_256_full():
    ebit = _ebit()
    case = ei.config(1)
    say("[gpu] one-fluid full 256^2")
    geo, mdot, ref = reference(case)
    for precision in (ebit.FP64, ebit.MIXED):
        opts = ebit.default_opts(rtol=1e-15, max_iters=400, precision=precision)
        p, u, st = gpu_one_fluid(case, mdot, opts)
        ep = rel(p, ref["p"])
        fl = velocity_floor(case, geo, ref["p"], ref["u"])
        eu = max(rel(u[a], ref["u"][a]) for a in range(case.dim))
        say(f"   precision {precision}: p {ep:.1e}  u {eu:.1e} (floor {fl:.1e})")
        assert ep < 1e-12
        bnd = update_bound(case, geo, p - ref["p"])
        for a in range(case.dim):
            du = np.abs(u[a] - ref["u"][a])
            assert np.all(du <= face_slack(bnd[a], ref["u"][a], case.u_l[a])), a


@pytest.mark.timeout(1200)
def test_one_fluid_film3d_256_full():
    """The 256^3 film against the oracle's one-fluid projection solved by its
    multigrid (oracle/mg.c): p element by element, per phase, at 1e-12; u
    face by face against the update of the measured pressure difference."""
    from oracle import mg
    from parity_util import phase_err
    ebit = _ebit()
    case = ei.config(4)
    say("[gpu] one-fluid full 256^3 film: oracle reference (multigrid solve)")
    geo = oracle.geometry.build(case)
    mdot, _ = oracle.flux.mass_flux(case, geo, case.T0)
    ref = onefluid.project_one_fluid(case, geo, mdot, case.u_l, mg.solver())
    say("   oracle reference done")
    for precision in (ebit.FP64, ebit.MIXED):
        opts = ebit.default_opts(rtol=1e-15, max_iters=400, precision=precision)
        p, u, st = gpu_one_fluid(case, mdot, opts)
        ep = phase_err(p, ref["p"], case.ccol)
        eu = max(rel(u[a], ref["u"][a]) for a in range(case.dim))
        say(f"   precision {precision}: p per phase {ep}  u {eu:.1e}  iters {st['iters']}")
        assert max(ep.values()) < 1e-12
        bnd = update_bound(case, geo, p - ref["p"])
        for a in range(case.dim):
            du = np.abs(u[a] - ref["u"][a])
            assert np.all(du <= face_slack(bnd[a], ref["u"][a], case.u_l[a])), a
