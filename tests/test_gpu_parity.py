"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
  * flags: bit-exact; cut pattern (NaN layout of theta): identical;
  * theta, facets, operator rows, right-hand sides, mass flux: FP64, same
    formulas in the same order, agreement to a few ulps (1e-13 relative);
  * one step (T, mdot, mdot on cut faces, p, u): the GPU solves until its
    compensated residual stagnates at the FP64 representability floor
    (reported as res_floor) and is compared with the oracle's refined direct
    solve element by element, per phase, at 1e-12, and velocities face by
    face against the face update of the measured pressure difference
    (tests/parity_util.py states every bar);
  * mixed precision (FP32 V-cycles inside the FP64 outer loop) and the
    defect-correction outer loop: the same bars at the same target.
"""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
import oracle
from parity_util import check_step, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


CASES = {
    "stefan64": lambda: ei.config(0),
    "ball2d_37": lambda: ei.random_case(2, 37, 3),
    "plane2d_50_mixedbc": lambda: ei.random_case(2, 50, 4, kind="plane", bc="mixed"),
    "ball2d_64x_aniso": lambda: _aniso(),
    "ball3d_13": lambda: ei.random_case(3, 13, 5),
    "plane3d_17_mixedbc": lambda: ei.random_case(3, 17, 6, kind="plane", bc="mixed"),
    "film3d_16_periodic": lambda: ei.film_3d(16),
    "bubble2d_40": lambda: ei.bubble(2, 40, 0.17, 1.0, 0.05, 1000.0, 0.1, sigma_u=1e-3, seed=9),
    "ball3d_70x21x19_aniso": lambda: _aniso3d(),
}


def _aniso():
    """Non-square grid: 45 x 29 cells (ragged tiles, odd sizes)."""
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
    """3D grid of 70 x 21 x 19 cells: two 64-wide tiles in x with a ragged
    second one, ragged y tiles and z-chunks, odd coarse levels."""
    dim, n = 3, (70, 21, 19, )
    h = 1.0 / 70
    ls = ei.Ball((0.47, 0.151, 0.137), 0.095, -1.0, dim)
    vcol, ccol, mk = ei.colours_and_markers(dim, n, h, ls)
    rng = np.random.default_rng(11)
    T0 = rng.uniform(-1, 1, ei.cell_shape(dim, n))
    u = [rng.normal(0, 1e-2, ei.face_shape(dim, n, a)) for a in range(dim)]
    return ei.Case("aniso3d", dim, n, h, ei.Props(rho_v=0.02, lam_v=0.25, h_lg=40.0), 2e-4,
                   [(0, 0.0)] * 6, [(1, 0.0)] * 6, mk, vcol, ccol, T0, u, [x.copy() for x in u])


def gpu_geometry(case):
    ebit = _ebit()
    ctx, dc = ebit.context_for(case, ebit.default_opts())
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    th = [torch.empty(ei.face_shape(case.dim, case.n, a), dtype=torch.float64, device="cuda")
          for a in range(case.dim)]
    fl = torch.empty(case.ncells, dtype=torch.uint8, device="cuda")
    fc = torch.empty(6 * case.ncells, dtype=torch.float64, device="cuda")
    ctx.get_geometry(th, fl, fc)
    out = {"theta": [t.cpu().numpy() for t in th], "flags": fl.cpu().numpy(),
           "facet": fc.cpu().numpy().reshape(6, -1)}
    ctx.close()
    return out


def gpu_step(case, opts):
    """One pass of the hot path through the C ABI; solver statuses are
    returned in the stats (not raised) so a failing case prints them."""
    ebit = _ebit()
    ctx, dc = ebit.context_for(case, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    out = {}
    T = torch.zeros_like(dc.T0)
    out["heat_stats"] = ctx.heat_solve(dc.T0, T, check=False)
    mdot = torch.zeros_like(dc.T0)
    mface = [torch.empty(ei.face_shape(case.dim, case.n, a), dtype=torch.float64, device="cuda")
             for a in range(case.dim)]
    out["flux_stats"] = ctx.mass_flux(T, mdot, mface)
    p = torch.zeros_like(dc.T0)
    out["proj_stats"] = ctx.project(dc.u_l, dc.u_v, mdot, p, check=False)
    torch.cuda.synchronize()
    out["T"] = T.cpu().numpy().ravel()
    out["mdot"] = mdot.cpu().numpy().ravel()
    out["mface"] = [m.cpu().numpy() for m in mface]
    out["p"] = p.cpu().numpy().ravel()
    out["u_l"] = [u.cpu().numpy() for u in dc.u_l]
    out["u_v"] = [u.cpu().numpy() for u in dc.u_v]
    ctx.close()
    return out



_REF = {}


def ref_of(name):
    if name not in _REF:
        case = CASES[name]()
        _REF[name] = (case, oracle.pipeline.run_step(case, case.T0, case.u_l, case.u_v))
    return _REF[name]


@pytest.mark.parametrize("name", list(CASES))
def test_geometry_parity(name):
    say(f"[gpu] geometry {name}")
    case, ref = ref_of(name)
    g = gpu_geometry(case)
    fl_ref = ref["geo"]["flags"].ravel()
    assert np.array_equal(g["flags"], fl_ref)
    for a in range(case.dim):
        tr, tg = ref["geo"]["theta"][a], g["theta"][a]
        assert np.array_equal(np.isnan(tr), np.isnan(tg))
        ok = ~np.isnan(tr)
        assert np.max(np.abs(tr[ok] - tg[ok]), initial=0) < 1e-13
    iface = ref["geo"]["is_if"]
    cF = g["facet"][:3].T[iface]
    nF = g["facet"][3:].T[iface]
    assert np.max(np.abs(cF - ref["geo"]["cF"][iface]), initial=0) < 1e-15
    assert np.max(np.abs(nF - ref["geo"]["nF"][iface]), initial=0) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_operator_and_rhs_parity(name):
    say(f"[gpu] operators {name}")
    ebit = _ebit()
    case, ref = ref_of(name)
    ctx, dc = ebit.context_for(case, ebit.default_opts())
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    rng = np.random.default_rng(1)
    x = rng.normal(size=case.ncells)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    ctx.apply(ebit.SYS_HEAT, xd, y)
    yh = ref["A_heat"] @ x
    assert rel(y.cpu().numpy(), yh) < 1e-14
    ctx.apply(ebit.SYS_PRESSURE, xd, y)
    yp = -(ref["L"] @ x)
    assert rel(y.cpu().numpy(), yp) < 1e-14
    b = torch.empty_like(xd)
    ctx.heat_rhs(dc.T0, b)
    assert rel(b.cpu().numpy(), ref["b_heat"]) < 1e-14
    # projection right-hand side and ghost values from the oracle's mass flux
    md = torch.tensor(ref["mdot"], device="cuda")
    ctx.project_rhs(dc.u_l, dc.u_v, md, b)
    torch.cuda.synchronize()
    assert rel(b.cpu().numpy(), -ref["b"]) < 1e-14
    for a in range(case.dim):
        assert rel(dc.u_l[a].cpu().numpy(), ref["u_l_ghost"][a]) < 1e-15
        assert rel(dc.u_v[a].cpu().numpy(), ref["u_v_ghost"][a]) < 1e-15
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp64-dc"])
@pytest.mark.parametrize("name", list(CASES))
def test_step_parity(name, precision):
    say(f"[gpu] step {name} {precision}")
    ebit = _ebit()
    case, ref = ref_of(name)
    opts = ebit.default_opts(rtol=1e-15, max_iters=400,
                             precision=ebit.MIXED if precision == "mixed" else ebit.FP64,
                             outer=ebit.OUTER_DC if precision.endswith("dc") else ebit.OUTER_PCG)
    g = gpu_step(case, opts)
    say("   heat", g["heat_stats"], "\n   proj", g["proj_stats"], "\n   flux", g["flux_stats"])
    assert g["heat_stats"]["status"] == 0 and g["proj_stats"]["status"] == 0
    assert g["flux_stats"]["fallbacks"] == ref["fallbacks"]
    check_step(case, ref, g)
    # discrete divergence after the update: it is the final residual of the
    # pressure system, so bounded by max(rtol, floor) ||b|| up to rounding
    ps = g["proj_stats"]
    umax = max(np.max(np.abs(g["u_l"][a])) for a in range(case.dim))
    bound = 2 * max(ps["rel_res"], ps["res_floor"]) * ps["bnorm"] + 1e-14 * umax / case.h
    assert ps["div_max"] <= bound, (ps["div_max"], bound)


WIDE = [("ball3d_13", "mixed"), ("film3d_16_periodic", "fp64"), ("ball3d_70x21x19_aniso", "mixed"),
        ("plane3d_17_mixedbc", "fp64-dc")]


@pytest.mark.parametrize("name,precision", WIDE, ids=[f"{n}-{p}" for n, p in WIDE])
def test_step_parity_wide_offsets(name, precision, monkeypatch):
    """The strided p-update with 64-bit cell offsets, which 3D grids of 2^30
    cells or more take instead of the LDS-staged one, forced on small grids:
    the same bars."""
    monkeypatch.setenv("EBIT_WIDE_OFFSETS", "1")
    test_step_parity(name, precision)
