"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (rtol 1e-9, FP64 and mixed precision).

* 2D bubble, 256 x 256: the oracle still solves it directly, so every output
  is compared element by element (one full step).
* 3D sphere, 128^3, and the 3D film, 256^3: the oracle cannot factor these;
  the checks are the oracle's geometry (flags bit-exact, theta), the residual
  of the GPU's T and p under the oracle's own operators and right-hand sides
  (built from the seeded inputs only), and the mass flux of the input
  temperature at sampled interface cells.
"""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()



def velocity_floor(case, ref):
    """Relative L2 size, on the velocity field, of the FP64 representation
    noise of p: each face update moves u by beta_f (p_up - p_lo)/h, so an
    eps-level rounding of p shows up as beta_f eps (|p_lo| + |p_up|)/h.  Two
    correctly rounded solutions can differ by this much in u."""
    p = ref["p"]
    eps = np.finfo(float).eps
    num = 0.0
    for a in range(case.dim):
        beta = oracle.project.face_beta(case, ref["geo"], a)
        lo, up = oracle.flux._face_cells(case, a)
        both = (lo >= 0) & (up >= 0)
        d = beta[both] * eps * (np.abs(p[lo[both]]) + np.abs(p[up[both]])) / case.h
        num += np.sum(d * d)
    unorm = np.sqrt(sum(np.sum(u * u) for u in ref["u_l"]))
    return np.sqrt(num) / unorm


def rel(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


_C2 = {}


def c2_ref():
    if not _C2:
        c = ei.config(1)
        _C2["case"] = c
        _C2["ref"] = oracle.pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    return _C2["case"], _C2["ref"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bubble2d_256_full_parity(precision):
    say(f"[gpu] full C2 256^2 {precision}")
    ebit = _ebit()
    c, ref = c2_ref()
    opts = ebit.default_opts(rtol=1e-15, max_iters=400, precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    ctx, dc = ebit.context_for(c, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, c.dt)
    T = dc.T0.clone()
    sh = ctx.heat_solve(T, T)
    m = torch.zeros_like(T)
    ctx.mass_flux(T, m)
    p = torch.zeros_like(T)
    sp = ctx.project(dc.u_l, dc.u_v, m, p)
    say("   heat", sh, "\n   proj", sp)
    assert sh["status"] == 0 and sp["status"] == 0
    errs = {"T": rel(T.cpu().numpy(), ref["T"]), "mdot": rel(m.cpu().numpy(), ref["mdot"]),
            "p": rel(p.cpu().numpy(), ref["p"]),
            "u_l": rel(np.concatenate([u.cpu().numpy().ravel() for u in dc.u_l]),
                       np.concatenate([u.ravel() for u in ref["u_l"]])),
            "u_v": rel(np.concatenate([u.cpu().numpy().ravel() for u in dc.u_v]),
                       np.concatenate([u.ravel() for u in ref["u_v"]]))}
    say("   errors", {k: f"{v:.1e}" for k, v in errs.items()})
    ufl = velocity_floor(c, ref)
    say(f"   velocity representation floor {ufl:.1e}")
    for k, v in errs.items():
        tol = max(1e-12, 2 * ufl) if k.startswith("u_") else 1e-12
        assert v < tol, (k, v, tol)
    ctx.close()


def _property_checks(case, name, heat_only=False):
    ebit = _ebit()
    say(f"[gpu] full {name}: oracle geometry, operators and right-hand sides")
    geo = oracle.geometry.build(case)
    opH = oracle.heat.operator(case, geo)
    bH = oracle.heat.rhs(case, geo, case.T0)
    iface = np.nonzero(geo["is_if"])[0]
    rng = np.random.default_rng(0)
    smp = rng.choice(iface, size=min(400, iface.size), replace=False)
    if not heat_only:
        # the projection's right-hand side needs mdot on every interface cell
        mo_all, _ = oracle.flux.mass_flux(case, geo, case.T0)
        ulg, uvg = oracle.project.ghost_velocities(case, geo, mo_all, case.u_l, case.u_v)
        rhs = -(oracle.project.divergence(case, ulg, uvg) - oracle.project.bc_rhs(case, geo))
        opP = oracle.project.operator(case, geo)
    for precision in ("fp64", "mixed"):
        say(f"[gpu] full {name} {precision}")
        opts = ebit.default_opts(rtol=1e-9, precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
        ctx, dc = ebit.context_for(case, opts)
        ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
        if precision == "fp64":
            fl = torch.empty(case.ncells, dtype=torch.uint8, device="cuda")
            th = [torch.empty(ei.face_shape(case.dim, case.n, a), dtype=torch.float64, device="cuda")
                  for a in range(case.dim)]
            ctx.get_geometry(th, fl, None)
            assert np.array_equal(fl.cpu().numpy(), geo["flags"].ravel())
            for a in range(case.dim):
                tg = th[a].cpu().numpy()
                assert np.array_equal(np.isnan(tg), np.isnan(geo["theta"][a]))
                ok = ~np.isnan(tg)
                assert np.max(np.abs(tg[ok] - geo["theta"][a][ok]), initial=0) < 1e-13
        T = torch.zeros_like(dc.T0)
        sh = ctx.heat_solve(dc.T0, T)
        say("   heat", sh)
        # residual of the GPU temperature under the oracle's heat operator
        r = bH - opH.matvec(T.cpu().numpy().ravel())
        rr = np.linalg.norm(r) / np.linalg.norm(bH)
        say(f"   heat residual under the oracle operator: {rr:.2e}")
        assert rr < 2e-9
        if not heat_only:
            # mass flux of the seeded input temperature, at sampled interface cells
            m = torch.zeros_like(dc.T0)
            ctx.mass_flux(dc.T0, m)
            mg = m.cpu().numpy().ravel()
            err = np.max(np.abs(mg[smp] - mo_all[smp])) / np.max(np.abs(mo_all[smp]))
            say(f"   mass flux at {smp.size} sampled cells: max rel err {err:.1e}")
            assert err < 1e-12
            # projection driven by that mass flux: residual under the oracle's system
            p = torch.zeros_like(dc.T0)
            u_l = [u.clone() for u in dc.u_l]
            u_v = [u.clone() for u in dc.u_v]
            sp = ctx.project(u_l, u_v, m, p)
            say("   proj", sp)
            r = rhs - opP.matvec(p.cpu().numpy().ravel())
            rr = np.linalg.norm(r) / np.linalg.norm(rhs)
            say(f"   pressure residual under the oracle operator: {rr:.2e}")
            assert rr < 2e-9
            assert sp["div_max"] <= 2e-9 * np.linalg.norm(rhs)
        ctx.close()


def test_bubble3d_128_properties():
    _property_checks(ei.config(2), "C3 128^3")


def test_film3d_256_properties():
    _property_checks(ei.config(4), "C5 256^3", heat_only=False)
