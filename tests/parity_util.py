"""Shared helpers of the GPU parity tests: the oracle's reference step (direct
or multigrid solve), the element-wise per-phase comparisons and the face
update bound for velocities.

Bars (applied by check_step):
  * T and p: element by element, per phase: max |GPU - oracle| over the
    phase's cells, over the largest |oracle| value of that phase (of the
    whole field when the phase's values are all below 1e-8 of it, i.e. a
    phase whose discrete solution is 0), <= 1e-12;
  * mdot: element by element on the interface cells, over max |mdot|;
    mdot on cut faces: the same NaN layout and values, over max |mdot|;
  * u: face by face, within what the face update u -= beta_f grad p makes of
    the measured pressure difference dp (beta_f (|dp_lo| + |dp_up|)/h, or
    2 beta_f |dp_c|/h on an outflow face), plus 1e-12 of the update (each
    side's theta, so beta_f on cut faces, agrees to ~1e-13) and of the ghost
    jump on cut faces (linear in mdot_f), plus rounding: the velocities are
    exactly the update of each side's own p;
  * u in relative L2 per phase field: <= max(1e-12, 0.5 x the FP64
    representation floor of p seen through beta_f/h), the level observed
    (the rounding of p alone moves u by up to that floor).
"""
import sys

import numpy as np

import oracle
from oracle import flux, geometry, heat, mg, project

EPS = np.finfo(float).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def phase_err(g, r, col):
    """{phase: max |g - r| over the phase / the phase's scale}.

    The scale is the largest |oracle value| in the phase.  A phase whose
    values are all below 1e-8 of the whole field's largest (a phase held at
    T_sat with a zero right-hand side: its discrete solution is 0, and both
    sides return their solver's rounding noise there) is measured against
    the whole field's scale instead."""
    g = np.asarray(g, float).ravel()
    r = np.asarray(r, float).ravel()
    col = np.asarray(col).ravel()
    whole = np.max(np.abs(r)) if r.size else 0.0
    out = {}
    for k in (0, 1):
        m = col == k
        if not np.any(m):
            continue
        sc = np.max(np.abs(r[m]))
        if sc < 1e-8 * whole:
            sc = whole
        d = np.max(np.abs(g[m] - r[m]))
        out[k] = d / sc if sc > 0 else d
    return out


def velocity_floor(case, geo, p, u_l):
    """Relative L2 size, on u_l, of the eps-level rounding of p through the
    face update u -= beta_f (p_up - p_lo)/h."""
    num = 0.0
    for a in range(case.dim):
        beta = project.face_beta(case, geo, a)
        lo, up = flux._face_cells(case, a)
        both = (lo >= 0) & (up >= 0)
        d = beta[both] * EPS * (np.abs(p[lo[both]]) + np.abs(p[up[both]])) / case.h
        num += np.sum(d * d)
    return np.sqrt(num) / np.sqrt(sum(np.sum(x * x) for x in u_l))


def update_bound(case, geo, dp):
    """Per axis, the most the face update can move a face velocity for a
    pressure error dp (per cell)."""
    out = []
    adp = np.abs(np.asarray(dp).ravel())
    for a in range(case.dim):
        beta = np.nan_to_num(project.face_beta(case, geo, a))
        lo, up = flux._face_cells(case, a)
        b = np.zeros(beta.shape)
        both = (lo >= 0) & (up >= 0)
        b[both] = beta[both] * (adp[lo[both]] + adp[up[both]]) / case.h
        only = (lo >= 0) ^ (up >= 0)
        cell = np.where(lo >= 0, lo, up)
        b[only] = 2.0 * beta[only] * adp[cell[only]] / case.h
        out.append(b)
    return out


def face_slack(bnd, u_ref, u_star, jump=0.0):
    """Allowance for |u_GPU - u_oracle| on each face: what the pressure
    difference makes of it (bnd); 1e-12 of the update u_ref - u* (beta_f on
    cut faces comes from each side's theta) and of the ghost jump
    mdot_f [1/rho] n on cut faces (mdot agrees to 1e-12); rounding."""
    return (1.001 * bnd + 1e-12 * (np.abs(u_ref - u_star) + np.abs(jump))
            + 4 * EPS * (np.abs(u_ref) + np.max(np.abs(u_ref))))


def reference_step(case, solver="direct", threads=0, log=say):
    """The oracle's step on the case's seeded inputs: geometry, heat solve,
    mass flux of T, ghost velocities, pressure solve, face update.  With
    solver='mg' the systems are solved by the oracle's multigrid (grids too
    large to factor); the sequence of calls is the oracle pipeline's."""
    if solver == "direct":
        return oracle.pipeline.run_step(case, case.T0, case.u_l, case.u_v)
    geo = geometry.build(case)
    log("   oracle: geometry built")
    opH = heat.operator(case, geo)
    bH = heat.rhs(case, geo, case.T0)
    info = {}
    T = mg.solve_op(opH, bH, threads=threads, info=info)
    log(f"   oracle: heat solved ({info['pcg_iters']} PCG iterations, rel_res {info['rel_res']:.1e})")
    del opH
    mdot, fb = flux.mass_flux(case, geo, T)
    log(f"   oracle: mass flux ({int(np.count_nonzero(geo['is_if']))} interface cells)")
    ulg, uvg = project.ghost_velocities(case, geo, mdot, case.u_l, case.u_v)
    rhs = project.divergence(case, ulg, uvg) - project.bc_rhs(case, geo)
    opP = project.operator(case, geo)
    info = {}
    p = mg.solve_op(opP, -rhs, threads=threads, info=info)
    log(f"   oracle: pressure solved ({info['pcg_iters']} PCG iterations, rel_res {info['rel_res']:.1e})")
    del opP
    ul1, uv1 = project.face_update(case, geo, p, ulg, uvg)
    return dict(geo=geo, b_heat=bH, T=T, mdot=mdot, fallbacks=fb, p=p, u_l=ul1, u_v=uv1, b=rhs,
                u_l_ghost=ulg, u_v_ghost=uvg)


def check_step(case, ref, g, tol=1e-12, log=say):
    """Assert the bars of the module docstring for one GPU step ``g`` (numpy
    fields T, mdot, mface, p, u_l, u_v) against the oracle's ``ref``; returns
    the observed levels."""
    col = case.ccol.ravel()
    geo = ref["geo"]
    obs = {}
    obs["T"] = phase_err(g["T"], ref["T"], col)
    obs["p"] = phase_err(g["p"], ref["p"], col)
    iface = geo["is_if"]
    msc = max(np.max(np.abs(ref["mdot"])), 1e-300)
    obs["mdot"] = np.max(np.abs(g["mdot"][iface] - ref["mdot"][iface]), initial=0.0) / msc
    off = ~iface
    assert np.all(g["mdot"][off] == 0.0)
    if g.get("mface") is not None:
        mf_ref = flux.mass_flux_faces(case, geo, ref["mdot"])
        e = 0.0
        for a in range(case.dim):
            assert np.array_equal(np.isnan(mf_ref[a]), np.isnan(g["mface"][a])), a
            ok = ~np.isnan(mf_ref[a])
            e = max(e, np.max(np.abs(g["mface"][a][ok] - mf_ref[a][ok]), initial=0.0) / msc)
        obs["mdot_face"] = e
    bnd = update_bound(case, geo, g["p"] - ref["p"])
    worst = 0.0
    for name_u, ghost in (("u_l", "u_l_ghost"), ("u_v", "u_v_ghost")):
        for a in range(case.dim):
            du = np.abs(g[name_u][a] - ref[name_u][a])
            cut = ~np.isnan(geo["theta"][a])
            jump = np.where(cut, ref["u_l_ghost"][a] - ref["u_v_ghost"][a], 0.0)
            sl = face_slack(bnd[a], ref[name_u][a], ref[ghost][a], jump)
            worst = max(worst, float(np.max(du / sl)))
    obs["u_face_vs_update_bound"] = worst
    fl = {}
    for name_u in ("u_l", "u_v"):
        obs[name_u] = rel(np.concatenate([x.ravel() for x in g[name_u]]),
                          np.concatenate([x.ravel() for x in ref[name_u]]))
        fl[name_u] = velocity_floor(case, geo, ref["p"], ref[name_u])
        obs[name_u + "_floor"] = fl[name_u]
    log("   observed", {k: (f"{v:.1e}" if np.isscalar(v) else {q: f"{w:.1e}" for q, w in v.items()})
                        for k, v in obs.items()})
    for k in ("T", "p"):
        for ph, v in obs[k].items():
            assert v <= tol, (k, ph, v)
    assert obs["mdot"] <= tol
    if "mdot_face" in obs:
        assert obs["mdot_face"] <= tol
    assert worst <= 1.0, worst
    for name_u in ("u_l", "u_v"):
        assert obs[name_u] <= max(tol, 0.5 * fl[name_u]), (name_u, obs[name_u], fl[name_u])
    return obs
