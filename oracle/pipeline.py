"""One pass of the elliptic hot path, in the order of the paper's time step
(Sec. 2.5: diffusion of T, then mass flux and ghost velocities, then the
projection), all in plain FP64 with direct solves."""
from __future__ import annotations

from . import flux, geometry, heat, project, solve


def run_step(case, T_star, u_l, u_v, theta_min=1e-3, solver=solve.direct):
    geo = geometry.build(case)
    A, b = heat.assemble(case, geo, T_star, theta_min)
    T = solver(A, b, heat.operator(case, geo, theta_min))
    mdot, fallbacks = flux.mass_flux(case, geo, T, theta_min)
    pr = project.project(case, geo, mdot, u_l, u_v, solver)
    return dict(geo=geo, A_heat=A, b_heat=b, T=T, mdot=mdot, fallbacks=fallbacks, **pr)
