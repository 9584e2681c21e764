"""Pins for the oracle's ghost fill and mass flux.

Independent references: the linear Stefan profile (the ghost extrapolation
and the two-point normal gradient are exact for it), the quasi-steady mass
flux of the Stefan closed form (Sec. 3.1), the erf bubble profile whose
interfacial gradient is known in closed form (O(h^2) convergence), and the
normal-gradient formula's exactness for quadratic profiles along the normal.
"""
import math

import numpy as np
import pytest

import ebit_inputs as ei
from oracle import closed, flux, geometry, heat, solve


def test_stefan_mass_flux_exact_for_linear_profile():
    c = ei.config(0)
    g = geometry.build(c)
    m, fb = flux.mass_flux(c, g, c.T0.ravel())
    pr = c.props
    expect = pr.lam_v * 1.0 / (0.3 * pr.h_lg)          # lam_v dT / (x_Gamma h_lg)
    iface = g["is_if"]
    assert fb == 0
    assert np.max(np.abs(m[iface] - expect)) < 1e-13 * expect
    assert np.all(m[~iface] == 0.0)
    # the ghost layer: vapour ghost in the first liquid column continues the line
    gh = flux.ghost_fill(c, g, c.T0.ravel()).reshape(c.T0.shape)
    x19 = 19.5 / 64
    assert np.allclose(gh[0, :, 19], 1.0 - x19 / 0.3, atol=1e-14)
    assert np.allclose(gh[0, :, 18], 0.0, atol=1e-15)    # liquid ghost at T_sat side
    assert np.all(np.isnan(gh[0, :, :18])) and np.all(np.isnan(gh[0, :, 20:]))


def test_stefan_quasi_steady_closed_form():
    """Sec. 3.1 closed form at X_Gamma = 0.3: the front's mass flux with the
    linear profile agrees with the similarity solution to O(beta^2)."""
    c = ei.config(0)
    pr = c.props
    beta = closed.stefan_beta(pr.cp_v, 1.0, pr.h_lg)
    alpha_v = pr.lam_v / (pr.rho_v * pr.cp_v)
    t = (0.3 / (2 * beta)) ** 2 / alpha_v
    assert abs(closed.stefan_position(t, beta, alpha_v) - 0.3) < 1e-14
    m_exact = closed.stefan_mdot(t, beta, alpha_v, pr.lam_v, 1.0, 0.0, pr.h_lg)
    g = geometry.build(c)
    m, _ = flux.mass_flux(c, g, c.T0.ravel())
    rel = abs(m[g["is_if"]][0] - m_exact) / m_exact
    assert rel < beta ** 2, (rel, beta)
    # and the discrete profile of the closed form at that time gives the
    # same mass flux to O(h^2) + O(beta^2)
    xc = (np.arange(64) + 0.5) / 64
    T = np.where(c.ccol[0] == 0, closed.stefan_T(xc[None, :], t, beta, alpha_v, 1.0, 0.0), 0.0)
    m2, _ = flux.mass_flux(c, g, T.ravel())
    assert abs(m2[g["is_if"]][0] - m_exact) / m_exact < 1e-3


def _bubble_mdot_error(n):
    c = ei.bubble(2, n, 0.1, 1.0, 0.02, 1000.0, 0.1)
    g = geometry.build(c)
    m, fb = flux.mass_flux(c, g, c.T0.ravel())
    exact = c.props.lam_l * 1.0 * 2.0 / (math.sqrt(math.pi) * 0.02) / c.props.h_lg
    return np.max(np.abs(m[g["is_if"]] - exact)) / exact, fb


def test_bubble_erf_mass_flux_converges():
    """Liquid T = erf((r - R)/delta): dT/dr at r = R is 2/(sqrt(pi) delta)."""
    errs = []
    for n in (256, 512, 1024):
        e, fb = _bubble_mdot_error(n)
        assert fb == 0
        errs.append(e)
    assert errs[-1] < 2e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.36 * e0, errs


@pytest.mark.parametrize("theta_cells", [19.2, 19.03, 19.51, 19.97])
def test_normal_gradient_quadratic_exact_away_from_ghosts(theta_cells):
    """Eq. normal_gradient is exact for T = T_G + g s + c s^2 when the two
    points' blocks see only real cells of the phase: a liquid-side quadratic
    with a vapour layer, checked from the liquid side."""
    n = 64
    c = ei.stefan_2d(n, x_gamma_cells=theta_cells)
    xg = theta_cells / n
    xc = (np.arange(n) + 0.5) / n
    gq, cq = 0.7, -3.1
    s = xc - xg
    T = np.where(c.ccol[0] == 1, gq * s + cq * s * s, 0.0)[None, None, :] * np.ones((1, n, 1))
    g = geometry.build(c)
    ghost = flux.ghost_fill(c, g, T.ravel())
    cen = g["cF"][g["is_if"]][0]
    vals = []
    for d in (1.0 / n, 2.0 / n):
        P = cen + d * np.array([1.0, 0.0, 0.0])
        # shift so that the block is fully liquid
        centre = [int(np.floor(P[0] * n)) + 1, 10, 0]
        vals.append(flux._interp(c, 1, T, ghost, P, centre))
    d1, d2 = 1.0 / n, 2.0 / n
    D = (d2 / d1 * vals[0] - d1 / d2 * vals[1]) / (d2 - d1)
    assert abs(D - gq) < 1e-10


def test_first_order_fallback_on_a_thin_slab():
    """A liquid slab 1.45 h thick (y in [8.905 h, 10.355 h]): one row of
    liquid centres (row 9), the interface cells in rows 8 and 10 with flat
    facets at y = 8.905 h (normal +y) and y = 10.355 h (normal -y).  On the
    liquid side the second point (2h along the normal) lands two rows past
    the slab, where neither a liquid cell nor a one-layer ghost exists, so
    the gradient falls back to the first-order difference from the liquid
    centre nearest the first point: the row-9 cell straight across, at 0.595 h
    (row 8) or 0.855 h (row 10) from the facet along the normal.  The vapour
    is at T_sat, so its side adds nothing.  Hence, worked out by hand,
        mdot = lam_l (T_9 - T_sat) / (0.595 h) / h_lg   in row 8,
        mdot = lam_l (T_9 - T_sat) / (0.855 h) / h_lg   in row 10,
    with one fallback per interface cell."""
    case = ei.thin_slab_2d()
    nx, ny = case.n[0], case.n[1]
    h = case.h
    g = geometry.build(case)
    x = (np.arange(nx) + 0.5) * h
    T = np.zeros((ny, nx))
    T[9] = 1.0 + 0.3 * np.sin(2 * np.pi * x)
    m, fb = flux.mass_flux(case, g, T.ravel())
    m = m.reshape(ny, nx)
    pr = case.props
    assert sorted(set(np.nonzero(g["is_if"])[0] // nx)) == [8, 10]
    assert fb == 2 * nx
    for row, dist in ((8, 0.595), (10, 0.855)):
        expect = pr.lam_l * (T[9] - pr.T_sat) / (dist * h) / pr.h_lg
        assert np.max(np.abs(m[row] - expect)) <= 1e-13 * np.max(np.abs(expect)), row
    others = np.ones(ny, bool)
    others[[8, 10]] = False
    assert np.all(m[others] == 0.0)
