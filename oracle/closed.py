"""Closed-form solutions used to pin the oracle (paper Sec. 3.1, 3.3).

Stefan problem (Sec. 3.1): X_Gamma(t) = 2 beta sqrt(alpha_v t) with beta the
root of beta exp(beta^2) erf(beta) = cp_v (T_w - T_sat)/(sqrt(pi) h_lg), and
the vapour profile T(x, t) = T_w + (T_sat - T_w) erf(x/(2 sqrt(alpha_v t)))/erf(beta).
Constant-mdot bubble (Sec. 3.3): R(t) = R0 + mdot t / rho_vap.
"""
from __future__ import annotations

import math

from scipy.optimize import brentq
from scipy.special import erf


def stefan_beta(cp_v, dT, h_lg):
    rhs = cp_v * dT / (math.sqrt(math.pi) * h_lg)
    return brentq(lambda b: b * math.exp(b * b) * erf(b) - rhs, 1e-12, 10.0, xtol=1e-15, rtol=1e-15)


def stefan_position(t, beta, alpha_v):
    return 2.0 * beta * math.sqrt(alpha_v * t)


def stefan_T(x, t, beta, alpha_v, T_w, T_sat):
    return T_w + (T_sat - T_w) * erf(x / (2.0 * math.sqrt(alpha_v * t))) / erf(beta)


def stefan_mdot(t, beta, alpha_v, lam_v, T_w, T_sat, h_lg):
    """Interface mass flux of the Stefan solution: lam_v |dT/dx| / h_lg at X_Gamma."""
    s = 2.0 * math.sqrt(alpha_v * t)
    dTdx = (T_sat - T_w) / erf(beta) * 2.0 / math.sqrt(math.pi) * math.exp(-beta * beta) / s
    return lam_v * (-dTdx) / h_lg


def bubble_radius(t, R0, mdot, rho_v):
    return R0 + mdot * t / rho_v
