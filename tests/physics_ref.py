"""Independent physics references for pinning the oracle.

Textbook solutions written from the mathematics, sharing nothing with the
oracle's discretisation:
  * the exact Riemann solver for the Euler equations of an ideal gas
    (pressure function with shock/rarefaction branches, root found by
    bracketing, self-similar sampling);
  * the Sedov-Taylor point blast: the similarity ODEs for a strong spherical
    shock integrated inward from the Rankine-Hugoniot state, and the energy
    integral that fixes xi_0 in R(t) = xi_0 (E t^2 / rho_0)^(1/5).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq


# ---------------------------------------------------------------------------
# Exact Riemann solver
# ---------------------------------------------------------------------------

def _pressure_fn(p, rho, pk, gamma):
    """Velocity jump across the wave connecting (rho, pk) to pressure p."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def exact_star(WL, WR, gamma):
    """(p*, u*) of the exact solution; W = (rho, u, p)."""
    rL, uL, pL = WL
    rR, uR, pR = WR

    def g(p):
        return _pressure_fn(p, rL, pL, gamma) + _pressure_fn(p, rR, pR, gamma) + (uR - uL)

    lo, hi = 1e-14 * min(pL, pR), max(pL, pR)
    while g(hi) < 0:
        hi *= 2.0
    ps = brentq(g, lo, hi, xtol=1e-15 * hi, rtol=4 * np.finfo(float).eps, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (_pressure_fn(ps, rR, pR, gamma) - _pressure_fn(ps, rL, pL, gamma))
    return ps, us


def exact_sample(WL, WR, gamma, s):
    """Exact solution (rho, u, p) at similarity coordinate s = x/t (scalar)."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    ps, us = exact_star(WL, WR, gamma)
    gm1, gp1 = gamma - 1.0, gamma + 1.0
    if s <= us:  # left of contact
        cL = math.sqrt(gamma * pL / rL)
        if ps > pL:
            SL = uL - cL * math.sqrt(gp1 / (2 * gamma) * ps / pL + gm1 / (2 * gamma))
            if s <= SL:
                return rL, uL, pL
            r = rL * ((ps / pL + gm1 / gp1) / (gm1 / gp1 * ps / pL + 1.0))
            return r, us, ps
        csL = cL * (ps / pL) ** (gm1 / (2 * gamma))
        if s <= uL - cL:
            return rL, uL, pL
        if s >= us - csL:
            return rL * (ps / pL) ** (1.0 / gamma), us, ps
        u = 2.0 / gp1 * (cL + gm1 / 2 * uL + s)
        c = 2.0 / gp1 * (cL + gm1 / 2 * (uL - s))
        r = rL * (c / cL) ** (2.0 / gm1)
        return r, u, pL * (c / cL) ** (2.0 * gamma / gm1)
    cR = math.sqrt(gamma * pR / rR)
    if ps > pR:
        SR = uR + cR * math.sqrt(gp1 / (2 * gamma) * ps / pR + gm1 / (2 * gamma))
        if s >= SR:
            return rR, uR, pR
        r = rR * ((ps / pR + gm1 / gp1) / (gm1 / gp1 * ps / pR + 1.0))
        return r, us, ps
    csR = cR * (ps / pR) ** (gm1 / (2 * gamma))
    if s >= uR + cR:
        return rR, uR, pR
    if s <= us + csR:
        return rR * (ps / pR) ** (1.0 / gamma), us, ps
    u = 2.0 / gp1 * (-cR + gm1 / 2 * uR + s)
    c = 2.0 / gp1 * (cR - gm1 / 2 * (uR - s))
    r = rR * (c / cR) ** (2.0 / gm1)
    return r, u, pR * (c / cR) ** (2.0 * gamma / gm1)


def shock_speed_right(WR, ps, gamma):
    rR, uR, pR = WR
    cR = math.sqrt(gamma * pR / rR)
    return uR + cR * math.sqrt((gamma + 1) / (2 * gamma) * ps / pR + (gamma - 1) / (2 * gamma))


# ---------------------------------------------------------------------------
# Sedov-Taylor blast (spherical, strong shock, uniform ambient at rest)
# ---------------------------------------------------------------------------

def _sedov_rhs(eta, y, gamma):
    """Similarity ODEs: u = R' f(eta), rho = rho0 g(eta), p = rho0 R'^2 h(eta),
    R ~ t^(2/5), from mass, momentum and entropy conservation."""
    f, g, h = y
    a = f - eta
    num = 1.5 * f * a - 3.0 * h / g + 2.0 * gamma * h * f / (g * eta)
    den = a * a - gamma * h / g
    fp = num / den
    gp = -g * (fp + 2.0 * f / eta) / a
    hp = h * (3.0 / a + gamma * gp / g)
    return [fp, gp, hp]


def sedov_profile(gamma, eta_min=1e-4, n=4001):
    """(eta, f, g, h) from the shock (eta=1) inward, Rankine-Hugoniot start."""
    y0 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    etas = np.linspace(1.0, eta_min, n)
    sol = solve_ivp(_sedov_rhs, (1.0, eta_min), y0, args=(gamma,), t_eval=etas, rtol=1e-11,
                    atol=1e-14, method="DOP853")
    return sol.t, sol.y[0], sol.y[1], sol.y[2]


def sedov_xi0(gamma) -> float:
    """xi_0 from the energy integral E = 4 pi rho0 R^3 R'^2 I, with
    R'^2 R^3 = (4/25) xi_0^5 E / rho0, I = int_0^1 (g f^2/2 + h/(gamma-1)) eta^2."""
    eta, f, g, h = sedov_profile(gamma)
    integrand = (0.5 * g * f * f + h / (gamma - 1.0)) * eta * eta
    I = -np.trapezoid(integrand, eta)  # eta decreasing
    return (25.0 / (16.0 * math.pi * I)) ** 0.2


def sedov_radius(E, t, rho0, gamma) -> float:
    return sedov_xi0(gamma) * (E * t * t / rho0) ** 0.2
