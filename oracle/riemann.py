"""Exact Riemann solver for the 1D Euler equations of an ideal gas (test infrastructure).

The shock-tube benchmarks of Secs. 3.1-3.3 are compared with the exact
Riemann solution.  The solver below is the standard one: the star pressure
p* is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the
Rankine-Hugoniot shock branch for p > p_K and the isentropic rarefaction
branch for p <= p_K; u* follows from the same functions and the solution is
sampled self-similarly in x/t.  The gas has p = rho T (m = 1) and sound speed
c = sqrt(gamma p / rho).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.optimize import brentq


@dataclasses.dataclass
class State:
    rho: float
    u: float
    p: float


def _f_and_branch(p: float, s: State, g: float) -> float:
    c = math.sqrt(g * s.p / s.rho)
    if p > s.p:   # shock: f = (p - pK) sqrt(A / (p + B))
        A = 2.0 / ((g + 1.0) * s.rho)
        B = (g - 1.0) / (g + 1.0) * s.p
        return (p - s.p) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * c / (g - 1.0) * ((p / s.p) ** ((g - 1.0) / (2.0 * g)) - 1.0)


@dataclasses.dataclass
class StarState:
    p: float
    u: float
    rho_L: float
    rho_R: float


def star_state(L: State, R: State, g: float) -> StarState:
    def fun(p):
        return _f_and_branch(p, L, g) + _f_and_branch(p, R, g) + (R.u - L.u)

    lo, hi = 1e-14, max(L.p, R.p)
    while fun(hi) < 0:
        hi *= 2.0
    ps = brentq(fun, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (L.u + R.u) + 0.5 * (_f_and_branch(ps, R, g) - _f_and_branch(ps, L, g))

    def rho_star(s: State):
        if ps > s.p:
            r = ps / s.p
            k = (g - 1.0) / (g + 1.0)
            return s.rho * (r + k) / (k * r + 1.0)
        return s.rho * (ps / s.p) ** (1.0 / g)

    return StarState(ps, us, rho_star(L), rho_star(R))


def shock_speed(s: State, ps: float, g: float, side: int) -> float:
    """Speed of a shock running into state s (side = -1 left wave, +1 right wave)."""
    c = math.sqrt(g * s.p / s.rho)
    return s.u + side * c * math.sqrt((g + 1.0) / (2.0 * g) * ps / s.p + (g - 1.0) / (2.0 * g))


def sample(L: State, R: State, g: float, xi: np.ndarray):
    """rho, u, p of the exact solution at similarity coordinates xi = (x - x0) / t."""
    st = star_state(L, R, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    cL = math.sqrt(g * L.p / L.rho)
    cR = math.sqrt(g * R.p / R.rho)
    for k, s in enumerate(xi.flat):
        if s <= st.u:   # left of the contact
            if st.p > L.p:
                SL = shock_speed(L, st.p, g, -1)
                val = (L.rho, L.u, L.p) if s <= SL else (st.rho_L, st.u, st.p)
            else:
                cs = cL * (st.p / L.p) ** ((g - 1.0) / (2.0 * g))
                head, tail = L.u - cL, st.u - cs
                if s <= head:
                    val = (L.rho, L.u, L.p)
                elif s >= tail:
                    val = (st.rho_L, st.u, st.p)
                else:
                    w = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (L.u - s)
                    val = (L.rho * w ** (2.0 / (g - 1.0)),
                           2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * L.u + s),
                           L.p * w ** (2.0 * g / (g - 1.0)))
        else:           # right of the contact
            if st.p > R.p:
                SR = shock_speed(R, st.p, g, +1)
                val = (R.rho, R.u, R.p) if s >= SR else (st.rho_R, st.u, st.p)
            else:
                cs = cR * (st.p / R.p) ** ((g - 1.0) / (2.0 * g))
                head, tail = R.u + cR, st.u + cs
                if s >= head:
                    val = (R.rho, R.u, R.p)
                elif s <= tail:
                    val = (st.rho_R, st.u, st.p)
                else:
                    w = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (R.u - s)
                    val = (R.rho * w ** (2.0 / (g - 1.0)),
                           2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * R.u + s),
                           R.p * w ** (2.0 * g / (g - 1.0)))
        rho.flat[k], u.flat[k], p.flat[k] = val
    return rho, u, p
