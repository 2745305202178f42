"""Closed-form reference solutions used to check the oracle (test infrastructure)."""
from __future__ import annotations

import math

import numpy as np

D = 2


def taylor_green(x, y, t, u0=0.01, p0=1.0, L=0.05, Re=1.0):
    """Eqs. (22)-(24): decaying Taylor-Green vortex on [0, 2L]^2."""
    k = np.pi / L
    ex = np.exp(-2.0 * np.pi ** 2 * u0 * t / (Re * L))
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * ex
    uy = u0 * np.sin(k * x) * np.cos(k * y) * ex
    p = p0 - p0 * u0 ** 2 / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * ex ** 2
    return ux, uy, p


def relative_l2(num, exact, u0):
    """Eq. (25): sqrt(mean(((num - exact) / u0)^2))."""
    num = np.asarray(num)
    exact = np.asarray(exact)
    return float(np.sqrt(np.mean(((num - exact) / u0) ** 2)))


def ce_delta2_xx(rho, T, tau, I, dux_dx, duy_dy):
    """Eq. (21): Chapman-Enskog estimate of Delta*_{2,xx}."""
    return 2.0 * rho * T * tau * ((1.0 - D - I) / (D + I) * dux_dx + 1.0 / (D + I) * duy_dy)


def ce_delta2_yy(rho, T, tau, I, dux_dx, duy_dy):
    """Eq. (21) with the roles of x and y exchanged (isotropy of the model)."""
    return ce_delta2_xx(rho, T, tau, I, duy_dy, dux_dx)


def sound_speed(gamma, T):
    """Adiabatic sound speed of the gas p = rho T: c = sqrt(gamma T), the sound speed named after Eq. (3)."""
    return math.sqrt(gamma * T)


def acoustic_plane_wave(x, rho0, T0, gamma, amp, k):
    """Right-running isentropic plane wave of the linearised Euler equations.

    drho = amp rho0 cos(k x), du = c drho / rho0, dT = (gamma - 1) T0 drho / rho0.
    """
    c = sound_speed(gamma, T0)
    drho = amp * rho0 * np.cos(k * x)
    return rho0 + drho, c * drho / rho0, T0 + (gamma - 1.0) * T0 * drho / rho0


def normal_shock(Ma, gamma, rho1=1.0, p1=1.0):
    """Rankine-Hugoniot state behind a shock of Mach number Ma moving into gas at rest.

    Returns (rho2, u2, T2, p2, shock_speed) with p = rho T.
    """
    g = gamma
    r = (g + 1.0) * Ma ** 2 / ((g - 1.0) * Ma ** 2 + 2.0)
    pr = (2.0 * g * Ma ** 2 - (g - 1.0)) / (g + 1.0)
    c1 = math.sqrt(g * p1 / rho1)
    s = Ma * c1
    rho2 = rho1 * r
    p2 = p1 * pr
    u2 = s * (1.0 - rho1 / rho2)
    return rho2, u2, p2 / rho2, p2, s
