"""Pins of the oracle's raw-moment construction (the DBM the CDBM of Sec. 2
is contrasted with): its equilibrium equals the CDBM's (the sixteen moment
functions span the same space at raw and at peculiar velocities, so the
same f^eq satisfies both sets of constraints), its quadrature reproduces the
central moments of Eq. (4), and its nonequilibrium measures are the
binomial shifts of the central ones of Eqs. (8)-(11)."""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W


def _states(n=40, seed=5):
    rng = np.random.default_rng(seed)
    rho = torch.as_tensor(rng.uniform(0.5, 2.0, n))
    ux = torch.as_tensor(rng.uniform(-0.3, 0.3, n))
    uy = torch.as_tensor(rng.uniform(-0.3, 0.3, n))
    T = torch.as_tensor(rng.uniform(0.5, 2.0, n))
    return rho, ux, uy, T


@pytest.mark.parametrize("vset,I", [("sound", 3.0), ("lax", 8.0), ("tg", 0.0)])
def test_raw_equilibrium_equals_central_equilibrium(vset, I):
    v, eta = W.VELOCITY_SETS[vset]
    vel, et = C.discrete_velocities(v, eta)
    st = _states()
    raw = C.raw_equilibrium(*st, I, vel, et)
    cen = C.equilibrium(*st, I, vel, et)
    err = float((raw - cen).abs().max() / cen.abs().max())
    assert err < 1e-11, err


def test_quadrature_moments_at_rest_are_the_central_closed_forms():
    """At u = 0 raw and central moments coincide: the quadrature must give the
    closed forms of Eq. (4) ((D+I) rho T, rho T, (D+I+2) rho T^2 ...)."""
    rho, _, _, T = _states()
    z = torch.zeros_like(rho)
    for I in (0.0, 1.0, 3.0, 8.0):
        got = C.raw_equilibrium_moments(rho, z, z, T, I)
        want = C.central_equilibrium_moments(rho, T, I)
        assert float((got - want).abs().max()) <= 1e-12 * float(want.abs().max())


def test_quadrature_moments_shift_with_the_flow():
    """Raw moments of a drifting Maxwellian by hand: sum v_x = rho u_x,
    sum v_x^2 = rho (u_x^2 + T), sum v_x^3 = rho u_x (u_x^2 + 3T),
    sum (|v|^2 + eta^2) = rho (|u|^2 + (D + I) T)."""
    rho, ux, uy, T = _states()
    I = 3.0
    m = C.raw_equilibrium_moments(rho, ux, uy, T, I)
    checks = {1: rho * ux, 2: rho * uy, 3: rho * (ux ** 2 + uy ** 2 + (2 + I) * T),
              4: rho * (ux ** 2 + T), 5: rho * ux * uy, 9: rho * ux * (ux ** 2 + 3 * T),
              10: rho * uy * (ux ** 2 + T)}
    for r, want in checks.items():
        assert float((m[:, r] - want).abs().max()) <= 1e-12 * float(want.abs().max() + 1), r


def _field(seed=6, n=10, steps=3):
    run = W.random_periodic(n, n, seed=seed, dt=2e-3, tau=5e-2, vset="tg")
    p = C.Params.from_run(run)
    f = C.run(C.initial_distribution(run.rho, run.ux, run.uy, run.T, p), p, steps)
    return p, f


def test_raw_measures_are_shifts_of_the_central_ones():
    """With delta = f - f^eq, whose mass, momentum and energy sums vanish,
    v = v* + u gives: Delta_2 = Delta*_2; Delta_{3,1,a} = Delta*_{3,1,a} +
    2 sum_b Delta*_{2,ab} u_b; Delta_{3,abc} = Delta*_{3,abc} + u_a Delta*_{2,bc}
    + u_b Delta*_{2,ac} + u_c Delta*_{2,ab}."""
    p, f = _field()
    raw = C.raw_nonequilibrium(f, p)
    cen = C.nonequilibrium(f, p)
    _, ux, uy, _ = C.fields(f, p)
    u = (ux, uy)
    d2 = {(0, 0): cen[0], (0, 1): cen[1], (1, 0): cen[1], (1, 1): cen[2]}
    scale = float(cen.abs().max())
    assert scale > 1e-8
    tol = 1e-9 * scale
    for k in range(3):
        assert float((raw[k] - cen[k]).abs().max()) <= tol
    for a in range(2):
        want = cen[3 + a] + 2 * (d2[(a, 0)] * u[0] + d2[(a, 1)] * u[1])
        assert float((raw[3 + a] - want).abs().max()) <= tol
    # Delta_3 slots xxx, xxy, xyy, yyy
    for slot, (a, b, c) in enumerate(((0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1))):
        want = cen[5 + slot] + u[a] * d2[(b, c)] + u[b] * d2[(a, c)] + u[c] * d2[(a, b)]
        assert float((raw[5 + slot] - want).abs().max()) <= tol


def test_raw_measures_equal_central_ones_at_rest():
    """A field with u = 0 everywhere: M(u) = M0, so every slot agrees."""
    n = 8
    x = W.cell_centres(n, 1.0 / n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * X)
    T = 1.0 / rho
    z = np.zeros_like(rho)
    v, eta = W.VELOCITY_SETS["sound"]
    p = C.Params(n, n, 1.0 / n, 1.0 / n, 1e-4, 1e-4, 3.0, v, eta)
    f = C.initial_distribution(rho, z, z, T, p)
    # a non-equilibrium part that keeps rho, j and 2E (so u stays 0)
    d = torch.zeros(16, n, n, dtype=torch.float64)
    d[0] = d[2] = 1e-3
    d[1] = d[3] = -1e-3
    f = f + d
    raw = C.raw_nonequilibrium(f, p)
    cen = C.nonequilibrium(f, p)
    assert float((raw - cen).abs().max()) <= 1e-10 * float(cen.abs().max())
