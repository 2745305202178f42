"""Pins of the oracle's space and time discretisation (Eqs. (12)-(20), RK2).

minmod is checked against the median of (X, Y, 0); the NND derivative is
checked for exactness on linear profiles, second-order convergence on smooth
periodic profiles, upwinding direction and the total-variation property; the
two-stage Runge-Kutta step against the closed form of uniform BGK relaxation
and against global conservation.
"""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W


def test_minmod_equals_median_with_zero():
    rng = np.random.default_rng(5)
    X = rng.standard_normal(20000) * 10 ** rng.uniform(-6, 3, 20000)
    Y = rng.standard_normal(20000) * 10 ** rng.uniform(-6, 3, 20000)
    special = np.array([0.0, -0.0, 1.0, -1.0, 2.0, -2.0, 3.5, -3.5])
    SX, SY = np.meshgrid(special, special)
    X = np.concatenate([X, SX.ravel(), [1.5, -1.5]])
    Y = np.concatenate([Y, SY.ravel(), [1.5, -1.5]])
    got = C.minmod(torch.from_numpy(X), torch.from_numpy(Y)).numpy()
    want = np.median(np.stack([X, Y, np.zeros_like(X)]), axis=0)
    np.testing.assert_array_equal(got, want)


def _profile_derivative(fx, v, dx, bc):
    """v df/dx of a single-velocity profile through the oracle's NND operator."""
    n = fx.size
    f = torch.zeros(16, 1, n, dtype=C.DT)
    f[:] = torch.from_numpy(fx)
    vr = torch.full((16,), float(v), dtype=C.DT)
    idx = C.ghost_index(n, bc)
    return C.nnd_derivative(f.index_select(2, idx), vr, dx, 2)[0, 0].numpy()


@pytest.mark.parametrize("v", [1.3, -0.7])
def test_nnd_exact_on_linear_profiles(v):
    n, dx = 40, 0.01
    x = W.cell_centres(n, dx)
    fx = 2.0 + 3.0 * x
    d = _profile_derivative(fx, v, dx, C.ZERO_GRADIENT)
    np.testing.assert_allclose(d[3:-3], v * 3.0, rtol=1e-12)


@pytest.mark.parametrize("v", [1.0, -1.0])
def test_nnd_second_order_on_smooth_profile(v):
    errs = []
    ns = [64, 128, 256, 512]
    for n in ns:
        dx = 1.0 / n
        x = W.cell_centres(n, dx)
        fx = 1.5 + np.sin(2 * np.pi * x)
        d = _profile_derivative(fx, v, dx, C.PERIODIC)
        errs.append(np.mean(np.abs(d - v * 2 * np.pi * np.cos(2 * np.pi * x))))
    order = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert -2.2 < order < -1.8, order


def _pure_advection(f0, p, steps):
    """Evolve with relaxation switched off (tau -> infinity)."""
    big = dict(p.__dict__)
    big["tau"] = 1e300
    q = C.Params(**big)
    return C.run(f0, q, steps)


def test_upwind_direction_and_speed():
    n = 200
    dx = 1.0 / n
    x = W.cell_centres(n, dx)
    bump = np.exp(-((x - 0.3) / 0.04) ** 2)
    v, eta = W.VELOCITY_SETS["sound"]
    p = C.Params(n, 1, dx, dx, 1e-3, 1e300, 3.0, v, eta, C.PERIODIC, C.PERIODIC)
    vel, _ = C.discrete_velocities(v, eta)
    f0 = torch.from_numpy(np.broadcast_to(1.0 + bump, (16, 1, n)).copy())
    steps = 100
    f = _pure_advection(f0, p, steps)
    t = steps * p.dt
    for i in range(16):
        prof = f[i, 0].numpy() - 1.0
        # circular mean of the bump position
        ang = np.angle(np.sum(prof * np.exp(2j * np.pi * x))) / (2 * np.pi) % 1.0
        expect = (0.3 + vel[i, 0].item() * t) % 1.0
        dist = min(abs(ang - expect), 1 - abs(ang - expect))
        assert dist < 0.5 * dx, (i, ang, expect)


def test_total_variation_does_not_grow():
    n = 100
    dx = 1.0 / n
    x = W.cell_centres(n, dx)
    step_prof = np.where((x > 0.2) & (x < 0.5), 2.0, 1.0)
    v, eta = W.VELOCITY_SETS["sound"]
    p = C.Params(n, 1, dx, dx, 2e-3, 1e300, 3.0, v, eta, C.PERIODIC, C.PERIODIC)
    f = torch.from_numpy(np.broadcast_to(step_prof, (16, 1, n)).copy())
    tv0 = np.abs(np.diff(np.r_[step_prof, step_prof[0]])).sum()
    for _ in range(40):
        f = _pure_advection(f, p, 1)
        for i in range(16):
            prof = f[i, 0].numpy()
            tv = np.abs(np.diff(np.r_[prof, prof[0]])).sum()
            assert tv <= tv0 + 1e-12
            assert prof.max() <= 2.0 + 1e-12 and prof.min() >= 1.0 - 1e-12


def _conserved_null_perturbation(vel, eta, rng):
    """A perturbation of f with zero mass, momentum and energy."""
    psi = torch.stack([torch.ones(16, dtype=C.DT), vel[:, 0], vel[:, 1],
                       vel[:, 0] ** 2 + vel[:, 1] ** 2 + eta ** 2])       # (4, 16)
    g = torch.from_numpy(rng.standard_normal(16))
    q, _ = torch.linalg.qr(psi.t())
    return g - q @ (q.t() @ g)


@pytest.mark.parametrize("z", [0.2, 1.0, 1.7])
def test_uniform_relaxation_follows_rk2_amplification(z):
    """A uniform state f = f^eq + delta (delta carrying no conserved moment)
    relaxes as delta (1 - z + z^2/2)^n with z = dt / tau, and rho, u, T stay put."""
    run = W.uniform(3, 2, rho=1.2, ux=0.1, uy=-0.05, T=0.9)
    p = C.Params.from_run(run)
    p.tau = p.dt / z
    vel, eta = C.discrete_velocities(p.v, p.eta)
    feq = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    delta = 0.01 * _conserved_null_perturbation(vel, eta, np.random.default_rng(2))
    f = feq + delta.reshape(16, 1, 1)
    nsteps = 7
    out = C.run(f, p, nsteps)
    amp = (1.0 - z + 0.5 * z * z) ** nsteps
    want = feq + amp * delta.reshape(16, 1, 1)
    np.testing.assert_allclose(out.numpy(), want.numpy(), rtol=0, atol=1e-13 * feq.abs().max().item() * 10)
    r, ux, uy, T = C.fields(out, p)
    np.testing.assert_allclose(r.numpy(), 1.2, rtol=1e-13)
    np.testing.assert_allclose(T.numpy(), 0.9, rtol=1e-13)


def test_equilibrium_is_a_fixed_point():
    run = W.uniform(4, 4, rho=0.7, ux=0.2, uy=0.1, T=1.3)
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    out = C.run(f, p, 5)
    np.testing.assert_allclose(out.numpy(), f.numpy(), rtol=0, atol=1e-14 * 50)


@pytest.mark.parametrize("vset,bc", [("sound", C.PERIODIC), ("tg", C.PERIODIC)])
def test_global_conservation_periodic(vset, bc):
    run = W.random_periodic(24, 20, seed=4, vset=vset, dt=2e-4, tau=2e-4)
    p = C.Params.from_run(run)
    vel, eta = C.discrete_velocities(p.v, p.eta)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    psis = [torch.ones(16, dtype=C.DT), vel[:, 0], vel[:, 1],
            vel[:, 0] ** 2 + vel[:, 1] ** 2 + eta ** 2]

    def totals(g):
        return [float((g * ps.reshape(16, 1, 1)).sum()) for ps in psis]

    t0 = totals(f)
    f = C.run(f, p, 150)
    t1 = totals(f)
    scale = float((f.abs() * psis[3].reshape(16, 1, 1)).sum())
    for a, b in zip(t0, t1):
        assert abs(a - b) <= 1e-12 * scale
