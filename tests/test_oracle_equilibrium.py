"""Pins of the oracle's equilibrium, moments and nonequilibrium measures.

Each check compares the oracle with something other than itself: Gauss-Hermite
quadrature of the continuous Maxwellian (Eq. (5)), the rank of the moment
matrix under the paper's velocity sets, conservation identities written out
here, and the Chapman-Enskog estimate printed as Eq. (21).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import cdbm as C
from oracle import analytic as A
import workloads as W

RNG = np.random.default_rng(1234)


def _gh(n):
    x, w = np.polynomial.hermite_e.hermegauss(n)
    return x, w / math.sqrt(2.0 * math.pi)


def maxwellian_expectation(fun, ux, uy, T, I, n=24):
    """E[fun(vx, vy, eta)] under Eq. (5) by tensor Gauss-Hermite quadrature."""
    x, w = _gh(n)
    vx = ux + math.sqrt(T) * x[:, None, None]
    vy = uy + math.sqrt(T) * x[None, :, None]
    eta = math.sqrt(I * T) * x[None, None, :]
    ww = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return float(np.sum(ww * fun(vx, vy, eta)))


# The 16 constraint functions of Eq. (4) written as functions of the raw
# velocity v (not v - u): a different basis of the same span, evaluated here
# independently of the oracle's moment matrix.
def _e(vx, vy, eta):
    return vx * vx + vy * vy + eta * eta


RAW = [
    lambda vx, vy, eta: np.ones_like(vx * vy * eta),
    lambda vx, vy, eta: vx + 0 * eta,
    lambda vx, vy, eta: vy + 0 * eta,
    lambda vx, vy, eta: _e(vx, vy, eta),
    lambda vx, vy, eta: vx ** 2 + 0 * eta,
    lambda vx, vy, eta: vx * vy + 0 * eta,
    lambda vx, vy, eta: vy ** 2 + 0 * eta,
    lambda vx, vy, eta: _e(vx, vy, eta) * vx,
    lambda vx, vy, eta: _e(vx, vy, eta) * vy,
    lambda vx, vy, eta: vx ** 3 + 0 * eta,
    lambda vx, vy, eta: vx ** 2 * vy + 0 * eta,
    lambda vx, vy, eta: vx * vy ** 2 + 0 * eta,
    lambda vx, vy, eta: vy ** 3 + 0 * eta,
    lambda vx, vy, eta: _e(vx, vy, eta) * vx ** 2,
    lambda vx, vy, eta: _e(vx, vy, eta) * vx * vy,
    lambda vx, vy, eta: _e(vx, vy, eta) * vy ** 2,
]


def random_states(k, vset):
    v, eta = W.VELOCITY_SETS[vset]
    out = []
    for _ in range(k):
        out.append((RNG.uniform(0.3, 3.0), RNG.uniform(-0.5, 0.5), RNG.uniform(-0.5, 0.5),
                    RNG.uniform(0.5, 2.0), RNG.choice([0.985, 1.0, 3.0, 8.0, 18.0])))
    return v, eta, out


def test_paper_velocity_sets_nonsingular(golden_dir):
    sets = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["velocity_sets"]
    for name, s in sets.items():
        if name.startswith("_"):
            continue
        vel, eta = C.discrete_velocities(s["v"], s["eta"])
        M0 = C.moment_matrix(torch.zeros(1, dtype=C.DT), torch.zeros(1, dtype=C.DT), vel, eta)[0]
        assert torch.linalg.matrix_rank(M0).item() == 16, name
        assert torch.linalg.cond(M0).item() < 1e7, name


def test_degenerate_sets_are_singular():
    # all eta zero: the energy rows lose their independent eta^2 part
    vel, eta = C.discrete_velocities((1.4, 1.1, 1.1, 1.0), (0, 0, 0, 0))
    M0 = C.moment_matrix(torch.zeros(1, dtype=C.DT), torch.zeros(1, dtype=C.DT), vel, eta)[0]
    assert torch.linalg.matrix_rank(M0).item() < 16
    # the literal reading of "(+-1, 0)" for the axis groups duplicates velocities
    vel2 = vel.clone()
    vel2[1] = vel2[0]
    vel2[3] = vel2[2]
    M1 = C.moment_matrix(torch.zeros(1, dtype=C.DT), torch.zeros(1, dtype=C.DT), vel2, eta + 1.0)[0]
    assert torch.linalg.matrix_rank(M1).item() < 16


def test_gamma_and_extra_dof():
    # gamma = (D + I + 2) / (D + I) with D = 2: I = 0 <-> gamma = 2, I = 3 <-> 1.4
    for g, I in ((2.0, 0.0), (1.4, 3.0), (5.0 / 3.0, 1.0), (1.2, 8.0)):
        assert abs(C.extra_dof_from_gamma(g) - I) < 1e-12


@pytest.mark.parametrize("vset", ["sod", "lax", "sound", "tg"])
def test_central_moment_closed_forms_match_quadrature(vset):
    """The closed forms used for fbar^eq equal the Maxwellian's central moments."""
    v, eta, states = random_states(4, vset)
    for rho, ux, uy, T, I in states:
        got = C.central_equilibrium_moments(torch.tensor([rho], dtype=C.DT),
                                            torch.tensor([T], dtype=C.DT), I)[0].numpy()
        # central moments: functions of c = v - u (quadrature about u = 0)
        want = np.array([rho * maxwellian_expectation(f, 0.0, 0.0, T, I) for f in RAW])
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("vset", ["sod", "lax", "sound", "tg", "shock"])
def test_equilibrium_reproduces_maxwellian_raw_moments(vset):
    """sum_i f_i^eq Psi(v_i) equals the integral of Eq. (5) against Psi, for
    all 16 constraint functions, written in raw velocities."""
    v, eta4, states = random_states(4, vset)
    vel, eta = C.discrete_velocities(v, eta4)
    scale = 1.0 if vset != "shock" else 10.0
    for rho, ux, uy, T, I in states:
        ux, uy, T = ux * scale, uy * scale, T * scale ** 2
        feq = C.equilibrium(torch.tensor([rho], dtype=C.DT), torch.tensor([ux], dtype=C.DT),
                            torch.tensor([uy], dtype=C.DT), torch.tensor([T], dtype=C.DT),
                            I, vel, eta)[0].numpy()
        vx, vy, et = vel[:, 0].numpy(), vel[:, 1].numpy(), eta.numpy()
        for k, fun in enumerate(RAW):
            disc = float(np.sum(feq * fun(vx, vy, et)))
            cont = rho * maxwellian_expectation(fun, ux, uy, T, I)
            ref = rho * maxwellian_expectation(lambda a, b, c: np.abs(fun(a, b, c)), ux, uy, T, I)
            assert abs(disc - cont) <= 1e-11 * max(ref, 1.0), (vset, k, disc, cont)


@pytest.mark.parametrize("vset", ["sod", "lax", "sound", "tg"])
def test_macroscopic_recovers_state(vset):
    v, eta4, states = random_states(6, vset)
    vel, eta = C.discrete_velocities(v, eta4)
    for rho, ux, uy, T, I in states:
        args = [torch.tensor([a], dtype=C.DT) for a in (rho, ux, uy, T)]
        feq = C.equilibrium(*args, I, vel, eta)          # (1, 16)
        r2, ux2, uy2, T2 = C.macroscopic(feq.t(), vel, eta, I)
        np.testing.assert_allclose([r2.item(), ux2.item(), uy2.item(), T2.item()],
                                   [rho, ux, uy, T], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("vset", ["sod", "lax", "sound", "tg"])
def test_collision_conserves_mass_momentum_energy(vset):
    """sum_i (f_i - f_i^eq(f)) psi_i = 0 for psi = 1, v_x, v_y, |v|^2 + eta^2."""
    run = W.random_periodic(6, 5, seed=7, vset=vset)
    p = C.Params.from_run(run)
    vel, eta = C.discrete_velocities(p.v, p.eta)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    g = torch.from_numpy(np.random.default_rng(3).standard_normal(f.shape))
    f = f + 0.05 * g * f.abs().mean()
    feq = C.equilibrium_of(f, p, vel, eta)
    neq = f - feq
    vx, vy, et = (t.reshape(16, 1, 1) for t in (vel[:, 0], vel[:, 1], eta))
    for psi in (torch.ones_like(vx), vx, vy, vx * vx + vy * vy + et * et):
        lhs = (neq * psi).sum(0)
        scale = ((f.abs() + feq.abs()) * psi.abs()).sum(0)
        # rounding of a 16x16 solve with cond(M) ~ 1e2..1e3
        assert (lhs.abs() / scale).max().item() < 1e-12


def test_nonequilibrium_vanishes_at_equilibrium():
    run = W.random_periodic(8, 6, seed=11)
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    d = C.nonequilibrium(f, p)
    assert d.shape == (12, 6, 8)
    assert d.abs().max().item() < 1e-12 * f.abs().max().item() * 10


def test_nonequilibrium_row_order():
    """Delta*_2 is symmetric-tensor ordered (xx, xy, yy): a deviation carrying
    only an xy-shear moment shows up in the xy slot and nowhere in the
    second-order xx, yy slots, and it flips sign with the deviation."""
    run = W.uniform(1, 1, ux=0.1, uy=-0.05, T=1.1)
    p = C.Params.from_run(run)
    vel, eta = C.discrete_velocities(p.v, p.eta)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    # perturb along the diagonal velocities with the vx*vy sign pattern: it adds
    # an xy second moment and leaves mass, momentum and energy unchanged
    sgn = torch.sign(vel[:, 0] * vel[:, 1])
    grp = torch.zeros(16, dtype=C.DT)
    grp[4:8] = 1.0
    pert = (0.01 * sgn * grp).reshape(16, 1, 1)
    d_plus = C.nonequilibrium(f + pert, p)[:, 0, 0]
    d_minus = C.nonequilibrium(f - pert, p)[:, 0, 0]
    assert abs(d_plus[1].item()) > 1e-3
    assert abs(d_plus[0].item()) < 1e-12 and abs(d_plus[2].item()) < 1e-12
    np.testing.assert_allclose(d_plus.numpy(), -d_minus.numpy(), atol=1e-13)


@pytest.mark.slow
def test_delta2_xx_matches_chapman_enskog():
    """Eq. (21) against the oracle in a smooth 1D compression/expansion flow."""
    n = 200
    dx = 1.0 / n
    x = W.cell_centres(n, dx)
    U = 0.02
    rho = np.ones((1, n))
    ux = (U * np.sin(2 * np.pi * x))[None, :]
    uy = np.zeros((1, n))
    T = np.ones((1, n))
    v, eta = W.VELOCITY_SETS["sound"]
    run = W.Run("ce", n, 1, dx, dx, 2e-5, 2e-4, 1.4, v, eta, W.PERIODIC, W.PERIODIC, 0,
                rho, ux, uy, T)
    p = C.Params.from_run(run)
    f = C.initial_distribution(rho, ux, uy, T, p)
    f = C.run(f, p, 100)   # t = 10 tau: the nonequilibrium part has relaxed onto its CE value
    r, u, _, Tn = (a.numpy()[0] for a in C.fields(f, p))
    d = C.nonequilibrium(f, p).numpy()[:, 0, :]
    dudx = (np.roll(u, -1) - np.roll(u, 1)) / (2 * dx)
    ce = A.ce_delta2_xx(r, Tn, p.tau, p.I, dudx, 0.0)
    big = np.abs(ce) > 0.5 * np.abs(ce).max()
    rel = np.abs(d[0][big] - ce[big]) / np.abs(ce).max()
    assert rel.max() < 0.1, rel.max()
    # the yy component follows Eq. (21) with x and y exchanged
    ce_yy = A.ce_delta2_yy(r, Tn, p.tau, p.I, dudx, 0.0)
    rel_yy = np.abs(d[2][big] - ce_yy[big]) / np.abs(ce_yy).max()
    assert rel_yy.max() < 0.1, rel_yy.max()
