"""Nonequilibrium measures of the raw-moment construction on the HIP path
(cdbm_tne_raw) against the oracle's raw_nonequilibrium, and beside the
central ones (cdbm_tne) on a shock tube in motion."""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W
from helpers import oracle_f0, to_np

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def _solver(run, precision):
    from paper_2502_16818_amd import Solver
    print(f"[case] {run.name} {run.nx}x{run.ny} bc=({run.bc_x},{run.bc_y}) precision={precision}",
          flush=True)
    return Solver.from_run(run, precision)


def _cases():
    a = W.random_periodic(37, 23, seed=1, dt=1e-4, tau=2e-4)
    b = W.random_periodic(40, 1, seed=3, dt=1e-4, tau=1e-4, vset="lax")
    c = W.random_periodic(19, 33, seed=4, dt=1e-4, tau=1e-4, vset="tg")
    return [a, b, c]


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("run", _cases(), ids=lambda r: r.name)
def test_raw_tne_matches_oracle(run, precision):
    """A perturbed (non-equilibrium) state in the handle's storage type; the
    oracle gets the same stored values, so both evaluate the measures of the
    same f in FP64 (the mixed form only stores f in FP32)."""
    p, f0 = oracle_f0(run)
    rng = np.random.default_rng(2)
    # small enough that T stays positive (the raw moments of the oracle are
    # quadratures of a Maxwellian of temperature T)
    pert = f0 * (1 + 1e-4 * torch.from_numpy(rng.standard_normal(f0.shape)))
    assert float(C.fields(pert, p)[3].min()) > 0
    s = _solver(run, precision)
    fg = pert.to(s.dtype).cuda().contiguous()
    stored = fg.double().cpu()
    got = to_np(s.tne_raw(fg))
    want = C.raw_nonequilibrium(stored, p).numpy()
    # the measures cancel f against f^eq, which the two sides compute in
    # different ways (to about cond(M0) eps of sum_i |f_i Psi_i|)
    vel, eta = C.discrete_velocities(p.v, p.eta)
    z = torch.zeros(1, dtype=torch.float64)
    M0 = C.moment_matrix(z, z, vel, eta)[0, 4:, :]
    scale = float((M0.abs() @ stored.reshape(16, -1).abs()).max())
    err = float(np.abs(got - want).max())
    print(f"  raw TNE max err {err:.2e}, max {np.abs(want).max():.2e}, scale {scale:.2e}")
    assert err <= 1e-9 * np.abs(want).max() + 1e-12 * scale
    cen = to_np(s.tne(fg))
    # second-order measures agree between the constructions (to rounding)
    assert np.abs(got[:3] - cen[:3]).max() <= 1e-9 * np.abs(cen[:3]).max()


def test_raw_and_central_measures_on_the_lax_tube():
    """The Sec. 3.2 Lax tube after 2000 steps (t = 0.04): where the gas
    moves, the raw heat-flux measure differs from the central one by the
    shift 2 Delta*_2 u of the second-order measure, which the raw measure
    mixes in; the central one is the heat flux alone."""
    run = W.lax_tube()
    s = _solver(run, FP64)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    g = s.step(f, nsteps=2000)
    raw = to_np(s.tne_raw(g))[:, 0, :]
    cen = to_np(s.tne(g))[:, 0, :]
    ux = to_np(s.moments(g)[1])[0]
    shift = 2 * cen[0] * ux
    scale = np.abs(cen[3]).max()
    assert np.abs(raw[3] - (cen[3] + shift)).max() <= 1e-9 * max(scale, np.abs(shift).max())
    # the shift is not small against the heat flux itself in the moving gas
    assert np.abs(shift).max() >= 0.1 * scale
    assert np.abs(raw[0] - cen[0]).max() <= 1e-9 * np.abs(cen[0]).max()
