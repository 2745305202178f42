"""Pins of the oracle adjoint: reverse-mode products against central finite
differences of the forward definition, on tiny grids."""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W


def _setup(nx=8, ny=6, seed=3, bc_x=C.PERIODIC, noise=0.05):
    run = W.random_periodic(nx, ny, seed=seed, dt=2e-4, tau=4e-4)
    run.bc_x = bc_x
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    rng = np.random.default_rng(seed + 10)
    # push f off equilibrium so the relaxation and minmod branches are all exercised
    f = f * (1 + noise * torch.from_numpy(rng.standard_normal(f.shape)))
    return run, p, f, rng


@pytest.mark.parametrize("bc_x", [C.PERIODIC, C.ZERO_GRADIENT])
def test_step_vjp_matches_central_differences(bc_x):
    run, p, f, rng = _setup(bc_x=bc_x)
    lam = torch.from_numpy(rng.standard_normal(f.shape))
    gf, gtau = C.step_vjp(f, lam, p)
    for _ in range(3):
        d = torch.from_numpy(rng.standard_normal(f.shape)) * f.abs().mean()
        h = 1e-6
        fd = ((C.step(f + h * d, p) - C.step(f - h * d, p)) * lam).sum() / (2 * h)
        ad = (gf * d).sum()
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * (gf.abs() * d.abs()).sum()), (fd, ad)
    ht = p.tau * 1e-5
    fd_tau = ((C.step(f, p, p.tau + ht) - C.step(f, p, p.tau - ht)) * lam).sum() / (2 * ht)
    assert abs(fd_tau - gtau) <= 1e-6 * abs(gtau)


def test_multi_step_vjp_chain_and_dot_product():
    # smooth state and smooth direction: minmod switches between near-equal
    # slopes then cost the finite difference only O(h) instead of O(1)
    run, p, f0, rng = _setup(nx=6, ny=5, noise=0.0)
    n = 5
    lam_end = torch.from_numpy(rng.standard_normal(f0.shape))
    # chain the one-step products backwards
    states = [f0]
    for _ in range(n):
        states.append(C.step(states[-1], p))
    lam = lam_end
    gtau = 0.0
    for k in reversed(range(n)):
        lam, gt = C.step_vjp(states[k], lam, p)
        gtau += gt
    d = f0 * torch.from_numpy(W.fourier_field(rng, run.nx, run.ny))[None] * \
        torch.from_numpy(rng.uniform(0.5, 1.5, (16, 1, 1)))
    h = 1e-6
    fd = ((C.run(f0 + h * d, p, n) - C.run(f0 - h * d, p, n)) * lam_end).sum() / (2 * h)
    assert abs(fd - (lam * d).sum()) <= 1e-6 * abs(fd)
    ht = p.tau * 1e-5
    fdt = ((C.run(f0, p, n, p.tau + ht) - C.run(f0, p, n, p.tau - ht)) * lam_end).sum() / (2 * ht)
    assert abs(fdt - gtau) <= 1e-6 * abs(gtau)


def test_init_and_moment_vjps_match_central_differences():
    run, p, f, rng = _setup()
    lam = torch.from_numpy(rng.standard_normal(f.shape))
    fields = [torch.from_numpy(a.copy()) for a in (run.rho, run.ux, run.uy, run.T)]
    grads = C.init_vjp(*fields, lam, p)
    for k in range(4):
        d = torch.from_numpy(rng.standard_normal(fields[k].shape))
        h = 1e-6
        plus = [a.clone() for a in fields]
        minus = [a.clone() for a in fields]
        plus[k] += h * d
        minus[k] -= h * d
        fd = ((C.initial_distribution(*plus, p) - C.initial_distribution(*minus, p)) * lam).sum() / (2 * h)
        assert abs(fd - (grads[k] * d).sum()) <= 1e-6 * abs(fd)
    g = [torch.from_numpy(rng.standard_normal(run.rho.shape)) for _ in range(4)]
    gf = C.moments_vjp(f, *g, p)
    d = torch.from_numpy(rng.standard_normal(f.shape))
    h = 1e-7
    outp = C.fields(f + h * d, p)
    outm = C.fields(f - h * d, p)
    fd = sum(((a - b) * gg).sum() for a, b, gg in zip(outp, outm, g)) / (2 * h)
    assert abs(fd - (gf * d).sum()) <= 1e-6 * abs(fd)
