"""Parity of the HIP forward path (init, fused step, moments, nonequilibrium,
totals) with the FP64 oracle, through the C ABI."""
import functools
import sys

import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W
from helpers import field_errors, oracle_after, oracle_f0, rel_l2, rel_max, to_np

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1   # CDBM_FP64, CDBM_MIXED of include/cdbm.h
AUTO, FUSED, SPLIT = 0, 1, 2   # CDBM_STEP_* of include/cdbm.h
FORMS = {"fused": FUSED, "split": SPLIT}


def _solver(run, precision, form=AUTO):
    from paper_2502_16818_amd import Solver
    print(f"[case] {run.name} {run.nx}x{run.ny} precision={precision} step_form={form}", flush=True)
    return Solver.from_run(run, precision, form)


def _cases():
    sod = W.sod_tube(nx=137, steps=3)
    lax = W.lax_tube(nx=150, dx=2e-3)
    rnd = W.random_periodic(137, 23, seed=1, dt=1e-4, tau=2e-4)     # 3 strips, ragged tail
    tg = W.taylor_green_paper(n=40)
    acl = W.lax_acoustic_2d(130, ny=19, seed=2)
    zg = W.random_periodic(61, 9, seed=5, dt=1e-4, tau=1e-4)
    zg.bc_x = W.ZERO_GRADIENT
    zg.bc_y = W.ZERO_GRADIENT
    tiny = W.random_periodic(3, 2, seed=6, dt=1e-4, tau=1e-4)
    one = W.random_periodic(1, 1, seed=7, dt=1e-4, tau=1e-4)
    return [sod, lax, rnd, tg, acl, zg, tiny, one] + _chunked_cases()


def _chunked_cases():
    """Widths that are multiples of four: the step moves rows in 16-byte
    chunks (both precisions), including strips whose loaded columns wrap or
    meet a zero-gradient side, and grids narrower than one strip."""
    rnd4 = W.random_periodic(136, 23, seed=11, dt=1e-4, tau=2e-4)   # 3 strips, ragged tail
    zg4 = W.random_periodic(68, 9, seed=12, dt=1e-4, tau=1e-4)
    zg4.bc_x = W.ZERO_GRADIENT
    zg4.bc_y = W.ZERO_GRADIENT
    zgx = W.random_periodic(124, 11, seed=13, dt=1e-4, tau=1e-4)
    zgx.bc_x = W.ZERO_GRADIENT
    narrow = W.random_periodic(8, 5, seed=14, dt=1e-4, tau=1e-4)
    for r, tag in ((rnd4, "rnd4"), (zg4, "zg4"), (zgx, "zgx"), (narrow, "narrow")):
        r.name = f"{r.name}_{tag}"
    return [rnd4, zg4, zgx, narrow]


@pytest.mark.parametrize("run", _cases(), ids=lambda r: r.name)
def test_init_moments_tne_fp64(run):
    s = _solver(run, FP64)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    p, f0 = oracle_f0(run)
    assert rel_max(to_np(f), f0.numpy()) < 1e-12
    got = [to_np(a) for a in s.moments(f)]
    want = [run.rho, run.ux, run.uy, run.T]
    for g, w in zip(got, want):
        assert np.abs(g - w).max() <= 1e-12 * max(np.abs(w).max(), 1.0)
    # nonequilibrium of a perturbed state
    rng = np.random.default_rng(0)
    pert = f0 * (1 + 0.01 * torch.from_numpy(rng.standard_normal(f0.shape)))
    fg = torch.from_numpy(np.ascontiguousarray(pert.numpy())).cuda()
    d_gpu = to_np(s.tne(fg))
    d_ref = C.nonequilibrium(pert, p).numpy()
    # f^eq of the two sides differ by ~cond(M) eps; the measures cancel f
    # against f^eq, so compare against the scale of sum_i |f_i Psi_i|
    assert np.abs(d_gpu - d_ref).max() <= 1e-9 * np.abs(d_ref).max()


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("run", _cases(), ids=lambda r: r.name)
@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_step_fp64_matches_oracle(run, nsteps, form):
    s = _solver(run, FP64, FORMS[form])
    f = s.init(run.rho, run.ux, run.uy, run.T)
    out = s.step(f, nsteps=nsteps)
    _, ref = oracle_after(run, nsteps)
    err = rel_max(to_np(out), ref.numpy())
    print(f"  max rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("form", sorted(FORMS))
def test_step_fp64_long_random_run(form):
    run = W.random_periodic(96, 70, seed=3, dt=1e-4, tau=2e-4)
    s = _solver(run, FP64, FORMS[form])
    f = s.init(run.rho, run.ux, run.uy, run.T)
    out = s.step(f, nsteps=60)       # takes the captured-graph path (>= 32 steps)
    p, ref = oracle_after(run, 60)
    got = [to_np(a) for a in s.moments(out)]
    want = [a.numpy() for a in C.fields(ref, p)]
    errs = field_errors(got, want, u_scale=0.29)
    print(errs)
    assert max(errs.values()) < 1e-12


@pytest.mark.slow
def test_sod_tube_full_run_fp64():
    """The 500 x 1 Sod tube, 5000 steps (t = 0.1), against the oracle."""
    run = W.sod_tube()
    s = _solver(run, FP64)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    out = s.step(f, nsteps=run.steps)
    p, ref = oracle_after(run, run.steps)
    got = [to_np(a) for a in s.moments(out)]
    want = [a.numpy() for a in C.fields(ref, p)]
    errs = field_errors(got, want, u_scale=1.0)
    print(errs)
    assert max(errs.values()) < 1e-12


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("run", _cases()[:6] + _chunked_cases(), ids=lambda r: r.name)
def test_step_mixed_against_fp64_oracle(run, form):
    s = _solver(run, MIXED, FORMS[form])
    f = s.init(run.rho, run.ux, run.uy, run.T)
    n = 20
    out = s.step(f, nsteps=n)
    p, ref = oracle_after(run, n)
    got = [to_np(a) for a in s.moments(out)]
    want = [a.numpy() for a in C.fields(ref, p)]
    umax = max(np.abs(want[1]).max(), np.abs(want[2]).max(), 1e-2)
    errs = field_errors(got, want, u_scale=umax)
    # non-equilibrium moments: they cancel f against f^eq, so the FP32
    # rounding of f (6e-8 of sum_i |f_i Psi_i|, grown over the steps) is not
    # small against them; the bound is 1 % of their largest value plus 1e-5
    # of that rounding scale (an equilibrium state has moments of rounding
    # size only)
    d_ref = C.nonequilibrium(ref, p).numpy()
    vel, eta = C.discrete_velocities(p.v, p.eta)
    _, ux, uy, _ = C.fields(ref, p)
    M = C.moment_matrix(ux.reshape(-1), uy.reshape(-1), vel, eta)[:, 4:, :]
    scale = float(torch.einsum("nri,ni->nr", M.abs(), ref.reshape(16, -1).t().abs()).max())
    d_err = float(np.abs(to_np(s.tne(out)) - d_ref).max())
    errs["tne"] = d_err / (np.abs(d_ref).max() + 1e-3 * scale)
    print(errs)
    assert errs["rho"] < 1e-5 and errs["T"] < 1e-5
    assert errs["ux"] < 1e-4 and errs["uy"] < 1e-4
    assert d_err <= 1e-2 * np.abs(d_ref).max() + 1e-5 * scale


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_fused_and_split_steps_are_bitwise_equal(precision):
    """Both step forms evaluate the same per-cell arithmetic in the same order;
    only where f^(1) lives (LDS or HBM) differs."""
    for run in [_cases()[2], _cases()[5]] + _chunked_cases()[:3]:
        outs = []
        for form in (FUSED, SPLIT):
            s = _solver(run, precision, form)
            f = s.init(run.rho, run.ux, run.uy, run.T)
            outs.append(s.step(f, nsteps=7))
            s.close()
        assert torch.equal(outs[0], outs[1]), run.name


@functools.lru_cache(maxsize=1)
def _piece_cases():
    """Grids whose FP32 launch splits every strip into row pieces and gives
    the strips' remaining rows (tails) to the compute units the pieces leave
    idle, with one to five tails per unit (on 256 compute units), on both
    row-movement forms and boundary kinds."""
    out = []
    for nx, ny, bc, tag in ((1001, 777, (0, 0), "percol"), (1000, 777, (1, 1), "zg"),
                            (1536, 1536, (0, 0), "k2"), (2048, 2048, (1, 0), "k5"),
                            (4096, 1000, (0, 1), "k4")):
        r = W.random_periodic(nx, ny, seed=nx + ny, dt=2e-5, tau=2e-4)
        r.bc_x, r.bc_y = bc
        r.name = f"{r.name}_{tag}"
        out.append(r)
    return out


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_fused_pieces_and_tails_equal_split_steps(precision):
    """Mid-size grids in the fused form (row pieces, strip tails on the spare
    compute units, several segments per block) against the split form, which
    reads every neighbour from HBM and has no pieces: bitwise equal over the
    whole grid after three steps."""
    for run in _piece_cases():
        outs = []
        for form in (FUSED, SPLIT):
            s = _solver(run, precision, form)
            f = s.init(run.rho, run.ux, run.uy, run.T)
            outs.append(s.step(f, nsteps=3))
            s.close()
            del f
        assert torch.equal(outs[0], outs[1]), run.name
        del outs


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_graph_replays_match_eager_steps(precision, form):
    """Long cdbm_step calls replay a captured graph of 32 steps (on torch's
    null stream as well); every replay must equal the same steps launched one
    call at a time.  The graph is replayed again after other work on the
    handle and with a longer run (two replays per call)."""
    run = _chunked_cases()[0]
    s = _solver(run, precision, FORMS[form])
    f0 = s.init(run.rho, run.ux, run.uy, run.T)
    eager = {}
    f = f0.clone()
    for k in range(1, 97):
        f = s.step(f)            # one step per call: no graph
        if k in (64, 96):
            eager[k] = f.clone()
    out = s.empty_f()
    for rep in range(3):
        s.step(f0, out, nsteps=64)
        torch.cuda.synchronize()
        assert torch.equal(out, eager[64]), rep
        _ = s.moments(s.step(f0, nsteps=3))   # other work on the handle in between
        torch.cuda.synchronize()
    s.step(f0, out, nsteps=96)
    torch.cuda.synchronize()
    assert torch.equal(out, eager[96])
    s.close()


def test_binding_rejects_wrong_buffers():
    """Wrong element type, too few elements or a strided view never reach the
    kernels: the binding raises before the call."""
    run = W.random_periodic(64, 8, seed=3, dt=1e-4, tau=1e-4)
    s = _solver(run, MIXED)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    with pytest.raises(ValueError, match="dtype"):
        s.step(f.double())
    with pytest.raises(ValueError, match="elements"):
        s.step(f[:, :4].contiguous())
    with pytest.raises(ValueError, match="contiguous"):
        s.step(f, s.empty_f().transpose(1, 2))
    with pytest.raises(ValueError, match="float64"):
        s.step_adjoint(f, torch.zeros_like(f))
    s.close()


def test_conserved_totals_periodic_fp64():
    run = W.random_periodic(64, 40, seed=9, dt=1e-4, tau=1e-4)
    s = _solver(run, FP64)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    t0 = to_np(s.totals(f))
    p, f0 = oracle_f0(run)
    vel, eta = C.discrete_velocities(p.v, p.eta)
    psis = [torch.ones(16, dtype=C.DT), vel[:, 0], vel[:, 1], vel[:, 0] ** 2 + vel[:, 1] ** 2 + eta ** 2]
    want = [float((f0 * ps.reshape(16, 1, 1)).sum()) for ps in psis]
    np.testing.assert_allclose(t0, want, rtol=1e-12, atol=1e-12 * abs(want[3]))
    out = s.step(f, nsteps=200)
    t1 = to_np(s.totals(out))
    np.testing.assert_allclose(t1, t0, rtol=0, atol=1e-12 * abs(t0[3]))


def test_nsteps_zero_copies_and_overlap_is_rejected():
    from paper_2502_16818_amd import CdbmError
    run = W.random_periodic(16, 8, seed=2)
    s = _solver(run, FP64)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    out = s.step(f, nsteps=0)
    assert torch.equal(out, f)
    with pytest.raises(CdbmError):
        s.step(f, f, nsteps=1)


def test_init_rejects_nonphysical_fields():
    from paper_2502_16818_amd import CdbmError
    run = W.random_periodic(16, 8, seed=2)
    s = _solver(run, FP64)
    rho = run.rho.copy()
    rho[3, 4] = -1.0
    with pytest.raises(CdbmError) as e:
        s.init(rho, run.ux, run.uy, run.T)
    assert e.value.code == -3
    T = run.T.copy()
    T[0, 0] = np.nan
    with pytest.raises(CdbmError):
        s.init(run.rho, run.ux, run.uy, T)
