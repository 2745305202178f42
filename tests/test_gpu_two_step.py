"""Two time steps per launch (CDBM_STEP_FUSED2, FP32 storage): bitwise equal
to the one-step fused launches, and against the oracle."""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W
from helpers import field_errors, oracle_after, to_np

pytestmark = pytest.mark.gpu

MIXED = 1
FUSED, FUSED2 = 1, 3


def _solver(run, form):
    from paper_2502_16818_amd import Solver
    print(f"[case] {run.name} {run.nx}x{run.ny} bc=({run.bc_x},{run.bc_y}) form={form}",
          flush=True)
    return Solver.from_run(run, MIXED, form)


def _cases():
    out = []
    for k, (nx, ny) in enumerate([(3, 2), (48, 7), (50, 37), (96, 40), (101, 64), (200, 130),
                                  (64, 300), (1, 33)]):
        r = W.random_periodic(nx, ny, seed=40 + k, dt=1e-4, tau=2e-4)
        r.bc_x = k % 2
        r.bc_y = (k // 2) % 2
        out.append(r)
    out.append(W.lax_acoustic_2d(n=256, ny=200, seed=1, steps=10))
    return out


@pytest.mark.parametrize("nsteps", [1, 2, 3, 8, 67])
@pytest.mark.parametrize("run", _cases(), ids=lambda r: f"{r.name}_bc{r.bc_x}{r.bc_y}")
def test_two_step_launch_equals_one_step_launches(run, nsteps):
    outs = []
    for form in (FUSED, FUSED2):
        s = _solver(run, form)
        f = s.init(run.rho, run.ux, run.uy, run.T)
        outs.append(s.step(f, nsteps=nsteps))
        torch.cuda.synchronize()
        s.close()
    assert torch.equal(outs[0], outs[1])


def test_two_step_against_oracle():
    run = W.random_periodic(70, 45, seed=5, dt=1e-4, tau=2e-4)
    s = _solver(run, FUSED2)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    out = s.step(f, nsteps=10)
    p, ref = oracle_after(run, 10)
    errs = field_errors([to_np(a) for a in s.moments(out)], [a.numpy() for a in C.fields(ref, p)],
                        u_scale=0.29)
    print(f"  10 steps, two per launch: {errs}")
    assert errs["rho"] < 1e-5 and errs["T"] < 1e-5 and errs["ux"] < 1e-4 and errs["uy"] < 1e-4


def test_two_step_headline_full_size():
    """The 4096 x 4096 throughput workload: 4 steps as two launches of two
    steps against four one-step launches, every value."""
    run = W.headline()
    outs = []
    for form in (FUSED, FUSED2):
        s = _solver(run, form)
        f = s.init(run.rho, run.ux, run.uy, run.T)
        outs.append(s.step(f, nsteps=4))
        torch.cuda.synchronize()
        del f
        s.close()
    assert torch.equal(outs[0], outs[1])


def test_two_step_graph_replays_match():
    """Runs of 64 or more pairs replay a captured graph: three replays with
    other work in between give the same bits."""
    run = W.random_periodic(130, 90, seed=9, dt=1e-4, tau=2e-4)
    s = _solver(run, FUSED2)
    f0 = s.init(run.rho, run.ux, run.uy, run.T)
    ref = s.step(f0, nsteps=130)
    out = s.empty_f()
    for rep in range(3):
        s.step(f0, out, nsteps=130)
        _ = s.step(f0, nsteps=3)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
