"""The throughput workload at its full size (4096 x 4096, zero-gradient x,
periodic y), in the launch configuration the benchmark times, against the
oracle on sampled cells.

f^{n+1} at a cell depends on f^n only within 4 cells along x or along y (two
Runge-Kutta stages of the 2-cell NND stencil), so the oracle's step on a
9 x 9 patch around the cell, cut from the GPU's own f^n, gives the cell's
exact f^{n+1} whatever boundary the patch itself gets: the patch boundary
reaches the centre only from 5 cells away.  At the domain's zero-gradient
x sides the patch is clipped to the domain and gets that boundary.  Samples
cover both x sides, the strip seams (every 120 columns in the mixed form,
every 56 in FP64), the seams of the
row pieces of any piece count up to 8, the periodic y wrap, and random
cells; both precision forms, two consecutive steps (from the equilibrium
start, then from a state with non-equilibrium parts).  Whole columns (every
row, against the oracle's step of the 9-column strip around them) cover the
row seams of whatever pieces and tails the launch assigns to blocks."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import cdbm as C
from helpers import check_column_step as _check_column
from helpers import check_patch_step as _check_step

FP64, MIXED = 0, 1


def _sample_cells(nx, ny, rng):
    seams = [k * 120 for k in (1, 2, 17, 33, 34)] + [k * 56 for k in (1, 2, 36, 72, 73)]
    xs_special = sorted({*range(0, 6), *range(nx - 6, nx),
                         *[c + d for c in seams for d in range(-3, 3) if 0 <= c + d < nx]})
    ys_special = {0, 1, 2, 3, ny - 4, ny - 3, ny - 2, ny - 1}
    for pieces in range(2, 9):
        length = -(-ny // pieces)
        for k in range(1, pieces):
            for d in (-2, -1, 0, 1):
                ys_special.add((k * length + d) % ny)
    ys_special = sorted(ys_special)
    cells = [(x, int(rng.integers(0, ny))) for x in xs_special]
    cells += [(int(rng.integers(0, nx)), y) for y in ys_special]
    cells += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(24)]
    cells += [(0, 0), (nx - 1, ny - 1), (0, ny - 1), (nx - 1, 0)]
    return cells


# Columns checked over their full height: inside the first strip, at a strip
# seam of each form, and at both zero-gradient sides.
FULL_COLUMNS = (0, 60, 2039, 2040, 4095)


def test_column_step_equals_full_grid_step():
    """The column check itself (CPU): on a small grid of the same setup, the
    oracle's step on the 9-column strip reproduces its full-grid step on the
    strip's centre column, at the zero-gradient sides and inside."""
    run = W.lax_acoustic_2d(40, ny=24, seed=3)
    p = C.Params.from_run(run)
    f0 = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    f0 = f0 * (1 + 1e-3 * torch.sin(torch.arange(f0.numel(), dtype=f0.dtype)).reshape(f0.shape))
    f1 = C.step(f0, p)
    for x in (0, 2, 4, 17, 35, 39):
        assert _check_column(run, f0, f1, x, FP64, tol=1e-14) <= 1e-14


def test_patch_step_equals_full_grid_step():
    """The sampling itself (CPU): on a small grid of the same setup, the
    oracle's step on each 9 x 9 patch reproduces its full-grid step at the
    patch centre, at the zero-gradient sides and across the periodic wrap."""
    run = W.lax_acoustic_2d(40, ny=24, seed=3)
    p = C.Params.from_run(run)
    f0 = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    f0 = f0 * (1 + 1e-3 * torch.sin(torch.arange(f0.numel(), dtype=f0.dtype)).reshape(f0.shape))
    f1 = C.step(f0, p)
    cells = [(0, 0), (1, 5), (3, 23), (4, 12), (20, 0), (35, 7), (36, 1), (39, 23), (38, 11)]
    assert _check_step(run, f0, f1, cells, FP64, tol=1e-14) <= 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_headline_full_size_sampled_cells_match_oracle(precision):
    from paper_2502_16818_amd import Solver
    run = W.headline(seed=0)
    print(f"[case] {run.name} {run.nx}x{run.ny} precision={precision}", flush=True)
    rng = np.random.default_rng(2024)
    cells = _sample_cells(run.nx, run.ny, rng)
    s = Solver.from_run(run, precision)
    f0 = s.init(run.rho, run.ux, run.uy, run.T)
    f1 = s.step(f0)
    f2 = s.step(f1)
    torch.cuda.synchronize()
    e1 = _check_step(run, f0, f1, cells, precision)
    e2 = _check_step(run, f1, f2, cells, precision)
    print(f"  {len(cells)} cells: worst relative error step 1 {e1:.2e}, step 2 {e2:.2e}")
    c1 = max(_check_column(run, f0, f1, x, precision) for x in FULL_COLUMNS)
    c2 = max(_check_column(run, f1, f2, x, precision) for x in FULL_COLUMNS)
    print(f"  {len(FULL_COLUMNS)} full columns: step 1 {c1:.2e}, step 2 {c2:.2e}")
    s.close()


# The largest grids of each row-movement form: the 16-byte-chunk form needs
# the f block below 2^32 bytes (32-bit offsets); one row more takes the
# per-column form with 64-bit offsets.
LARGEST = [(MIXED, 8192, 8192), (MIXED, 8192, 8193), (FP64, 4096, 8192), (FP64, 4096, 8193)]


@pytest.mark.gpu
@pytest.mark.slow
@pytest.mark.parametrize("precision,nx,ny", LARGEST,
                         ids=[f"{'fp64' if p == FP64 else 'mixed'}-{nx}x{ny}" for p, nx, ny in LARGEST])
def test_largest_grids_sampled_cells_match_oracle(precision, nx, ny):
    from paper_2502_16818_amd import Solver
    run = W.lax_acoustic_2d(nx, ny=ny, seed=4)
    print(f"[case] {run.name} {nx}x{ny} precision={precision}", flush=True)
    rng = np.random.default_rng(nx + ny)
    cells = [(x, int(rng.integers(0, ny))) for x in (0, 3, 55, 56, 119, 120, nx // 2, nx - 4, nx - 1)]
    cells += [(int(rng.integers(0, nx)), y) for y in (0, 1, ny // 2, ny - 2, ny - 1)]
    cells += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(8)]
    s = Solver.from_run(run, precision)
    f0 = s.init(run.rho, run.ux, run.uy, run.T)
    f1 = s.step(f0)
    torch.cuda.synchronize()
    e = _check_step(run, f0, f1, cells, precision)
    c = max(_check_column(run, f0, f1, x, precision) for x in (1, 120, nx - 2))
    print(f"  {len(cells)} cells: worst relative error {e:.2e}; 3 full columns {c:.2e}")
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_headline_full_size_run_matches_single_steps_and_oracle(precision):
    """The launch path the benchmark times: 36 steps in one call (two direct
    launches, a 32-step graph replay, two more launches) equal 36 single-step
    calls bit for bit, and the 36th step matches the oracle's step from the
    35th state on the sampled cells and full columns."""
    from paper_2502_16818_amd import Solver
    run = W.headline(seed=1)
    print(f"[case] {run.name} {run.nx}x{run.ny} precision={precision} 36-step run", flush=True)
    s = Solver.from_run(run, precision)
    f0 = s.init(run.rho, run.ux, run.uy, run.T)
    many = s.step(f0, nsteps=36)
    prev = f0
    for _ in range(35):
        prev = s.step(prev)
    last = s.step(prev)
    torch.cuda.synchronize()
    assert torch.equal(many, last)
    rng = np.random.default_rng(36)
    cells = _sample_cells(run.nx, run.ny, rng)
    e = _check_step(run, prev, last, cells, precision)
    c = max(_check_column(run, prev, last, x, precision) for x in FULL_COLUMNS)
    print(f"  step 36: {len(cells)} cells worst relative error {e:.2e}; full columns {c:.2e}")
    s.close()
