"""Parity of the batched ensemble step with the oracle and with single-grid runs."""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W
from helpers import check_patch_step, oracle_after, rel_max, to_np

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def _params(runs, precision):
    from paper_2502_16818_amd import make_params
    return [make_params(r.nx, r.ny, r.dx, r.dy, r.dt, r.tau, r.gamma, r.v, r.eta, r.bc_x, r.bc_y,
                        precision) for r in runs]


# Widths that rule out the 16-byte-chunk form of the batch kernel, and widths
# that are all multiples of four (chunked form in both precisions).
SIZE_SETS = {
    "ragged": [(37, 23), (130, 7), (5, 61), (64, 64), (1, 1), (200, 1)],
    "chunked": [(36, 23), (132, 7), (8, 61), (64, 64), (4, 1), (200, 1)],
}


def _mixed_set(sizes="ragged"):
    """Grids of uneven size with their own gamma, tau, dt and boundary conditions."""
    rng = np.random.default_rng(21)
    runs = []
    for k, (nx, ny) in enumerate(SIZE_SETS[sizes]):
        r = W.random_periodic(nx, ny, seed=30 + k, dt=float(rng.uniform(2e-5, 1e-4)),
                              tau=float(10 ** rng.uniform(-4.3, -3.5)),
                              gamma=float(rng.uniform(1.1, 1.67)))
        r.bc_x = int(rng.integers(0, 2))
        r.bc_y = int(rng.integers(0, 2))
        runs.append(r)
    return runs


@pytest.mark.parametrize("sizes", sorted(SIZE_SETS))
def test_batch_fp64_matches_oracle_per_grid(sizes):
    from paper_2502_16818_amd import Batch
    runs = _mixed_set(sizes)
    b = Batch(_params(runs, FP64))
    f = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    nsteps = 5
    out = b.step(f, nsteps=nsteps)
    for k, r in enumerate(runs):
        print(f"[grid {k}] {r.nx}x{r.ny} bc=({r.bc_x},{r.bc_y}) gamma={r.gamma:.3f}", flush=True)
        _, ref = oracle_after(r, nsteps)
        assert rel_max(to_np(b.view(out, k)), ref.numpy()) < 1e-12


@pytest.mark.parametrize("sizes", sorted(SIZE_SETS))
@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_batch_is_bitwise_equal_to_single_grid_runs(precision, sizes):
    from paper_2502_16818_amd import Batch, Solver
    runs = _mixed_set(sizes)
    b = Batch(_params(runs, precision))
    f = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    nsteps = 40          # long enough to replay the captured graph
    out = b.step(f, nsteps=nsteps)
    for k, r in enumerate(runs):
        s = Solver.from_run(r, precision)
        g = s.init(r.rho, r.ux, r.uy, r.T)
        assert torch.equal(g, b.view(f, k))
        h = s.step(g, nsteps=nsteps)
        assert torch.equal(h, b.view(out, k)), k
        s.close()


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_batch_graph_replays_match_eager_steps(precision):
    """cdbm_batch_step replays a captured graph of 32 steps on long runs;
    every replay must equal the same steps launched one call at a time, also
    after other work on the batch in between."""
    from paper_2502_16818_amd import Batch
    runs = [W.random_periodic(nx, ny, seed=nx) for nx, ny in ((136, 23), (64, 40), (248, 9))]
    b = Batch(_params(runs, precision))
    f0 = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    f = f0.clone()
    for _ in range(64):
        f = b.step(f)
    out = b.empty_f()
    for rep in range(3):
        b.step(f0, out, nsteps=64)
        torch.cuda.synchronize()
        assert torch.equal(out, f), rep
        _ = b.step(f0, nsteps=5)
        torch.cuda.synchronize()
    b.close()


def test_batch_rejects_inconsistent_velocity_sets():
    from paper_2502_16818_amd import Batch, CdbmError
    runs = _mixed_set()[:2]
    ps = _params(runs, FP64)
    ps[1].eta[0] = 2.5
    with pytest.raises(CdbmError) as e:
        Batch(ps)
    assert e.value.code == -1


def test_batched_ensemble_workload_runs_and_conserves_mass():
    """The 96-grid ensemble (sizes 128..1024) in the mixed form: one step
    against the oracle on sampled cells (see check_patch_step), then 20
    steps, finite, and total mass of each periodic grid conserved to FP32
    rounding."""
    from paper_2502_16818_amd import Batch, Solver
    runs = W.batched_ensemble()
    b = Batch(_params(runs, MIXED))
    f = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    m0 = [b.view(f, k).double().sum().item() for k in range(len(runs))]
    # one step of the whole ensemble, in the launch the benchmark times,
    # against oracle patch steps on sampled cells of every eighth grid
    f1 = b.step(f)
    rng = np.random.default_rng(96)
    for k in range(0, len(runs), 8):
        r = runs[k]
        cells = [(0, 0), (r.nx - 1, r.ny - 1), (119, int(rng.integers(0, r.ny))),
                 (int(rng.integers(0, r.nx)), int(rng.integers(0, r.ny)))]
        check_patch_step(r, b.view(f, k), b.view(f1, k), cells, MIXED)
    out = b.step(f, nsteps=20)
    assert torch.isfinite(out).all()
    for k in range(len(runs)):
        m1 = b.view(out, k).double().sum().item()
        assert abs(m1 - m0[k]) <= 2e-6 * abs(m0[k])


LAYOUTS = {"contiguous_fill0": (0, 0, 0, 0), "contiguous_fill28": (0, 28, 0, 0),
           "rows16": (1, 0, 16, 0), "rows96": (1, 0, 96, 0), "rows384": (1, 0, 384, 0),
           "rows96_tail8": (1, 0, 96, 8), "rows192_tail64": (1, 0, 192, 64),
           "rows384_tail96": (1, 0, 384, 96)}


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
@pytest.mark.parametrize("sizes", sorted(SIZE_SETS))
@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_batch_layouts_are_bitwise_equal(precision, sizes, layout):
    """Every launch layout gives the default layout's result bit for bit,
    over a run long enough to replay the captured graph twice (the row-piece
    form's counters must be back at zero after every launch)."""
    from paper_2502_16818_amd import Batch
    runs = _mixed_set(sizes)
    b = Batch(_params(runs, precision))
    f = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    ref = b.step(f, nsteps=67)
    lay, fill, rows, tail = LAYOUTS[layout]
    b.set_launch(lay, fill, rows, tail)
    assert b.get_launch() == {"layout": lay, "fill_rows": fill, "piece_rows": rows,
                              "tail_rows": tail}
    for rep in range(2):
        out = b.step(f, nsteps=67)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
    b.close()


def test_batch_rejects_bad_layouts():
    from paper_2502_16818_amd import Batch, CdbmError
    b = Batch(_params(_mixed_set()[:2], FP64))
    for bad in ((2, 14, 0), (0, -1, 0), (0, 2000, 0), (1, 0, 8), (1, 0, 100000), (1, 0, 96, 4),
                (0, 14, 0, 16)):
        with pytest.raises(CdbmError) as e:
            b.set_launch(*bad)
        assert e.value.code == -1
    assert b.get_launch()["layout"] == 0
    b.close()


def test_autotuned_ensemble_is_no_slower_than_the_default(tmp_path):
    """The tuner on the 96-grid ensemble (mixed): its choice is the fastest of
    its timed candidates, among them the default contiguous split, so it must
    not run slower than the default (5 % timing noise allowed); its result
    stays bitwise that of the default; a second tuner call finds the JSON
    cache entry and applies it without timing."""
    import json
    from paper_2502_16818_amd import Batch
    runs = W.batched_ensemble()
    b = Batch(_params(runs, MIXED))
    f = b.init([(r.rho, r.ux, r.uy, r.T) for r in runs])
    ref = b.step(f, nsteps=5)

    def ms_per_step(n=40):
        out = b.empty_f()
        b.step(f, out, nsteps=8)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(f, out, nsteps=n)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    t_default = ms_per_step()
    cache = str(tmp_path / "tune.json")
    chosen = b.autotune(f, b.empty_f(), cache)
    t_tuned = ms_per_step()
    print(f"  default {t_default:.4f} ms/step, tuned {chosen} {t_tuned:.4f} ms/step")
    assert t_tuned <= 1.05 * t_default
    assert torch.equal(b.step(f, nsteps=5), ref)
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.split("|")[1] == "mixed"
    assert {k: val[k] for k in ("layout", "fill_rows", "piece_rows", "tail_rows")} == chosen
    # a new batch of the same key takes the cached layout
    b2 = Batch(_params(runs, MIXED))
    assert b2.autotune(f, b2.empty_f(), cache) == chosen
    assert b2.get_launch() == chosen
    b.close()
    b2.close()
    # an entry written without tail_rows (the earlier cache format) reads as
    # tail_rows 0
    with open(cache, "w") as fh:
        fh.write("{\n" + json.dumps(key) + ': {"layout": 1, "fill_rows": 0, "piece_rows": 192, '
                 '"ms_per_step": 1.6}\n}\n')
    b3 = Batch(_params(runs, MIXED))
    want = {"layout": 1, "fill_rows": 0, "piece_rows": 192, "tail_rows": 0}
    assert b3.autotune(f, b3.empty_f(), cache) == want
    assert b3.get_launch() == want
    b3.close()
