"""cdbm_conserved_totals_static (no allocation, static scratch) against
cdbm_conserved_totals on the same buffers, through the C ABI: two calls in a
row on one GPU, the second on a smaller grid, in both precision forms."""
import ctypes

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def _totals_both(run, precision):
    from paper_2502_16818_amd import Solver, cdbm
    print(f"[case] {run.name} {run.nx}x{run.ny} precision={precision}", flush=True)
    s = Solver.from_run(run, precision)
    f = s.init(run.rho, run.ux, run.uy, run.T)
    f = s.step(f, nsteps=3)
    ref = s.totals(f)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    rc = cdbm.load().cdbm_conserved_totals_static(ctypes.byref(s.params), f.data_ptr(),
                                                  out.data_ptr(),
                                                  torch.cuda.current_stream().cuda_stream)
    assert rc == 0, cdbm.load().cdbm_last_error()
    torch.cuda.synchronize()
    s.close()
    return out, ref


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_static_totals_equal_handle_totals_on_two_calls(precision):
    big = W.random_periodic(300, 211, seed=21, dt=1e-4, tau=2e-4)
    small = W.random_periodic(37, 5, seed=22, dt=1e-4, tau=2e-4)
    for run in (big, small):
        got, want = _totals_both(run, precision)
        print(f"  static {got.tolist()} handle {want.tolist()}")
        assert torch.equal(got, want)


def test_static_totals_reject_bad_parameters():
    from paper_2502_16818_amd import cdbm, make_params
    p = make_params(0, 4, 0.1, 0.1, 1e-4, 1e-4, 1.4, (1.4, 1.1, 1.1, 1.0), (3.0, 0.0, 0.0, 0.0))
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    f = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = cdbm.load().cdbm_conserved_totals_static(ctypes.byref(p), f.data_ptr(), out.data_ptr(),
                                                  None)
    assert rc == -1 and b"out of range" in cdbm.load().cdbm_last_error()
