"""Shared helpers of the test-suite: oracle runs and comparisons (CPU side)."""
import numpy as np
import torch

from oracle import cdbm as C


def oracle_f0(run):
    p = C.Params.from_run(run)
    return p, C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)


def oracle_after(run, nsteps):
    p, f = oracle_f0(run)
    return p, C.run(f, p, nsteps)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.sqrt(np.mean(b * b))), floor)
    return float(np.sqrt(np.mean((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.mean((a - b) ** 2)))


def field_errors(got_fields, want_fields, u_scale):
    """Relative L2 errors of (rho, u_x, u_y, T); velocities are normalised by u_scale."""
    names = ("rho", "ux", "uy", "T")
    out = {}
    for n, g, w in zip(names, got_fields, want_fields):
        g = np.asarray(g, dtype=np.float64)
        w = np.asarray(w, dtype=np.float64)
        if n in ("ux", "uy"):
            out[n] = float(np.sqrt(np.mean((g - w) ** 2)) / u_scale)
        else:
            out[n] = rel_l2(g, w)
    return out


def to_np(t):
    if isinstance(t, torch.Tensor):
        return t.detach().cpu().double().numpy()
    return np.asarray(t)


# Oracle steps on patches (the full-size parity tests).  f^{n+1} at a cell
# depends on f^n only within 4 cells along x or along y (two Runge-Kutta
# stages of the 2-cell NND stencil), so the oracle's step on the 9 x 9 patch
# around the cell, cut from the GPU's own f^n, gives the cell's exact f^{n+1}
# whatever boundary the patch itself gets.  At a zero-gradient x side the
# patch is clipped to the domain and gets that boundary.
PATCH_HALO = 4
# max |difference| / max |f| of the patch, by precision form (0 FP64, 1 mixed).
# Mixed: f^{n+1} and f^(1) are rounded to FP32 (half an ulp each, 6e-8 of
# |f|) and the advection runs in FP32 on increments much smaller than f.
FP64_MIXED_PATCH_TOL = {0: 1e-12, 1: 3e-7}


def patch_indices(run, x, y):
    """Columns and rows of the 9 x 9 patch around (x, y), the centre's
    position in it and the patch's x boundary (y must be periodic)."""
    nx, ny = run.nx, run.ny
    h = PATCH_HALO
    w = 2 * h + 1
    if run.bc_x == C.ZERO_GRADIENT and x < h:
        cols, cx, bcx = np.arange(0, w), x, C.ZERO_GRADIENT
    elif run.bc_x == C.ZERO_GRADIENT and x >= nx - h:
        cols, cx, bcx = np.arange(nx - w, nx), x - (nx - w), C.ZERO_GRADIENT
    else:
        cols, cx, bcx = np.arange(x - h, x + h + 1) % nx, h, C.PERIODIC
    assert run.bc_y == C.PERIODIC
    rows = np.arange(y - h, y + h + 1) % ny
    return cols, rows, cx, h, bcx


def check_patch_step(run, f_prev, f_next, cells, precision, tol=None):
    """Compare f_next at each (x, y) of `cells` with the oracle's step of the
    patch of f_prev around it; returns the worst relative error."""
    tol = FP64_MIXED_PATCH_TOL[precision] if tol is None else tol
    p0 = C.Params.from_run(run)
    worst = 0.0
    for x, y in cells:
        cols, rows, cx, cy, bcx = patch_indices(run, x, y)
        ci = torch.as_tensor(cols, device=f_prev.device)
        ri = torch.as_tensor(rows, device=f_prev.device)
        fp = f_prev.index_select(1, ri).index_select(2, ci).double().cpu()
        p = C.Params(len(cols), len(rows), p0.dx, p0.dy, p0.dt, p0.tau, p0.I, p0.v, p0.eta,
                     bcx, C.PERIODIC)
        want = C.step(fp, p)[:, cy, cx]
        got = f_next[:, y, x].double().cpu()
        err = float((got - want).abs().max() / fp.abs().max())
        worst = max(worst, err)
        assert err <= tol, (x, y, err)
    return worst


def check_column_step(run, f_prev, f_next, x, precision, tol=None):
    """Compare the whole column x of f_next (every row) with the oracle's step
    of the 9-column, full-height strip of f_prev around it (periodic in y, so
    the strip's only boundary is 4 columns away); returns the worst relative
    error, max |difference| / max |f| of the strip.  Every row seam of any
    assignment of rows to blocks lies on the column."""
    tol = FP64_MIXED_PATCH_TOL[precision] if tol is None else tol
    p0 = C.Params.from_run(run)
    cols, _, cx, _, bcx = patch_indices(run, x, 0)
    ci = torch.as_tensor(cols, device=f_prev.device)
    fp = f_prev.index_select(2, ci).double().cpu()
    p = C.Params(len(cols), run.ny, p0.dx, p0.dy, p0.dt, p0.tau, p0.I, p0.v, p0.eta,
                 bcx, C.PERIODIC)
    want = C.step(fp, p)[:, :, cx]
    got = f_next[:, :, x].double().cpu()
    diff = (got - want).abs().amax(dim=0)
    err = float(diff.max() / fp.abs().max())
    assert err <= tol, (x, int(diff.argmax()), err)
    return err
