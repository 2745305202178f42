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
