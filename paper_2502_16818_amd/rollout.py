"""Differentiable rollout of the CDBM over the hand-written adjoint.

``CDBMRollout.apply(rho0, ux0, uy0, T0, tau, solver, nsteps, every)`` runs
f0 = f^eq(rho0, u0, T0), advances nsteps steps and returns the final
(rho, u_x, u_y, T).  Its backward pass uses only the library's reverse-mode
entry points: the moments adjoint seeds dL/df at the final step, every step
is transposed with cdbm_step_adjoint (its dL/dtau terms stay in the handle's
per-block accumulator until one cdbm_tau_collect at the end), and the
initial-equilibrium adjoint maps dL/df0 to the initial fields.  Forward
states are checkpointed every `every` steps; the backward pass recomputes
the states of one segment at a time from its checkpoint, and, while a
segment's first Runge-Kutta stages fit in KEEP_STAGE_BYTES, keeps them
(cdbm_step_keep_stage) so that the step adjoints need not recompute them
(cdbm_step_adjoint_stage; the gradients are the same bit for bit).  With
kept stages, two buffer sets let the next segment's recompute run on a
second stream while the current segment's step adjoints run (the two kinds
of launch are short on small grids and leave the GPU idle on their own).
"""
from __future__ import annotations

import time
from typing import Optional

import torch

from .cdbm import MIXED, Solver

# Kept stages are used while one segment's first stages (one f per step)
# take at most this much device memory; the backward pass then holds the
# states and stages of two segments, four times that at most.
KEEP_STAGE_BYTES = 8 << 30


def _segments(nsteps: int, every: int):
    out = []
    k = 0
    while k < nsteps:
        n = min(every, nsteps - k)
        out.append((k, n))
        k += n
    return out


class CDBMRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, ux0, uy0, T0, tau, solver: Solver, nsteps: int, every: int):
        if abs(float(tau) - solver.params.tau) > 1e-15 * abs(solver.params.tau):
            raise ValueError("tau must equal the relaxation time the solver was created with")
        fields = [t.detach().to(torch.float64).contiguous() for t in (rho0, ux0, uy0, T0)]
        f = solver.init(*fields)
        buf = solver.empty_f()
        ckpts = []
        for _, n in _segments(nsteps, every):
            ckpts.append(f.clone())
            solver.step(f, buf, nsteps=n)
            f, buf = buf, f
        out = solver.moments(f)
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.every = every
        ctx.ckpts = ckpts
        ctx.f_final = f
        ctx.save_for_backward(*fields)
        ctx.tau_like = torch.as_tensor(tau)
        return out

    @staticmethod
    def backward(ctx, g_rho, g_ux, g_uy, g_T):
        s: Solver = ctx.solver
        grads = []
        for g in (g_rho, g_ux, g_uy, g_T):
            grads.append(torch.zeros((s.ny, s.nx), dtype=torch.float64, device="cuda")
                         if g is None else g.to(torch.float64).contiguous())
        lam = s.moments_adjoint(ctx.f_final, *grads)
        lam_next = s.empty_lam()
        dtau = torch.zeros(1, dtype=torch.float64, device="cuda")
        # drop any terms an interrupted reverse pass left in the accumulator
        s.tau_collect(torch.zeros(1, dtype=torch.float64, device="cuda"))
        segs = list(zip(reversed(_segments(ctx.nsteps, ctx.every)), reversed(ctx.ckpts)))
        nmax = min(ctx.every, ctx.nsteps)
        fbytes = ctx.f_final.numel() * ctx.f_final.element_size()
        if nmax * fbytes <= KEEP_STAGE_BYTES:
            lam = _reverse_kept(s, segs, nmax, lam, lam_next)
        else:
            states = [s.empty_f() for _ in range(nmax)]
            for (_, n), ck in segs:
                states[0].copy_(ck)
                for j in range(1, n):
                    s.step(states[j - 1], states[j], nsteps=1)
                for j in reversed(range(n)):
                    s.step_adjoint(states[j], lam, lam_next, defer_tau=True)
                    lam, lam_next = lam_next, lam
        s.tau_collect(dtau)
        rho0, ux0, uy0, T0 = ctx.saved_tensors
        g0 = s.init_adjoint(rho0, ux0, uy0, T0, lam)
        gtau = dtau.reshape(()).to(ctx.tau_like.dtype).to(ctx.tau_like.device) \
            if ctx.needs_input_grad[4] else None
        return (*g0, gtau, None, None, None)


def _reverse_kept(s: Solver, segs, nmax: int, lam, lam_next):
    """Step adjoints of every segment (last first) with kept stages; returns
    dL/df0.  A segment's states and first stages are recomputed on a side
    stream into one of two buffer sets while the current stream transposes
    the segment before it; events order each set's reuse.  The kernels and
    their inputs are those of a one-stream pass, so the results are too."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(main)   # checkpoints and buffers were written on main
    sets = [([s.empty_f() for _ in range(nmax)], [s.empty_f() for _ in range(nmax)],
             s.empty_f()) for _ in range(2)]
    ready = [torch.cuda.Event(), torch.cuda.Event()]
    free = [None, None]

    def recompute(k):
        (_, n), ck = segs[k]
        states, stages, spare = sets[k % 2]
        with torch.cuda.stream(side):
            if free[k % 2] is not None:
                side.wait_event(free[k % 2])
            states[0].copy_(ck)
            for j in range(n):
                s.step_keep_stage(states[j], stages[j], states[j + 1] if j + 1 < n else spare)
            ready[k % 2].record(side)

    recompute(0)
    for k in range(len(segs)):
        if k + 1 < len(segs):
            recompute(k + 1)
        (_, n), _ = segs[k]
        states, stages, _ = sets[k % 2]
        main.wait_event(ready[k % 2])
        for j in reversed(range(n)):
            s.step_adjoint(states[j], lam, lam_next, f1=stages[j], defer_tau=True)
            lam, lam_next = lam_next, lam
        done = torch.cuda.Event()
        done.record(main)
        free[k % 2] = done
    return lam


def rollout(solver: Solver, rho0, ux0, uy0, T0, tau, nsteps: int, every: int = 100):
    return CDBMRollout.apply(rho0, ux0, uy0, T0, tau, solver, nsteps, every)


def adjoint_forward_ratio(n: int = 256, steps: int = 2000, every: int = 100,
                          precision: int = MIXED, seed: int = 0, keep_grads: bool = False) -> dict:
    """Wall-time ratio of the backward to the forward pass of the gradient
    workload: n x n periodic grid, smooth random fields, L2 mismatch of the
    final density against a target run from perturbed fields with 1.1 tau.
    With keep_grads, the result also holds the gradients ("grads": the four
    field gradients and dL/dtau, on the device)."""
    import workloads as W

    base, tgt = W.adjoint_problem(n=n, seed=seed, steps=steps)
    s_t = Solver.from_run(tgt, precision)
    ft = s_t.init(tgt.rho, tgt.ux, tgt.uy, tgt.T)
    ft = s_t.step(ft, nsteps=steps)
    rho_t = s_t.moments(ft)[0].clone()
    s_t.close()
    del ft

    s = Solver.from_run(base, precision)
    dev = torch.device("cuda")
    fields = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True)
              for a in (base.rho, base.ux, base.uy, base.T)]
    tau = torch.tensor(base.tau, dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho, ux, uy, T = rollout(s, *fields, tau, steps, every)
    loss = ((rho - rho_t) ** 2).mean()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {
        "workload": f"{n}x{n} periodic, {steps} steps, checkpoint every {every}",
        "precision": "mixed" if precision == MIXED else "fp64",
        "forward_ms_per_step": (t1 - t0) * 1e3 / steps,
        "backward_ms_per_step": (t2 - t1) * 1e3 / steps,
        "ratio": (t2 - t1) / (t1 - t0),
        "loss": float(loss.detach()),
        "grad_tau": float(tau.grad),
        "grad_norms": [float(f.grad.norm()) for f in fields],
    }
    if keep_grads:
        out["grads"] = [f.grad.detach().clone() for f in fields] + [tau.grad.detach().clone()]
    s.close()
    return out
