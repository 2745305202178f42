"""FP64 reference implementation of the CDBM (test infrastructure only).

Everything here follows Sec. 2 of the paper step by step, on torch CPU
tensors in float64, with no blocking, fusion or algebraic shortcut beyond
what the equations state.  Distributions are stored as f[i, y, x] with the
16 discrete velocities first (i = 0..15 stands for the paper's i = 1..16).

Readings taken where the text is silent or garbled:
* Eq. (2) prints "(+-1, 0)" for the axis groups; the four axis velocities are
  read as v(1,0), v(0,1), v(-1,0), v(0,-1) (the literal duplicate reading
  makes the moment matrix singular).  Diagonal groups are v(+-1, +-1), i.e.
  components +-v.  Each group is ordered counter-clockwise from +x.
* D = 2 throughout, so gamma = (4 + I) / (2 + I) (the text under Eq. (5)).
* T is defined by the energy moment of Eq. (4):
  sum_i f_i (|v_i - u|^2 + eta_i^2) = rho (D + I) T.
* Eq. (12) is used with the sign that makes it a derivative:
  v dF/dr = [H(r + 1/2) - H(r - 1/2)] / dr.
* The two-stage Runge-Kutta step is Heun's (SSP) form,
  f1 = f + dt L(f),  f^{n+1} = f/2 + (f1 + dt L(f1)) / 2,
  with the equilibrium re-evaluated at each stage.  Parity unpinned for this
  choice: the paper does not say which two-stage form it uses; what every
  second-order two-stage form shares (the amplification 1 - z + z^2/2 of a
  uniform relaxation) is pinned, Heun against the midpoint form is not.
* Two ghost layers per side are refreshed before every stage: periodic wrap
  or a zero-gradient copy of the edge cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import torch

D = 2
DT = torch.float64

PERIODIC = 0
ZERO_GRADIENT = 1

_AXIS = ((1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0))
_DIAG = ((1.0, 1.0), (-1.0, 1.0), (-1.0, -1.0), (1.0, -1.0))


def extra_dof_from_gamma(gamma: float) -> float:
    """Invert gamma = (D + I + 2) / (D + I) (text under Eq. (5)) for I."""
    return 2.0 / (gamma - 1.0) - D


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    tau: float
    I: float
    v: Tuple[float, float, float, float]
    eta: Tuple[float, float, float, float]
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC

    @staticmethod
    def from_run(run) -> "Params":
        return Params(run.nx, run.ny, run.dx, run.dy, run.dt, run.tau,
                      extra_dof_from_gamma(run.gamma), tuple(run.v), tuple(run.eta),
                      run.bc_x, run.bc_y)


def discrete_velocities(v4, eta4) -> Tuple[torch.Tensor, torch.Tensor]:
    """Eqs. (2)-(3): the 16 velocities (16, 2) and their eta_i (16,)."""
    vel, eta = [], []
    for g, dirs in enumerate((_AXIS, _DIAG, _AXIS, _DIAG)):
        for d in dirs:
            vel.append((v4[g] * d[0], v4[g] * d[1]))
            eta.append(eta4[g])
    return torch.tensor(vel, dtype=DT), torch.tensor(eta, dtype=DT)


def moment_rows(cx: torch.Tensor, cy: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
    """The 16 moment functions Psi_r of Eq. (4), as listed under Eq. (6).

    cx, cy are (peculiar) velocity components and eta the extra-DoF
    variable, all broadcastable; returns a tensor with a new leading axis of
    length 16 (row r = 1..16 of M at index r - 1).
    """
    e = cx * cx + cy * cy + eta * eta
    one = torch.ones_like(e)
    return torch.stack([
        one,                # 1
        cx, cy,             # v*
        e,                  # v*.v* + eta^2
        cx * cx, cx * cy, cy * cy,          # v* v*
        e * cx, e * cy,                     # (v*.v* + eta^2) v*
        cx * cx * cx, cx * cx * cy, cx * cy * cy, cy * cy * cy,   # v* v* v*
        e * cx * cx, e * cx * cy, e * cy * cy,                    # (v*.v* + eta^2) v* v*
    ])


def moment_matrix(ux: torch.Tensor, uy: torch.Tensor, vel: torch.Tensor,
                  eta: torch.Tensor) -> torch.Tensor:
    """M(u) of Eq. (6): M[..., r, i] = Psi_r(v_i - u, eta_i).  ux, uy: (N,)."""
    cx = vel[:, 0][None, :] - ux[:, None]
    cy = vel[:, 1][None, :] - uy[:, None]
    rows = moment_rows(cx, cy, eta[None, :].expand_as(cx))   # (16, N, 16)
    return rows.permute(1, 0, 2)


def central_equilibrium_moments(rho: torch.Tensor, T: torch.Tensor, I: float) -> torch.Tensor:
    """Left-hand side of Eq. (4): moments of the Maxwellian Eq. (5) about u.

    With c = v - u Gaussian of variance T per translational component and eta
    Gaussian of variance I T (Eq. (5)): odd moments vanish, E[c_a c_b] = T d_ab,
    E[c_x^4] = 3 T^2, E[c_x^2 c_y^2] = T^2, E[eta^2] = I T.  Hence
    E[|c|^2 + eta^2] = (D + I) T and E[(|c|^2 + eta^2) c_a c_b] = (D + 2 + I) T^2 d_ab.
    Returns (N, 16) in the row order of Eq. (6).
    """
    a = D + I
    z = torch.zeros_like(rho)
    return torch.stack([
        rho, z, z, rho * a * T,
        rho * T, z, rho * T,
        z, z,
        z, z, z, z,
        rho * (a + 2.0) * T * T, z, rho * (a + 2.0) * T * T,
    ], dim=-1)


def equilibrium(rho, ux, uy, T, I, vel, eta) -> torch.Tensor:
    """Eq. (7): f^eq = M(u)^{-1} fbar^eq, one 16x16 solve per cell.

    rho, ux, uy, T: (N,) -> (N, 16).
    """
    M = moment_matrix(ux, uy, vel, eta)
    fbar = central_equilibrium_moments(rho, T, I)
    return torch.linalg.solve(M, fbar.unsqueeze(-1)).squeeze(-1)


def macroscopic(f: torch.Tensor, vel, eta, I):
    """Density, flow velocity and temperature from the first three moments of
    Eq. (4) with f_i in place of f_i^eq (the statement after Eq. (7)).

    f: (16, ...) -> rho, ux, uy, T each of shape f.shape[1:].
    """
    shape = (16,) + (1,) * (f.dim() - 1)
    vx = vel[:, 0].reshape(shape)
    vy = vel[:, 1].reshape(shape)
    et = eta.reshape(shape)
    rho = f.sum(0)
    ux = (f * vx).sum(0) / rho
    uy = (f * vy).sum(0) / rho
    cx = vx - ux.unsqueeze(0)
    cy = vy - uy.unsqueeze(0)
    T = (f * (cx * cx + cy * cy + et * et)).sum(0) / ((D + I) * rho)
    return rho, ux, uy, T


def equilibrium_of(f: torch.Tensor, p: Params, vel, eta) -> torch.Tensor:
    """f^eq of the macroscopic state carried by f.  f: (16, ny, nx)."""
    rho, ux, uy, T = macroscopic(f, vel, eta, p.I)
    feq = equilibrium(rho.reshape(-1), ux.reshape(-1), uy.reshape(-1), T.reshape(-1),
                      p.I, vel, eta)
    return feq.t().reshape(f.shape)


def initial_distribution(rho, ux, uy, T, p: Params) -> torch.Tensor:
    """f = f^eq(rho, u, T) per cell; fields (ny, nx) -> (16, ny, nx)."""
    vel, eta = discrete_velocities(p.v, p.eta)
    rho, ux, uy, T = (torch.as_tensor(a, dtype=DT) for a in (rho, ux, uy, T))
    feq = equilibrium(rho.reshape(-1), ux.reshape(-1), uy.reshape(-1), T.reshape(-1),
                      p.I, vel, eta)
    return feq.t().reshape((16,) + tuple(rho.shape))


def nonequilibrium(f: torch.Tensor, p: Params) -> torch.Tensor:
    """Eqs. (8)-(11): sum_i (f_i - f_i^eq) Psi_r(v_i - u) for rows r = 5..16.

    Returns (12, ny, nx) ordered Delta*_2 (xx, xy, yy), Delta*_{3,1} (x, y),
    Delta*_3 (xxx, xxy, xyy, yyy), Delta*_{4,2} (xx, xy, yy).
    """
    vel, eta = discrete_velocities(p.v, p.eta)
    rho, ux, uy, T = macroscopic(f, vel, eta, p.I)
    n = rho.numel()
    feq = equilibrium(rho.reshape(-1), ux.reshape(-1), uy.reshape(-1), T.reshape(-1),
                      p.I, vel, eta)                       # (N, 16)
    M = moment_matrix(ux.reshape(-1), uy.reshape(-1), vel, eta)   # (N, 16, 16)
    dev = f.reshape(16, n).t() - feq
    out = torch.einsum("nri,ni->nr", M, dev)
    return out[:, 4:].t().reshape((12,) + tuple(rho.shape))


def minmod(X: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
    """Eq. (16): 0 if Y = 0 or XY <= 0; X if |X / Y| <= 1; otherwise Y.

    |X / Y| <= 1 is tested as |X| <= |Y| (Y is nonzero on that branch).
    """
    zero = torch.zeros_like(X)
    pick = torch.where(X.abs() <= Y.abs(), X, Y)
    return torch.where((Y == 0) | (X * Y <= 0), zero, pick)


def nnd_derivative(fpad: torch.Tensor, vr: torch.Tensor, dr: float, axis: int) -> torch.Tensor:
    """NND approximation of v_ir dF_i/dr, Eqs. (12)-(20).

    fpad: distributions with two ghost layers on both sides along `axis`
    (velocity index on axis 0); vr: (16,) velocity components along r.
    Returns the derivative at the interior cells.
    """
    n = fpad.shape[axis] - 4
    shape = [1] * fpad.dim()
    shape[0] = 16
    vr = vr.reshape(shape)
    fp = 0.5 * (vr + vr.abs()) * fpad            # Eq. (19)
    fm = 0.5 * (vr - vr.abs()) * fpad            # Eq. (20)

    def s(t, start, length):
        return t.narrow(axis, start, length)

    dfp = s(fp, 1, n + 3) - s(fp, 0, n + 3)      # Eq. (17): dfp[j] = Delta f+(j + 1/2)
    dfm = s(fm, 1, n + 3) - s(fm, 0, n + 3)      # Eq. (18)
    # faces j + 1/2 for padded j = 1 .. n + 1
    HL = s(fp, 1, n + 1) + 0.5 * minmod(s(dfp, 1, n + 1), s(dfp, 0, n + 1))   # Eq. (14)
    HR = s(fm, 2, n + 1) - 0.5 * minmod(s(dfm, 1, n + 1), s(dfm, 2, n + 1))   # Eq. (15)
    H = HL + HR                                                               # Eq. (13)
    return (s(H, 1, n) - s(H, 0, n)) / dr                                     # Eq. (12)


def ghost_index(n: int, bc: int) -> torch.Tensor:
    """Source cell of each of the n + 4 padded positions (two ghosts per side)."""
    j = torch.arange(-2, n + 2)
    if bc == PERIODIC:
        return torch.remainder(j, n)
    return j.clamp(0, n - 1)


def advection(f: torch.Tensor, p: Params, vel) -> torch.Tensor:
    """-v_i . grad f_i for every velocity, with the NND derivative per axis."""
    ix = ghost_index(p.nx, p.bc_x)
    iy = ghost_index(p.ny, p.bc_y)
    fx = f.index_select(2, ix)
    fy = f.index_select(1, iy)
    return -(nnd_derivative(fx, vel[:, 0], p.dx, 2) + nnd_derivative(fy, vel[:, 1], p.dy, 1))


def rhs(f: torch.Tensor, p: Params, tau=None) -> torch.Tensor:
    """Right-hand side of Eq. (1): -v_i . grad f_i - (f_i - f_i^eq) / tau."""
    vel, eta = discrete_velocities(p.v, p.eta)
    tau = p.tau if tau is None else tau
    return advection(f, p, vel) - (f - equilibrium_of(f, p, vel, eta)) / tau


def step(f: torch.Tensor, p: Params, tau=None) -> torch.Tensor:
    """One time step of the two-stage Runge-Kutta scheme (Heun form)."""
    f1 = f + p.dt * rhs(f, p, tau)
    return 0.5 * f + 0.5 * (f1 + p.dt * rhs(f1, p, tau))


def run(f: torch.Tensor, p: Params, nsteps: int, tau=None) -> torch.Tensor:
    for _ in range(nsteps):
        f = step(f, p, tau)
    return f


def run_from_fields(run_cfg, nsteps: int | None = None) -> torch.Tensor:
    """Initialise f = f^eq from a workloads.Run and advance it."""
    p = Params.from_run(run_cfg)
    f = initial_distribution(run_cfg.rho, run_cfg.ux, run_cfg.uy, run_cfg.T, p)
    return run(f, p, run_cfg.steps if nsteps is None else nsteps)


def fields(f: torch.Tensor, p: Params):
    vel, eta = discrete_velocities(p.v, p.eta)
    return macroscopic(f, vel, eta, p.I)


# ---------------------------------------------------------------------------
# Adjoint: reverse-mode derivative of the definition above.
# ---------------------------------------------------------------------------

def step_vjp(f: torch.Tensor, lam: torch.Tensor, p: Params):
    """(dF/df)^T lam and (dF/dtau)^T lam for one step F = step(., p).

    Computed by reverse-mode differentiation of `step`; minmod passes the
    derivative to X when |X| = |Y| (the branch order of Eq. (16)).
    """
    f = f.detach().clone().requires_grad_(True)
    tau = torch.tensor(p.tau, dtype=DT, requires_grad=True)
    out = step(f, p, tau)
    gf, gtau = torch.autograd.grad(out, (f, tau), lam)
    return gf, float(gtau)


def init_vjp(rho, ux, uy, T, lam_f: torch.Tensor, p: Params):
    """Gradient of <lam_f, f^eq(rho, u, T)> with respect to the four fields."""
    ins = [torch.as_tensor(a, dtype=DT).clone().requires_grad_(True) for a in (rho, ux, uy, T)]
    f0 = initial_distribution(*ins, p)
    return torch.autograd.grad(f0, ins, lam_f)


def moments_vjp(f: torch.Tensor, g_rho, g_ux, g_uy, g_T, p: Params) -> torch.Tensor:
    """(d(rho, u, T)/df)^T (g_rho, g_ux, g_uy, g_T)."""
    f = f.detach().clone().requires_grad_(True)
    vel, eta = discrete_velocities(p.v, p.eta)
    outs = macroscopic(f, vel, eta, p.I)
    grads = [torch.as_tensor(g, dtype=DT) for g in (g_rho, g_ux, g_uy, g_T)]
    return torch.autograd.grad(outs, f, grads)[0]


# ---------------------------------------------------------------------------
# Raw-moment DBM (the construction Sec. 2 contrasts the CDBM with): the same
# sixteen moment functions evaluated at the raw velocities v_i instead of the
# peculiar ones v_i - u.
# ---------------------------------------------------------------------------

def raw_equilibrium_moments(rho, ux, uy, T, I: float, order: int = 6) -> torch.Tensor:
    """Raw moments sum over Psi_r(v, eta) of the Maxwellian Eq. (5), by
    Gauss-Hermite quadrature: v = u + sqrt(T) xi per translational component
    and eta = sqrt(I T) zeta with xi, zeta standard normal (exact for the
    polynomial Psi_r, of degree <= 4 in v and 2 in eta, at `order` >= 4
    nodes).  rho, ux, uy, T: (N,) -> (N, 16) in the row order of Eq. (6)."""
    import numpy as np
    x, w = np.polynomial.hermite_e.hermegauss(order)
    w = w / w.sum()
    xi = torch.as_tensor(x, dtype=DT)
    wt = torch.as_tensor(w, dtype=DT)
    rho, ux, uy, T = (torch.as_tensor(a, dtype=DT).reshape(-1) for a in (rho, ux, uy, T))
    s = torch.sqrt(T)[:, None, None, None]
    se = torch.sqrt(I * T)[:, None, None, None]
    vx = ux[:, None, None, None] + s * xi[None, :, None, None]
    vy = uy[:, None, None, None] + s * xi[None, None, :, None]
    et = se * xi[None, None, None, :]
    vx, vy, et = torch.broadcast_tensors(vx, vy, et)
    W3 = (wt[:, None, None] * wt[None, :, None] * wt[None, None, :])[None]
    rows = moment_rows(vx, vy, et)                     # (16, N, q, q, q)
    return rho[:, None] * (rows * W3[None]).sum(dim=(2, 3, 4)).t()


def raw_equilibrium(rho, ux, uy, T, I, vel, eta) -> torch.Tensor:
    """f^eq of the raw-moment construction: M0 f^eq = m^eq, with M0 the
    matrix of Eq. (6) at u = 0 and m^eq the raw Maxwellian moments; one
    16 x 16 solve per cell.  -> (N, 16)."""
    m = raw_equilibrium_moments(rho, ux, uy, T, I)
    n = m.shape[0]
    zero = torch.zeros(n, dtype=DT)
    M0 = moment_matrix(zero, zero, vel, eta)
    return torch.linalg.solve(M0, m.unsqueeze(-1)).squeeze(-1)


def raw_nonequilibrium(f: torch.Tensor, p: Params) -> torch.Tensor:
    """Nonequilibrium measures of the raw-moment construction:
    sum_i (f_i - f_i^eq) Psi_r(v_i) for rows r = 5..16 (the raw velocity in
    place of the peculiar one of Eqs. (8)-(11)), with f^eq from
    raw_equilibrium.  Returns (12, ny, nx) in the slot order of
    nonequilibrium()."""
    vel, eta = discrete_velocities(p.v, p.eta)
    rho, ux, uy, T = macroscopic(f, vel, eta, p.I)
    n = rho.numel()
    feq = raw_equilibrium(rho.reshape(-1), ux.reshape(-1), uy.reshape(-1), T.reshape(-1),
                          p.I, vel, eta)
    zero = torch.zeros(n, dtype=DT)
    M0 = moment_matrix(zero, zero, vel, eta)
    dev = f.reshape(16, n).t() - feq
    out = torch.einsum("nri,ni->nr", M0, dev)
    return out[:, 4:].t().reshape((12,) + tuple(rho.shape))
