"""Seeded synthetic workloads for the CDBM hot path.

This module only *describes* runs: grid shapes, spacings, time steps,
relaxation times, the adjustable discrete-velocity parameters of Eqs. (2)-(3),
boundary conditions and the initial macroscopic fields (rho, u_x, u_y, T).
It holds none of the method's arithmetic (no moments, no equilibrium, no
fluxes), so both the HIP path and the CPU oracle can consume it without
sharing any of the computation that the parity tests compare.

Velocity-set parameters are the ones printed in Sec. 3 for each benchmark:
Sod tube (Sec. 3.1), Lax tube (Sec. 3.2), Ma = 15 shock (Sec. 3.3), sound wave
(Sec. 3.4) and Taylor-Green vortex (Sec. 3.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

PERIODIC = 0
ZERO_GRADIENT = 1

# (v_a, v_b, v_c, v_d), (eta_a, eta_b, eta_c, eta_d) as printed in Sec. 3.
VELOCITY_SETS = {
    "sod": ((2.5, 2.5, 1.2, 1.1), (0.0, 0.0, 0.0, 1.2)),        # Sec. 3.1
    "lax": ((4.4, 4.4, 3.0, 1.8), (0.0, 0.0, 5.0, 0.0)),        # Sec. 3.2
    "shock": ((21.8, 21.8, 17.8, 9.8), (18.8, 0.0, 0.0, 0.0)),  # Sec. 3.3
    "sound": ((1.4, 1.1, 1.1, 1.0), (3.0, 0.0, 0.0, 0.0)),      # Sec. 3.4
    "tg": ((0.2, 0.2, 2.0, 2.0), (0.0, 5.0, 0.0, 2.6)),         # Sec. 3.5
}

# The Sec. 3.4 set expressed for a reference temperature of 2 instead of 1:
# every speed and eta scaled by sqrt(2) (velocities of the model scale with
# sqrt(T)).  Used for the smooth random fields, whose T spans [0.5, 2]: with
# the unscaled set the linearised scheme grows slowly on fine grids
# (dx = 1/256), which dominates gradients over 2000 steps.
VELOCITY_SETS["sound_t2"] = (tuple(math.sqrt(2.0) * v for v in VELOCITY_SETS["sound"][0]),
                             tuple(math.sqrt(2.0) * e for e in VELOCITY_SETS["sound"][1]))


@dataclasses.dataclass
class Run:
    """One run of the method: grid, parameters and initial fields.

    Fields are float64 numpy arrays of shape (ny, nx), x fastest; cell j sits
    at x = (j + 1/2) dx (cell-centred grid).
    """

    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    tau: float
    gamma: float
    v: Tuple[float, float, float, float]
    eta: Tuple[float, float, float, float]
    bc_x: int
    bc_y: int
    steps: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def with_fields(self, rho, ux, uy, T, **kw) -> "Run":
        return dataclasses.replace(self, rho=rho, ux=ux, uy=uy, T=T, **kw)


def cell_centres(n: int, d: float, origin: float = 0.0) -> np.ndarray:
    return origin + (np.arange(n, dtype=np.float64) + 0.5) * d


def _two_state(nx, ny, x, x_split, left, right):
    """Piecewise-constant (rho, u_x, u_y, T) with the left state for x < x_split."""
    mask = np.broadcast_to((x < x_split)[None, :], (ny, nx))
    out = []
    for l, r in zip(left, right):
        out.append(np.where(mask, float(l), float(r)).astype(np.float64))
    return out


def sod_tube(nx: int = 500, dx: float = 2e-3, dt: float = 2e-5, tau: float = 2e-5,
             gamma: float = 1.4, steps: int = 5000, vset: str = "sod") -> Run:
    """Sod-type Riemann tube on an nx x 1 grid, diaphragm at the middle.

    States are the Sec. 3.1 ones, (rho, u_x, u_y, T) = (1, 0, 0, 1) | (0.125, 0, 0, 0.8),
    i.e. p = rho T = 1 | 0.1.  Zero-gradient ends in x; periodic in y (one row).
    """
    x = cell_centres(nx, dx)
    rho, ux, uy, T = _two_state(nx, 1, x, 0.5 * nx * dx, (1.0, 0.0, 0.0, 1.0),
                                (0.125, 0.0, 0.0, 0.8))
    v, eta = VELOCITY_SETS[vset]
    return Run("sod", nx, 1, dx, dx, dt, tau, gamma, v, eta, ZERO_GRADIENT, PERIODIC,
               steps, rho, ux, uy, T)


def lax_tube(nx: int = 1000, dx: float = 2e-3, dt: float = 2e-5, tau: float = 1e-4,
             gamma: float = 1.4, steps: int = 10000) -> Run:
    """The Sec. 3.2 Lax tube: L = (0.445, 0.698, 0, 7.928) on [0,1), R = (0.5, 0, 0, 1.142)."""
    x = cell_centres(nx, dx)
    rho, ux, uy, T = _two_state(nx, 1, x, 1.0, (0.445, 0.698, 0.0, 7.928),
                                (0.5, 0.0, 0.0, 1.142))
    v, eta = VELOCITY_SETS["lax"]
    return Run("lax", nx, 1, dx, dx, dt, tau, gamma, v, eta, ZERO_GRADIENT, PERIODIC,
               steps, rho, ux, uy, T)


def paper_sod_tube(t_end: float = 0.02) -> Run:
    """The Sec. 3.1 Sod tube at the paper's shape: 1500 x 1 cells of 1e-4 on
    [0, 0.15], diaphragm at 0.075, dt = 2e-5, tau = 1e-4, gamma = 2 (I = 0),
    Sec. 3.1 velocity set, zero-gradient ends.  The end time is not stated;
    t_end = 0.02 keeps every wave inside the tube."""
    nx, dx, dt = 1500, 1e-4, 2e-5
    x = cell_centres(nx, dx)
    rho, ux, uy, T = _two_state(nx, 1, x, 0.075, (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.8))
    v, eta = VELOCITY_SETS["sod"]
    return Run("paper_sod", nx, 1, dx, dx, dt, 1e-4, 2.0, v, eta, ZERO_GRADIENT, PERIODIC,
               int(round(t_end / dt)), rho, ux, uy, T)


def paper_shock_tube(t_end: float = 0.04, tau: float = 2e-6) -> Run:
    """The Sec. 3.3 Ma = 15 shock at the paper's shape: 10000 x 1 cells of
    2e-4 on [0, 2], post-shock state for x <= 0.02, dt = 2e-6, gamma = 1.4,
    Sec. 3.3 velocity set, zero-gradient ends.  tau and the end time are not
    stated; tau = dt and t_end = 0.04 (the shock moves about 0.71)."""
    nx, dx, dt = 10000, 2e-4, 2e-6
    x = cell_centres(nx, dx)
    rho, ux, uy, T = _two_state(nx, 1, x, 0.02, (5.8696, 14.7245, 0.0, 44.6938),
                                (1.0, 0.0, 0.0, 1.0))
    v, eta = VELOCITY_SETS["shock"]
    return Run("paper_shock", nx, 1, dx, dx, dt, tau, 1.4, v, eta, ZERO_GRADIENT, PERIODIC,
               int(round(t_end / dt)), rho, ux, uy, T)


def taylor_green_paper(n: int = 100, t_end: float = 0.1, dt: float = 2e-5) -> Run:
    """The Sec. 3.5 Taylor-Green vortex on [0, 2L]^2 at t = 0 (Eqs. (22)-(24)).

    u0 = 0.01, p0 = 1, L = 0.05, rho0 = 1 (so T = p), gamma = 1.4, tau = 5e-4.
    """
    u0, p0, L = 0.01, 1.0, 0.05
    d = 2 * L / n
    x = cell_centres(n, d)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ux = -u0 * np.cos(np.pi * X / L) * np.sin(np.pi * Y / L)
    uy = u0 * np.sin(np.pi * X / L) * np.cos(np.pi * Y / L)
    p = p0 - p0 * u0 ** 2 / 4 * (np.cos(2 * np.pi * X / L) + np.cos(2 * np.pi * Y / L))
    rho = np.ones_like(p)
    v, eta = VELOCITY_SETS["tg"]
    steps = int(round(t_end / dt))
    return Run("taylor_green_paper", n, n, d, d, dt, 5e-4, 1.4, v, eta, PERIODIC, PERIODIC,
               steps, rho, ux, uy, p / rho)


def taylor_green_2pi(n: int = 512, U0: float = 0.1, tau: float = 1e-4, dt: float = 1e-4,
                     steps: int = 10000, gamma: float = 1.4) -> Run:
    """Taylor-Green vortex on [0, 2 pi)^2: u = U0 sin x cos y, v = -U0 cos x sin y.

    rho = 1 and the incompressible pressure p = 1 + (U0^2/4)(cos 2x + cos 2y)
    (the sign that balances (u.grad)u for this velocity field), T = p / rho.
    Velocity set: the Sec. 3.5 one.
    """
    d = 2 * np.pi / n
    x = cell_centres(n, d)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ux = U0 * np.sin(X) * np.cos(Y)
    uy = -U0 * np.cos(X) * np.sin(Y)
    p = 1.0 + U0 ** 2 / 4 * (np.cos(2 * X) + np.cos(2 * Y))
    rho = np.ones_like(p)
    v, eta = VELOCITY_SETS["tg"]
    return Run("taylor_green_2pi", n, n, d, d, dt, tau, gamma, v, eta, PERIODIC, PERIODIC,
               steps, rho, ux, uy, p / rho)


def sound_wave_cone(nx: int = 1600, ny: int = 1200, dx: float = 5e-4, dt: float = 2e-5,
                    tau: float = 1e-4, gamma: float = 1.4, t_end: float = 0.2) -> Run:
    """The Sec. 3.4 two-dimensional sound wave: 1600 x 1200 cells of 5e-4,
    dt = 2e-5, tau = 1e-4, gamma = 1.4, Sec. 3.4 velocity set, to t = 0.2.

    The paper states neither the background nor the source.  Reading: gas at
    rest with rho = 1 and T = 1 (so that its kinematic viscosity T tau is the
    1e-4 it quotes), zero-gradient sides, and a perturbation that is
    introduced continuously at a point moving to the right at twice the
    sound speed from x0 (see SoundSource); the disturbance it leaves spreads
    at the sound speed, so its envelope is a cone of half-angle theta with
    sin(theta) = 1/2."""
    v, eta = VELOCITY_SETS["sound"]
    one = np.ones((ny, nx))
    return Run("sound_wave_cone", nx, ny, dx, dx, dt, tau, gamma, v, eta, ZERO_GRADIENT,
               ZERO_GRADIENT, int(round(t_end / dt)), one, 0.0 * one, 0.0 * one, one.copy())


@dataclasses.dataclass
class SoundSource:
    """A moving point source of equilibrium gas at rest (a density pulse at
    the background temperature): at time t it adds, per unit time,
    rate * exp(-|r - r_s(t)|^2 / (2 width^2)) of density at the cells within
    4 widths of r_s(t) = (x0 + speed t, y0).  The velocity-space shape of the
    added gas is the equilibrium of the background state, which each side
    computes with its own equilibrium."""

    x0: float
    y0: float
    speed: float
    width: float
    rate: float

    def window(self, run: Run, t: float):
        """Cell ranges (x slice, y slice) and the density added per unit time
        on them at time t, as a (ny_w, nx_w) float64 array."""
        xs = self.x0 + self.speed * t
        r = 4.0 * self.width
        i0 = max(0, int(np.floor((xs - r) / run.dx)))
        i1 = min(run.nx, int(np.ceil((xs + r) / run.dx)) + 1)
        j0 = max(0, int(np.floor((self.y0 - r) / run.dy)))
        j1 = min(run.ny, int(np.ceil((self.y0 + r) / run.dy)) + 1)
        x = (np.arange(i0, i1) + 0.5) * run.dx
        y = (np.arange(j0, j1) + 0.5) * run.dy
        X, Y = np.meshgrid(x, y, indexing="xy")
        g = self.rate * np.exp(-((X - xs) ** 2 + (Y - self.y0) ** 2) / (2 * self.width ** 2))
        return slice(i0, i1), slice(j0, j1), g


def sound_wave_source(run: Run, mach: float = 2.0, x0_frac: float = 0.3125,
                      width_cells: float = 4.0, rate: float = 1.0) -> SoundSource:
    """The moving source of sound_wave_cone: speed mach * sqrt(gamma T) with
    T = 1, starting at x0 = x0_frac * Lx (0.25 of the 0.8-long domain, so
    that the first disturbance stays inside it until t = 0.2) on the
    mid-line."""
    c = math.sqrt(run.gamma * 1.0)
    return SoundSource(x0_frac * run.nx * run.dx, 0.5 * run.ny * run.dy, mach * c,
                       width_cells * run.dx, rate)


def cone_sin_theta(drho: np.ndarray, run: Run, src: SoundSource, t: float,
                   d_range=(0.06, 0.30)):
    """Half-angle of the Mach cone in a density perturbation field drho
    (ny, nx) at time t.  In every column between d_range[0] and d_range[1]
    behind the apex x0 + speed t, on each side of the mid-line, the Mach wave
    is the largest value of drho; its position is refined to a fraction of a
    cell by the parabola through that cell and its two neighbours.  A
    straight line fitted to those positions on each side gives tan(theta).
    (The outer edge of the disturbance, say where drho falls to half its
    peak, lies further out the older the wave is, as the wave spreads; the
    peak does not move with the spreading.)  Returns (sin(theta), per-side
    tan(theta), number of columns).  Field analysis only: no arithmetic of
    the method."""
    xa = src.x0 + src.speed * t
    x = (np.arange(run.nx) + 0.5) * run.dx
    y = (np.arange(run.ny) + 0.5) * run.dy
    cols = np.nonzero((xa - x >= d_range[0]) & (xa - x <= d_range[1]))[0]
    jm = int(np.searchsorted(y, src.y0))
    slopes = []
    for side in (1, -1):
        xs, ys = [], []
        for i in cols:
            col = drho[jm:, i] if side > 0 else drho[jm - 1::-1, i]
            yy = y[jm:] if side > 0 else y[jm - 1::-1]
            k = int(np.argmax(col))
            if k == 0 or k + 1 >= col.size:
                continue
            a, b, c = col[k - 1], col[k], col[k + 1]
            den = a - 2.0 * b + c
            off = 0.5 * (a - c) / den if den != 0.0 else 0.0
            ys.append(yy[k] + off * (yy[k + 1] - yy[k]))
            xs.append(x[i])
        slope = np.polyfit(np.asarray(xs), np.abs(np.asarray(ys) - src.y0), 1)[0]
        slopes.append(float(-slope))
    tan = float(np.mean(slopes))
    return tan / math.sqrt(1.0 + tan * tan), slopes, int(len(cols))


HEADLINE_GAMMAS = (1.2, 1.4, 5.0 / 3.0)

# Velocity set of the headline workload per specific-heat ratio: the Sec. 3.2
# Lax set where it is stable in 2D (gamma = 1.4, 5/3).  For gamma = 1.2
# (I = 8) that set blows up within a few hundred steps; raising eta_c to
# about sqrt(I T) = 8 in the hot left state (the rule of thumb given after
# Eq. (3)) and eta_b to 5 keeps the 4096^2 run finite over 2000 steps.
HEADLINE_SETS = {
    1.4: VELOCITY_SETS["lax"],
    5.0 / 3.0: VELOCITY_SETS["lax"],
    1.2: ((4.4, 4.4, 3.0, 1.8), (0.0, 5.0, 8.0, 0.0)),
}


def lax_acoustic_2d(n: int = 4096, seed: int = 0, steps: int = 2000, ny: int | None = None,
                    dx: float = 2e-3, dt: float = 2e-5, tau: float = 1e-4,
                    gamma: float | None = None) -> Run:
    """Lax tube extruded in y with an oblique density wave on top (the headline workload).

    Cells of size dx (the Sec. 3.2 spacing by default) on [0, L) x [0, L ny / n),
    L = n dx.  Lax states of Sec. 3.2 with the diaphragm at x = L / 2; the density
    is multiplied by 1 + 1e-3 cos(2 pi (2 x / L + 3 y / L) + phi).  phi ~ U[0, 2 pi)
    and, unless given, gamma ~ U{1.2, 1.4, 5/3}, both from numpy's
    default_rng(seed).  Zero-gradient in x, periodic in y; velocity set from
    HEADLINE_SETS.
    """
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2 * np.pi)
    g_pick = HEADLINE_GAMMAS[int(rng.integers(0, len(HEADLINE_GAMMAS)))]
    if gamma is None:
        gamma = g_pick
    length = n * dx
    x = cell_centres(n, dx)
    y = cell_centres(ny, dx)
    rho, ux, uy, T = _two_state(n, ny, x, 0.5 * length, (0.445, 0.698, 0.0, 7.928),
                                (0.5, 0.0, 0.0, 1.142))
    X, Y = np.meshgrid(x, y, indexing="xy")
    rho = rho * (1.0 + 1e-3 * np.cos(2 * np.pi * (2 * X / length + 3 * Y / length) + phi))
    key = min(HEADLINE_SETS, key=lambda g: abs(g - gamma))
    v, eta = HEADLINE_SETS[key]
    return Run(f"lax_acoustic_{n}x{ny}_seed{seed}", n, ny, dx, dx, dt, tau, gamma, v, eta,
               ZERO_GRADIENT, PERIODIC, steps, rho, ux, uy, T)


def fourier_field(rng: np.random.Generator, nx: int, ny: int, modes: int = 5) -> np.ndarray:
    """Periodic sum of `modes` plane waves with wave numbers in {1..4}^2 (domain [0,1)^2),
    random amplitudes and phases, normalised so that max |s| = 1."""
    x = cell_centres(nx, 1.0 / nx)
    y = cell_centres(ny, 1.0 / ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    s = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(1, 5, size=2)
        amp = rng.uniform(0.2, 1.0)
        ph = rng.uniform(0.0, 2 * np.pi)
        s += amp * np.cos(2 * np.pi * (kx * X + ky * Y) + ph)
    return s / np.abs(s).max()


def smooth_random_fields(rng: np.random.Generator, nx: int, ny: int, umax: float = 0.29):
    """rho, T in [0.5, 2] as 1.25 + 0.75 s and a velocity with max |u| = umax."""
    rho = 1.25 + 0.75 * fourier_field(rng, nx, ny)
    T = 1.25 + 0.75 * fourier_field(rng, nx, ny)
    ux = fourier_field(rng, nx, ny)
    uy = fourier_field(rng, nx, ny)
    mag = np.sqrt(ux ** 2 + uy ** 2).max()
    return rho, ux * umax / mag, uy * umax / mag, T


def random_periodic(nx: int, ny: int, seed: int, dt: float = 1e-5, tau: float = 1e-4,
                    gamma: float = 1.4, vset: str = "sound", steps: int = 1,
                    umax: float = 0.29) -> Run:
    """Smooth random fields on a periodic [0,1)^2 grid (dx = 1/nx, dy = 1/ny)."""
    rng = np.random.default_rng(seed)
    rho, ux, uy, T = smooth_random_fields(rng, nx, ny, umax)
    v, eta = VELOCITY_SETS[vset]
    return Run(f"random_{nx}x{ny}_seed{seed}", nx, ny, 1.0 / nx, 1.0 / ny, dt, tau, gamma,
               v, eta, PERIODIC, PERIODIC, steps, rho, ux, uy, T)


BATCH_SIZES = tuple(range(128, 1025, 64))


def batched_ensemble(ngrids: int = 96, seed: int = 0, dt: float = 1e-5, steps: int = 1000,
                     sizes: Tuple[int, ...] = BATCH_SIZES, vset: str = "sound_t2") -> List[Run]:
    """Independent periodic [0,1)^2 grids of uneven size, each with its own gamma and tau.

    N ~ U{sizes}, gamma ~ U[1.1, 1.67], tau = 10^U[-5, -3]; fields from smooth_random_fields.
    """
    rng = np.random.default_rng(seed)
    runs = []
    for g in range(ngrids):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        gamma = float(rng.uniform(1.1, 1.67))
        tau = float(10.0 ** rng.uniform(-5.0, -3.0))
        rho, ux, uy, T = smooth_random_fields(rng, n, n)
        v, eta = VELOCITY_SETS[vset]
        runs.append(Run(f"batch{g}_{n}", n, n, 1.0 / n, 1.0 / n, dt, tau, gamma, v, eta,
                        PERIODIC, PERIODIC, steps, rho, ux, uy, T))
    return runs


def adjoint_problem(n: int = 256, seed: int = 0, steps: int = 2000, dt: float = 2e-5,
                    tau: float = 1e-4, gamma: float = 1.4, perturb: float = 0.01,
                    vset: str = "sound_t2"):
    """Initial fields and a perturbed target run for the gradient workload.

    Returns (run, target_run): the target starts from fields perturbed by `perturb`
    times an independent smooth field (seed + 1) and uses tau * 1.1.
    """
    base = random_periodic(n, n, seed, dt=dt, tau=tau, gamma=gamma, steps=steps, vset=vset)
    rng = np.random.default_rng(seed + 1)
    pr = fourier_field(rng, n, n)
    pu = fourier_field(rng, n, n)
    pv = fourier_field(rng, n, n)
    pt = fourier_field(rng, n, n)
    tgt = base.with_fields(base.rho * (1 + perturb * pr), base.ux + perturb * 0.29 * pu,
                           base.uy + perturb * 0.29 * pv, base.T * (1 + perturb * pt),
                           tau=tau * 1.1, name=base.name + "_target")
    return base, tgt


def uniform(nx: int, ny: int, rho=1.0, ux=0.0, uy=0.0, T=1.0, vset="sound", dt=1e-5,
            tau=1e-4, gamma=1.4, dx=None) -> Run:
    dx = 1.0 / nx if dx is None else dx
    v, eta = VELOCITY_SETS[vset]
    full = lambda c: np.full((ny, nx), float(c))
    return Run("uniform", nx, ny, dx, dx, dt, tau, gamma, v, eta, PERIODIC, PERIODIC, 1,
               full(rho), full(ux), full(uy), full(T))


def headline(seed: int = 0, steps: int = 2000, n: int = 4096) -> Run:
    """The throughput workload: 4096 x 4096 cells of lax_acoustic_2d."""
    return lax_acoustic_2d(n, seed=seed, steps=steps)


def headline_sample(side: int, seed: int = 0, steps: int = 2000) -> Run:
    """The headline setup on a side x side grid with the same cell size, time
    step, relaxation time, gamma and velocity set (a smaller domain)."""
    return lax_acoustic_2d(side, seed=seed, steps=steps)


__all__ = [n for n in dir() if not n.startswith("_")]
