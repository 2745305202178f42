"""Physics pins of the oracle: exact Riemann solutions, Rankine-Hugoniot,
acoustic speed sqrt(gamma T) and Taylor-Green decay (Secs. 3.1-3.5)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import analytic as A
from oracle import cdbm as C
from oracle import riemann as R
import workloads as W


def test_riemann_solver_matches_textbook_star_states(golden_dir):
    tab = json.load(open(os.path.join(golden_dir, "riemann_textbook.json")))
    g = tab["gamma"]
    for t in tab["tests"]:
        st = R.star_state(R.State(*t["L"]), R.State(*t["R"]), g)
        for got, want in ((st.p, t["p"]), (st.u, t["u"]), (st.rho_L, t["rhoL"]), (st.rho_R, t["rhoR"])):
            assert abs(got - want) <= 5e-5 * max(abs(want), 1.0) + 1e-5, (t, got, want)


def test_paper_shock_state_is_rankine_hugoniot(golden_dir):
    s = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["shock_ma15"]
    rho2, u2, T2, p2, speed = A.normal_shock(s["Ma"], s["gamma"])
    L = s["left"]
    assert abs(rho2 - L[0]) < 1e-4 and abs(u2 - L[1]) < 1e-4
    assert abs(T2 - L[3]) < 5e-4 and abs(p2 - L[4]) < 1e-4
    # p = rho T for the printed numbers
    assert abs(L[0] * L[3] - L[4]) < 2e-3
    # the exact Riemann solution of the printed states is a single right shock
    st = R.star_state(R.State(L[0], L[1], L[4]), R.State(1.0, 0.0, 1.0), s["gamma"])
    assert abs(st.p - L[4]) / L[4] < 1e-4 and abs(st.u - L[1]) / L[1] < 1e-4
    assert abs(R.shock_speed(R.State(1.0, 0.0, 1.0), st.p, s["gamma"], 1) - speed) < 1e-3


@pytest.mark.slow
def test_sod_tube_against_exact_riemann():
    run = W.sod_tube()       # 500 x 1, dx = 2e-3, 5000 steps to t = 0.1, gamma = 1.4
    p = C.Params.from_run(run)
    f = C.run_from_fields(run)
    rho, ux, _, T = (a.numpy()[0] for a in C.fields(f, p))
    x = W.cell_centres(run.nx, run.dx)
    t = run.steps * run.dt
    re, ue, pe = R.sample(R.State(1.0, 0.0, 1.0), R.State(0.125, 0.0, 0.1), 1.4, (x - 0.5) / t)
    assert np.mean(np.abs(rho - re)) < 1e-2
    assert np.mean(np.abs(ux - ue)) < 1e-2
    assert np.mean(np.abs(rho * T - pe)) < 1e-2
    # shock position: where the density crosses the mid-value between rho*_R and rho_R
    st = R.star_state(R.State(1.0, 0.0, 1.0), R.State(0.125, 0.0, 0.1), 1.4)
    shock_x = 0.5 + R.shock_speed(R.State(0.125, 0.0, 0.1), st.p, 1.4, 1) * t
    mid = 0.5 * (st.rho_R + 0.125)
    k = np.where((rho[:-1] > mid) & (rho[1:] <= mid) & (x[:-1] > 0.6))[0]
    assert k.size >= 1 and abs(x[k[-1]] - shock_x) < 3 * run.dx


@pytest.mark.parametrize("gamma", [1.2, 1.4, 5.0 / 3.0])
def test_acoustic_wave_speed(gamma):
    """A small right-running plane wave travels at sqrt(gamma T)."""
    n, T0, rho0, amp = 64, 1.0, 1.0, 1e-4
    dx = 1.0 / n
    x = W.cell_centres(n, dx)
    k = 2 * np.pi
    r, u, T = A.acoustic_plane_wave(x, rho0, T0, gamma, amp, k)
    v, eta = W.VELOCITY_SETS["sound"]
    run = W.Run("ac", n, 1, dx, dx, 5e-4, 1e-3, gamma, v, eta, W.PERIODIC, W.PERIODIC, 0,
                r[None], u[None], np.zeros((1, n)), T[None])
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)

    def phase(g):
        rho = C.fields(g, p)[0].numpy()[0]
        return np.angle(np.sum((rho - rho.mean()) * np.exp(-1j * k * x)))

    ph0 = phase(f)
    steps = 400
    f = C.run(f, p, steps)
    t = steps * p.dt
    dphi = (phase(f) - ph0 + np.pi) % (2 * np.pi) - np.pi
    c_num = -dphi / (k * t)
    assert abs(c_num - A.sound_speed(gamma, T0)) / A.sound_speed(gamma, T0) < 0.01


@pytest.mark.slow
def test_taylor_green_convergence(golden_dir):
    """Eq. (25) error of u_x against Eqs. (22)-(24) at t = 0.1 on the grids of
    Fig. 8; the paper reports a slope of 1.69."""
    tg = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["taylor_green"]
    ns = [20, 30, 40]
    errs = []
    for n in ns:
        run = W.taylor_green_paper(n=n, t_end=0.1)
        p = C.Params.from_run(run)
        f = C.run_from_fields(run)
        _, ux, _, _ = (a.numpy() for a in C.fields(f, p))
        x = W.cell_centres(n, run.dx)
        X, Y = np.meshgrid(x, x, indexing="xy")
        ex, _, _ = A.taylor_green(X, Y, run.steps * run.dt, tg["u0"], tg["p0"], tg["L"], tg["Re"])
        errs.append(A.relative_l2(ux, ex, tg["u0"]))
    slope = np.polyfit(np.log([2 * tg["L"] / n for n in ns]), np.log(errs), 1)[0]
    assert 1.5 < slope < 2.1, (slope, errs)
    assert errs[-1] < 0.05


def _fan_cases():
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "riemann_textbook.json")))
    cases = [(R.State(*t["L"]), R.State(*t["R"]), tab["gamma"]) for t in tab["tests"][:4]]
    lax = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "paper_printed.json")))["lax_paper"]
    L, Rt = lax["left"], lax["right"]
    for g in (1.2, 1.4, 5.0 / 3.0):
        cases.append((R.State(L[0], L[1], L[0] * L[3]), R.State(Rt[0], Rt[1], Rt[0] * Rt[3]), g))
    return cases


@pytest.mark.parametrize("case", range(7))
def test_rarefaction_fans_keep_their_riemann_invariants(case):
    """Inside a rarefaction fan of the sampled exact solution the entropy
    p / rho^gamma and the Riemann invariant u +- 2c / (gamma - 1) of the
    family that is not crossed keep the values of the state the fan opens
    from; the fan's head moves at u_K -+ c_K and its tail at u* -+ c*_K, with
    the undisturbed and star states just outside (Toro tests 1-4 and the Sec.
    3.2 Lax states at three gammas)."""
    L, Rs, g = _fan_cases()[case]
    st = R.star_state(L, Rs, g)
    fans = 0
    for side, K in ((-1, L), (1, Rs)):
        if st.p > K.p:
            continue                      # a shock on this side
        fans += 1
        cK = math.sqrt(g * K.p / K.rho)
        rho_s = st.rho_L if side < 0 else st.rho_R
        cs = math.sqrt(g * st.p / rho_s)
        head, tail = K.u + side * cK, st.u + side * cs
        lo, hi = min(head, tail), max(head, tail)
        xi = np.linspace(lo, hi, 41)[1:-1]
        rho, u, p = R.sample(L, Rs, g, xi)
        c = np.sqrt(g * p / rho)
        inv = u - side * 2.0 * c / (g - 1.0)
        want = K.u - side * 2.0 * cK / (g - 1.0)
        assert np.abs(inv - want).max() <= 1e-10 * (abs(want) + cK)
        ent = p / rho ** g
        assert np.abs(ent / (K.p / K.rho ** g) - 1.0).max() <= 1e-10
        # the fan is centred: the characteristic speed u -+ c equals x / t
        assert np.abs(u + side * c - xi).max() <= 1e-10 * (abs(K.u) + cK)
        eps = 1e-9 * (hi - lo)
        outside = head + side * eps
        r0, u0, p0 = R.sample(L, Rs, g, np.array([outside]))
        assert (r0[0], u0[0], p0[0]) == (K.rho, K.u, K.p)
        r1, u1, p1 = R.sample(L, Rs, g, np.array([tail + side * eps]))
        assert abs(p1[0] - st.p) <= 1e-6 * st.p and abs(r1[0] - rho_s) <= 1e-6 * rho_s
        r2, u2, p2 = R.sample(L, Rs, g, np.array([tail - side * eps]))
        assert (r2[0], u2[0], p2[0]) == (rho_s, st.u, st.p)
    assert fans >= 1
