"""Pins of the oracle's thermodynamic-nonequilibrium slots (Eqs. (8)-(11))
and of its heat-flux measure against a Chapman-Enskog estimate.

Every slot of the TNE output (Delta*_2 xx, xy, yy; Delta*_{3,1} x, y;
Delta*_3 xxx, xxy, xyy, yyy; Delta*_{4,2} xx, xy, yy) is fixed two ways:

* hand-worked special cases: a state at rest plus a perturbation that
  changes none of rho, j and 2E, so that f^eq and u stay those of the state
  at rest and each Delta* is the plain sum over the perturbation of the
  velocity monomial the slot names, worked out by hand below for the
  velocities involved (a swap of any two slots, a sign or a dropped eta^2
  moves a value that is checked);
* reflections: mirroring a general non-equilibrium field in x (or
  exchanging x and y) must map each slot to the slot and sign its
  monomial dictates, on a field with flow, gradients and all 16 f_i off
  equilibrium.
"""
import numpy as np
import pytest
import torch

from oracle import cdbm as C
import workloads as W

SLOTS = ("2xx", "2xy", "2yy", "31x", "31y", "3xxx", "3xxy", "3xyy", "3yyy",
         "42xx", "42xy", "42yy")

# velocity index of each direction in each group (counter-clockwise from +x)
A = {"+x": 0, "+y": 1, "-x": 2, "-y": 3}          # axis group a; group c adds 8
B = {"pp": 4, "mp": 5, "mm": 6, "pm": 7}          # diagonal group b: (+1,+1), (-1,+1), ...


def _params(vset="sound", I=3.0):
    v, eta = W.VELOCITY_SETS[vset]
    return C.Params(1, 1, 1.0, 1.0, 1e-4, 1e-4, I, v, eta, C.PERIODIC, C.PERIODIC)


def _tne_of_perturbation(p, delta):
    """TNE of f^eq(rho = 1, u = 0, T = 1) + delta on a 1 x 1 grid."""
    one = torch.ones((1, 1), dtype=torch.float64)
    zero = torch.zeros((1, 1), dtype=torch.float64)
    f = C.initial_distribution(one, zero, zero, one, p)
    f = f + torch.as_tensor(delta, dtype=torch.float64).reshape(16, 1, 1)
    out = C.nonequilibrium(f, p).reshape(12).numpy()
    return dict(zip(SLOTS, out))


def _expect(got, want, scale):
    for k in SLOTS:
        w = want.get(k, 0.0)
        assert abs(got[k] - w) <= 1e-9 * scale, (k, got[k], w)


def test_even_axis_perturbation_fixes_xx_and_yy_slots():
    """delta = e(+x) + e(-x) - e(+y) - e(-y) in group a: Delta*_2xx = 2 e v_a^2,
    Delta*_2yy = -2 e v_a^2, Delta*_{4,2} xx / yy = +- 2 e v_a^2 (v_a^2 + eta_a^2)."""
    p = _params()
    va, ea = p.v[0], p.eta[0]
    e = 1e-3
    d = np.zeros(16)
    d[A["+x"]] = d[A["-x"]] = e
    d[A["+y"]] = d[A["-y"]] = -e
    got = _tne_of_perturbation(p, d)
    _expect(got, {"2xx": 2 * e * va ** 2, "2yy": -2 * e * va ** 2,
                  "42xx": 2 * e * va ** 2 * (va ** 2 + ea ** 2),
                  "42yy": -2 * e * va ** 2 * (va ** 2 + ea ** 2)}, e * va ** 4)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_odd_axis_perturbation_fixes_heat_flux_and_cubic_slots(axis):
    """delta = e [e(+r) - e(-r)] in group a minus e v_a / v_c [e(+r) - e(-r)] in
    group c (zero net momentum): Delta*_{3,1,r} = 2 e v_a [(v_a^2 + eta_a^2) -
    (v_c^2 + eta_c^2)] and Delta*_{3,rrr} = 2 e v_a (v_a^2 - v_c^2); every other slot 0."""
    p = _params("lax", I=3.0)
    va, vc, ea, ec = p.v[0], p.v[2], p.eta[0], p.eta[2]
    e = 1e-3
    d = np.zeros(16)
    d[A["+" + axis]], d[A["-" + axis]] = e, -e
    d[8 + A["+" + axis]], d[8 + A["-" + axis]] = -e * va / vc, e * va / vc
    got = _tne_of_perturbation(p, d)
    q = 2 * e * va * ((va ** 2 + ea ** 2) - (vc ** 2 + ec ** 2))
    c3 = 2 * e * va * (va ** 2 - vc ** 2)
    _expect(got, {"31" + axis: q, "3" + axis * 3: c3}, e * 100.0)


def test_diagonal_perturbation_separates_xxy_from_xyy():
    """delta = e [e(+,+) + e(-,+) - e(+,-) - e(-,-)] in group b, its y momentum
    4 e v_b removed with -2 e v_b / v_a [e(+y) - e(-y)] in group a:
    Delta*_{3,xxy} = 4 e v_b^3, Delta*_{3,xyy} = 0, Delta*_{3,yyy} = 4 e v_b (v_b^2 - v_a^2),
    Delta*_{3,1,y} = 4 e v_b [(2 v_b^2 + eta_b^2) - (v_a^2 + eta_a^2)]."""
    p = _params("tg", I=3.0)
    va, vb, ea, eb = p.v[0], p.v[1], p.eta[0], p.eta[1]
    e = 1e-3
    d = np.zeros(16)
    d[B["pp"]] = d[B["mp"]] = e
    d[B["pm"]] = d[B["mm"]] = -e
    k = 2 * e * vb / va
    d[A["+y"]], d[A["-y"]] = -k, k
    got = _tne_of_perturbation(p, d)
    _expect(got, {"3xxy": 4 * e * vb ** 3, "3yyy": 4 * e * vb * (vb ** 2 - va ** 2),
                  "31y": 4 * e * vb * ((2 * vb ** 2 + eb ** 2) - (va ** 2 + ea ** 2))},
            e * 100.0)


def test_diagonal_shear_perturbation_fixes_xy_slots():
    """delta = e [e(+,+) - e(-,+) + e(-,-) - e(+,-)] in group d: Delta*_2xy = 4 e v_d^2,
    Delta*_{4,2,xy} = 4 e v_d^2 (2 v_d^2 + eta_d^2); every other slot 0."""
    p = _params("sod", I=3.0)
    vd, ed = p.v[3], p.eta[3]
    e = 1e-3
    d = np.zeros(16)
    d[8 + B["pp"]], d[8 + B["mp"]], d[8 + B["mm"]], d[8 + B["pm"]] = e, -e, e, -e
    got = _tne_of_perturbation(p, d)
    _expect(got, {"2xy": 4 * e * vd ** 2, "42xy": 4 * e * vd ** 2 * (2 * vd ** 2 + ed ** 2)},
            e * 10.0)


# Velocity index maps of the reflections: x -> -x, and x <-> y.
_MIRROR_X = {A["+x"]: A["-x"], A["-x"]: A["+x"], A["+y"]: A["+y"], A["-y"]: A["-y"],
             B["pp"]: B["mp"], B["mp"]: B["pp"], B["mm"]: B["pm"], B["pm"]: B["mm"]}
_SWAP_XY = {A["+x"]: A["+y"], A["+y"]: A["+x"], A["-x"]: A["-y"], A["-y"]: A["-x"],
            B["pp"]: B["pp"], B["mm"]: B["mm"], B["mp"]: B["pm"], B["pm"]: B["mp"]}
# the image of each slot and its sign under the two reflections
_SLOT_MIRROR_X = {"2xx": ("2xx", 1), "2xy": ("2xy", -1), "2yy": ("2yy", 1), "31x": ("31x", -1),
                  "31y": ("31y", 1), "3xxx": ("3xxx", -1), "3xxy": ("3xxy", 1),
                  "3xyy": ("3xyy", -1), "3yyy": ("3yyy", 1), "42xx": ("42xx", 1),
                  "42xy": ("42xy", -1), "42yy": ("42yy", 1)}
_SLOT_SWAP_XY = {"2xx": ("2yy", 1), "2xy": ("2xy", 1), "2yy": ("2xx", 1), "31x": ("31y", 1),
                 "31y": ("31x", 1), "3xxx": ("3yyy", 1), "3xxy": ("3xyy", 1),
                 "3xyy": ("3xxy", 1), "3yyy": ("3xxx", 1), "42xx": ("42yy", 1),
                 "42xy": ("42xy", 1), "42yy": ("42xx", 1)}


def _perm(m):
    full = dict(m)
    full.update({8 + i: 8 + j for i, j in m.items()})
    return [full[i] for i in range(16)]


def _nonequilibrium_field(n=12, steps=3):
    """A square periodic field off equilibrium: smooth random fields advanced
    a few steps with a long relaxation time, so every f_i carries gradients."""
    run = W.random_periodic(n, n, seed=3, dt=2e-3, tau=5e-2, vset="tg")
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    return p, C.run(f, p, steps)


@pytest.mark.parametrize("which", ["mirror_x", "swap_xy"])
def test_reflections_map_each_slot_to_its_image(which):
    p, f = _nonequilibrium_field()
    if which == "mirror_x":
        perm, slot_map = _perm(_MIRROR_X), _SLOT_MIRROR_X
        # new f_i(x, y) = f_{perm(i)}(-x, y): reverse the columns
        g = f[perm].flip(2)
        back = lambda t: t.flip(1)
    else:
        perm, slot_map = _perm(_SWAP_XY), _SLOT_SWAP_XY
        g = f[perm].transpose(1, 2).contiguous()
        back = lambda t: t.transpose(0, 1)
    d = C.nonequilibrium(f, p)
    dg = C.nonequilibrium(g, p)
    scale = float(d.abs().max())
    assert scale > 1e-6
    for k, name in enumerate(SLOTS):
        img, sign = slot_map[name]
        j = SLOTS.index(img)
        # slot `img` of the reflected field, mapped back, is sign * slot `name`
        diff = float((back(dg[j]) - sign * d[k]).abs().max())
        assert diff <= 1e-9 * scale, (which, name, img, diff)


@pytest.mark.parametrize("I,vset", [(3.0, "sound"), (8.0, "lax")])
def test_heat_flux_matches_chapman_enskog(I, vset):
    """Delta*_{3,1} is twice the heat flux: for the BGK gas of Eq. (1) the
    Chapman-Enskog flux at rest is q = -(D + I + 2)/2 rho T tau grad T, so
    Delta*_{3,1,x} = -(D + I + 2) rho T tau dT/dx on a smooth temperature wave
    at uniform pressure (after the initial layer of a few tau), and
    Delta*_{3,1,y} = 0."""
    n, amp, tau, dt, steps = 64, 0.01, 1e-3, 1e-4, 200
    dx = 1.0 / n
    x = W.cell_centres(n, dx)
    T = 1.0 + amp * np.sin(2 * np.pi * x)
    rho = 1.0 / T
    v, eta = W.VELOCITY_SETS[vset]
    p = C.Params(n, 1, dx, dx, dt, tau, I, v, eta, C.PERIODIC, C.PERIODIC)
    zero = np.zeros((1, n))
    f = C.initial_distribution(rho[None], zero, zero, T[None], p)
    f = C.run(f, p, steps)
    r, ux, _, Tn = (a.numpy()[0] for a in C.fields(f, p))
    q = C.nonequilibrium(f, p).numpy()[:, 0, :]
    dTdx = (np.roll(Tn, -1) - np.roll(Tn, 1)) / (2 * dx)
    ce = -(2.0 + I + 2.0) * r * Tn * tau * dTdx
    assert np.abs(ux).max() < 3e-3 * amp   # no flow to speak of
    err = np.abs(q[3] - ce).max() / np.abs(ce).max()
    assert err < 0.10, err
    assert np.abs(q[4]).max() < 1e-10 * np.abs(ce).max() + 1e-15
