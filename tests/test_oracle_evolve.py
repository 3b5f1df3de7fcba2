"""Pins of the oracle's time-stepped evolution harness (oracle/evolve.py):

* advance() against a tight numerical integration of the rate equation
  dx/dt = alpha n (1 - x)^2 - k x (section 2.2, Eq. dndt) by scipy's implicit
  Radau method, over ionising, recombining, gas-free, k = 0 and long steps;
  and the property any exact solution has: two steps equal one of their sum.
* smooth3() on a constant field (unchanged), a unit impulse inside (the
  binomial weights 1/8, 1/16, 1/32, 1/64 by hand) and at a corner (weights
  renormalised over the 8 cells inside, by hand).
* next_dt() on fields whose answer follows from Eq. dtelec by hand, with the
  front mask, the doubling bound (Eq. dtchange), dt_max and the time left.
* The whole loop on Test 1 (section 4.1): a 5e48 ph/s source at the corner of
  a 6.6 kpc box of n_H = 1e-3, x = 1 - 1.2e-3; the ionised volume's
  equivalent front radius follows r_s(t) = R_s (1 - e^{-t/t_rec})^{1/3}
  (Eq. rstr) within 2 % at t_rec / 2 and 3 % at 2 t_rec.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import evolve as EV
from paper_1012_2865_amd import workloads as W

ALPHA = 2.59e-13


def _ode(x0, k, n, dt):
    a = ALPHA * n
    sol = solve_ivp(lambda t, x: a * (1.0 - x) ** 2 - k * x, (0.0, dt), [x0], method="Radau",
                    rtol=1e-12, atol=1e-15)
    return float(sol.y[0, -1])


@pytest.mark.parametrize("x0,k,n,dt", [
    (0.9988, 1e-12, 1e-3, 1e12),      # ionising, a few e-foldings
    (0.9988, 1e-12, 1e-3, 1e10),      # ionising, short step
    (1e-4, 0.0, 1e-3, 3e15),          # recombining only (k = 0, double root at 1)
    (0.3, 1e-14, 1.0, 1e13),          # dense: recombinations dominate
    (0.05, 5e-13, 1e-2, 4e12),        # below equilibrium, rising back
    (1.0, 3e-11, 1e-4, 1e9),          # from neutral, fast
])
def test_advance_follows_the_rate_equation(x0, k, n, dt):
    got = float(EV.advance(np.array([x0]), np.array([k]), np.array([n]), dt)[0])
    want = _ode(x0, k, n, dt)
    assert got == pytest.approx(want, rel=1e-8, abs=1e-12)


def test_advance_special_cases_and_semigroup():
    rng = np.random.default_rng(5)
    x0 = rng.uniform(0.0, 1.0, 200)
    k = 10 ** rng.uniform(-16, -11, 200)
    n = 10 ** rng.uniform(-4, 0, 200)
    t1, t2 = 10 ** rng.uniform(9, 14, 200), 10 ** rng.uniform(9, 14, 200)
    one = EV.advance(x0, k, n, t1 + t2)
    two = EV.advance(EV.advance(x0, k, n, t1), k, n, t2)
    assert np.allclose(one, two, rtol=1e-9, atol=1e-13)
    assert np.all((one >= 0.0) & (one <= 1.0))
    # no gas: unchanged; very long step: the equilibrium root
    assert EV.advance(np.array([0.4]), np.array([1e-12]), np.array([0.0]), 1e15)[0] == 0.4
    a = ALPHA * 1e-2
    k1 = 1e-12
    root = 2 * a / ((2 * a + k1) + math.sqrt(k1 * k1 + 4 * a * k1))
    assert EV.advance(np.array([1.0]), np.array([k1]), np.array([1e-2]), 1e16)[0] == pytest.approx(root, rel=1e-12)


def test_smooth3_weights_by_hand():
    f = np.full((5, 6, 7), 3.25)
    assert np.allclose(EV.smooth3(f), 3.25, rtol=1e-15)
    imp = np.zeros((5, 5, 5))
    imp[2, 2, 2] = 1.0
    s = EV.smooth3(imp)
    assert s[2, 2, 2] == pytest.approx(1 / 8)
    assert s[2, 2, 3] == pytest.approx(1 / 16) and s[1, 2, 2] == pytest.approx(1 / 16)
    assert s[2, 3, 3] == pytest.approx(1 / 32)
    assert s[3, 3, 3] == pytest.approx(1 / 64)
    assert s[2, 2, 4] == 0.0
    corner = np.zeros((4, 4, 4))
    corner[0, 0, 0] = 1.0
    s = EV.smooth3(corner)
    # inside neighbours of the corner: weights (1/2 or 1/4)^3, their sum (3/4)^3
    assert s[0, 0, 0] == pytest.approx((1 / 8) / (27 / 64))
    assert s[1, 1, 1] == pytest.approx(1 / 64)        # an inner cell: its weights sum to 1
    # cell (1,0,0)'s neighbourhood: x-axis sum 1, y and z sums 3/4
    assert s[0, 0, 1] == pytest.approx((1 / 4 * 1 / 2 * 1 / 2) / (1 * 9 / 16))


def test_next_dt_by_hand():
    n = np.full((4, 4, 4), 1e-2)
    x = np.full((4, 4, 4), 0.5)
    k = np.full((4, 4, 4), 2e-13)
    dx = 1e20
    sig = 6.3e-18                      # tau_cell = 6.3e-18 * 1e-2 * 0.5 * 1e20 = 3.15 > 0.5
    rate = 2e-13 + 0.5 * 1e-2 * ALPHA
    want = 0.1 / rate
    assert EV.next_dt(k, x, n, dx, sig, 0.1, 0.5, 1e20, None, 1e30) == pytest.approx(want, rel=1e-14)
    assert EV.next_dt(k, x, n, dx, sig, 0.1, 0.5, 1e20, want / 3, 1e30) == pytest.approx(2 * want / 3, rel=1e-14)
    assert EV.next_dt(k, x, n, dx, sig, 0.1, 0.5, want / 5, None, 1e30) == pytest.approx(want / 5, rel=1e-14)
    assert EV.next_dt(k, x, n, dx, sig, 0.1, 0.5, 1e20, None, want / 7) == pytest.approx(want / 7, rel=1e-14)
    # outside the front (tau_cell below 0.5 everywhere): dt_max
    assert EV.next_dt(k, x, n, dx, sig, 0.1, 5.0, 123.0, None, 1e30) == 123.0
    # one front cell in a field at dt_max: the smoothed minimum sits on that cell
    x2 = np.full((4, 4, 4), 1e-4)
    x2[0, 0, 0] = 0.5
    dt_max = 10 * want
    s = (1 / 8 * want + (27 / 64 - 1 / 8) * dt_max) / (27 / 64)
    assert EV.next_dt(k, x2, n, dx, sig, 0.1, 0.5, dt_max, None, 1e30) == pytest.approx(s, rel=1e-13)


def _test1(n_cells, t_over_trec, dt_max_over_trec):
    box = 6.6 * W.KPC_CM
    g = W.uniform_grid(n_cells, box / n_cells, 1e-3, 1.0 - 1.2e-3)
    p = W.Problem([g], np.array([[0.0, 0.0, 0.0, 5e48]]), W.hydrogen_spectrum([13.6]), W.Params())
    t_rec = 1.0 / (ALPHA * 1e-3)
    x, _, steps, t, dts = EV.evolve(p, t_over_trec * t_rec, eps=0.1, dt_max=dt_max_over_trec * t_rec)
    v_ion = float(np.sum(1.0 - x)) * (box / n_cells) ** 3
    r = (6.0 * v_ion / math.pi) ** (1.0 / 3.0)                 # one octant of a sphere
    rs = (3.0 * 5e48 / (4.0 * math.pi * ALPHA * 1e-6)) ** (1.0 / 3.0)
    r_an = rs * (1.0 - math.exp(-t / t_rec)) ** (1.0 / 3.0)
    return r / r_an, steps, t / t_rec


@pytest.mark.parametrize("n_cells,t_over,dtm,tol", [(32, 0.5, 1 / 400, 0.02), (16, 2.0, 1 / 400, 0.03)])
def test_test1_front_follows_the_analytic_radius(n_cells, t_over, dtm, tol):
    ratio, steps, t = _test1(n_cells, t_over, dtm)
    print(f"{n_cells}^3 to {t:.2f} t_rec in {steps} steps: r_I / r_s = {ratio:.4f}")
    assert t == pytest.approx(t_over, rel=1e-12)
    assert abs(ratio - 1.0) < tol


def test_nested_grids_step_together_and_covered_cells_keep_x():
    # an optically thick root whose source's photons die in its first cells;
    # the child far away sees no radiation, so its gas only recombines:
    # x(t) = 1 - (1 - x0) / (1 + a t (1 - x0)) exactly, with a = alpha n_H
    n = 16
    g = W.uniform_grid(n, W.DX_C1, 1.0, 0.5)
    child = W.Grid(n_h=np.full((8, 8, 8), 2.0, np.float32), x_hi=np.full((8, 8, 8), 0.25, np.float32),
                   dx_cm=W.DX_C1 / 2, parent=0, offset=(10, 10, 10))
    p = W.Problem([g, child], np.array([[0.5, 0.5, 0.5, 1e49]]), W.hydrogen_spectrum([13.6]), W.Params())
    t_end = 3e12
    xs, res, steps, t, dts = EV.evolve(p, t_end, eps=0.1, dt_max=t_end / 20)
    assert isinstance(xs, list) and len(xs) == 2 and t == pytest.approx(t_end, rel=1e-12)
    assert steps >= 20 and np.max(res["k_ph"][1]) == 0.0
    a = ALPHA * 2.0
    want = 1.0 - 0.75 / (1.0 + a * t * 0.75)
    assert np.allclose(xs[1], want, rtol=1e-9, atol=0.0)
    # the root cells under the child keep their neutral fraction; the others near the source ionise
    assert np.all(xs[0][10:14, 10:14, 10:14] == 0.5)
    assert xs[0][0, 0, 0] < 0.5
