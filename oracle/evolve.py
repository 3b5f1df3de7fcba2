"""Time-stepped photo-ionisation around the oracle trace.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark check the GPU
library's time stepping against this; the product path never imports it.

The cycle of section 3.1 with its chemistry step (step 6) reduced to the
hydrogen-only rate equation of section 2.2 (Eq. dndt) with no collisional
term, n_e = n_p = (1 - x) n_H for neutral fraction x, held k_ph over the step:

    dx/dt = a (1 - x)^2 - k x,     a = alpha_B n_H, k = k_ph,

and the radiative-transfer timestep of section 3.4.1:

* per cell dt_cell = eps / (k + n_e alpha_B) (Eq. dtelec, C_H = 0), only in
  cells of the ionisation front, read as cells whose own optical depth
  tau_cell = sigma_bar n_H x dx exceeds tau_front (0.5), sigma_bar the
  photon-weighted cross-section of the spectrum; every other cell, and every
  cell whose limit exceeds it, takes dt_max (the step the caller would take
  without radiation);
* the field of dt_cell is smoothed over 3^3 cells with the binomial
  (1, 2, 1)/4 weights per axis, normalised over the neighbours inside the
  grid;
* dt = min over cells of the smoothed field, at most twice the previous step
  (Eq. dtchange), at most dt_max and the time left.

Every cell then advances by the exact solution of the rate equation over dt
(advance below). One trace per step; a last trace with the final x.
"""
from __future__ import annotations

import copy

import numpy as np

from . import oracle as _oracle
from .equilibrium import ALPHA_B, covered_root_cells, equilibrium_x


def advance(x0, k_ph, n_h, dt, alpha_b: float = ALPHA_B):
    """Exact solution of dx/dt = a (1-x)^2 - k x at time dt from x0, a and k
    held. With x1 the root in [0, 1] of the right-hand side and
    D = sqrt(k^2 + 4ak) = a (x2 - x1), u = x - x1 obeys the Bernoulli
    equation du/dt = a u^2 - D u, whose solution is

        u(dt) = u0 e^{-D dt} / (1 - a u0 g),   g = (1 - e^{-D dt}) / D

    (g = dt at D = 0, where x1 = 1). Cells without gas (a = 0) keep x."""
    x0 = np.asarray(x0, dtype=np.float64)
    a = alpha_b * np.asarray(n_h, dtype=np.float64)
    k = np.asarray(k_ph, dtype=np.float64)
    x1 = equilibrium_x(k, n_h, alpha_b)
    d = np.sqrt(k * k + 4.0 * a * k)
    dtv = np.broadcast_to(np.asarray(dt, dtype=np.float64), x0.shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(d > 0.0, -np.expm1(-d * dtv) / d, dtv)
    u0 = x0 - x1
    u = u0 * np.exp(-d * dtv) / (1.0 - a * u0 * g)
    x = np.clip(x1 + u, 0.0, 1.0)
    return np.where(a > 0.0, x, x0)


def smooth3(f):
    """Normalised 3^3 binomial smoothing: weights w(i) w(j) w(k) with
    w(0) = 1/2, w(+-1) = 1/4, summed over the neighbours inside the grid and
    divided by the sum of their weights. Plain loops over the 27 offsets."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    w1 = {-1: 0.25, 0: 0.5, 1: 0.25}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                w = w1[dz] * w1[dy] * w1[dx]
                # target cells (z, y, x) whose neighbour (z+dz, y+dy, x+dx) is inside
                zs = slice(max(0, -dz), nz - max(0, dz))
                ys = slice(max(0, -dy), ny - max(0, dy))
                xs = slice(max(0, -dx), nx - max(0, dx))
                zn = slice(max(0, dz), nz - max(0, -dz))
                yn = slice(max(0, dy), ny - max(0, -dy))
                xn = slice(max(0, dx), nx - max(0, -dx))
                num[zs, ys, xs] += w * f[zn, yn, xn]
                den[zs, ys, xs] += w
    return num / den


def sigma_bar(spectrum) -> float:
    """Photon-weighted cross-section sum_g frac_g sigma_g (equal shares by default)."""
    sig = np.asarray(spectrum.sigma_cm2, dtype=np.float64)
    frac = getattr(spectrum, "frac", None)
    frac = np.full(sig.shape, 1.0 / sig.size) if frac is None else np.asarray(frac, dtype=np.float64)
    return float(np.sum(frac * sig))


def cell_limits(k_ph, x, n_h, dx_cm, sig_bar, eps, tau_front, dt_max, alpha_b: float = ALPHA_B):
    """dt_cell of Eq. dtelec in the front, dt_max elsewhere, at most dt_max."""
    x = np.asarray(x, dtype=np.float64)
    n = np.asarray(n_h, dtype=np.float64)
    k = np.asarray(k_ph, dtype=np.float64)
    rate = k + (1.0 - x) * n * alpha_b
    front = sig_bar * n * x * dx_cm > tau_front
    with np.errstate(divide="ignore"):
        lim = np.where(rate > 0.0, eps / rate, np.inf)
    return np.where(front, np.minimum(lim, dt_max), dt_max)


def next_dt(k_ph, x, n_h, dx_cm, sig_bar, eps, tau_front, dt_max, dt_prev, t_left, alpha_b: float = ALPHA_B):
    """The step of section 3.4.1 (module docstring); dt_prev None on the first step."""
    dt = float(np.min(smooth3(cell_limits(k_ph, x, n_h, dx_cm, sig_bar, eps, tau_front, dt_max, alpha_b))))
    if dt_prev is not None:
        dt = min(dt, 2.0 * dt_prev)
    return min(dt, dt_max, t_left)


def evolve(problem, t_end: float, eps: float = 0.1, tau_front: float = 0.5, dt_max: float | None = None,
           max_steps: int = 100000, alpha_b: float = ALPHA_B, x0=None, n_threads: int = 1):
    """Evolve a problem's neutral fraction from x0 (default: its x_hi; a
    list per grid when it has several) for t_end seconds. Every grid takes
    the same step: the smallest of its own smoothed limits (each grid smoothed
    on its own), covered root cells excluded (they take dt_max and keep their
    x). Returns (x, last trace result, steps, time reached, list of steps
    taken); x is a float64 array for a single grid, else a list per grid."""
    p = copy.copy(problem)
    p.grids = [copy.copy(g) for g in problem.grids]
    if dt_max is None:
        dt_max = t_end
    sb = sigma_bar(p.spectrum)
    covered = covered_root_cells(problem)
    if x0 is None:
        xs = [np.asarray(g.x_hi, dtype=np.float64).copy() for g in problem.grids]
    else:
        xs = [np.asarray(v, dtype=np.float64).copy() for v in (x0 if isinstance(x0, (list, tuple)) else [x0])]
    t, dt_prev, dts = 0.0, None, []
    while t < t_end and len(dts) < max_steps:
        for g, x in zip(p.grids, xs):
            g.x_hi = x.astype(np.float32)
        res = _oracle.trace(p, n_threads=n_threads)
        dt = np.inf
        for q, g in enumerate(p.grids):
            lim = cell_limits(res["k_ph"][q], xs[q], g.n_h, g.dx_cm, sb, eps, tau_front, dt_max, alpha_b)
            if q == 0:
                lim[covered] = dt_max
            dt = min(dt, float(np.min(smooth3(lim))))
        if dt_prev is not None:
            dt = min(dt, 2.0 * dt_prev)
        dt = min(dt, dt_max, t_end - t)
        for q, g in enumerate(p.grids):
            x_new = advance(xs[q], res["k_ph"][q], g.n_h, dt, alpha_b)
            if q == 0:
                x_new[covered] = xs[0][covered]
            xs[q] = x_new
        t += dt
        dt_prev = dt
        dts.append(dt)
    for g, x in zip(p.grids, xs):
        g.x_hi = x.astype(np.float32)
    res = _oracle.trace(p, n_threads=n_threads)
    return (xs[0] if len(xs) == 1 else xs), res, len(dts), t, dts

