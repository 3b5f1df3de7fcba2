"""Photo-ionisation equilibrium iteration around the oracle (Stromgren pin).

TEST INFRASTRUCTURE ONLY: used by the tests to pin the oracle's k_ph
normalisation against the Stromgren radius; never called by the product path.

Hydrogen-only rate equation (section 2.2, Eq. dndt) at dn/dt = 0 with no
collisional term and n_e = n_p = (1 - x) n_H for neutral fraction x:

    alpha_B n_H (1 - x)^2 = k_ph x,

alpha_B = 2.59e-13 cm^3/s (case B at 1e4 K, section 2.2). The iteration
traces, solves that quadratic per cell, damps x <- (x + x_new)/2 and repeats
until max |dx| < tol.
"""
from __future__ import annotations

import copy

import numpy as np

from . import oracle as _oracle

ALPHA_B = 2.59e-13   # cm^3 s^-1, case-B recombination coefficient at 1e4 K


def equilibrium_x(k_ph: np.ndarray, n_h: np.ndarray, alpha_b: float = ALPHA_B) -> np.ndarray:
    """Root in [0, 1] of alpha n (1-x)^2 = k x, written without cancellation:
    x = 2a / ((2a + k) + sqrt(k^2 + 4 a k)) with a = alpha n."""
    a = alpha_b * np.asarray(n_h, dtype=np.float64)
    k = np.asarray(k_ph, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        x = 2.0 * a / ((2.0 * a + k) + np.sqrt(k * k + 4.0 * a * k))
    return np.where(a > 0.0, x, 1.0)


def covered_root_cells(problem) -> np.ndarray:
    """Root cells that a child grid covers (their radiation field lives in the
    child; they keep their neutral fraction in the updates)."""
    root = problem.grids[0]
    mask = np.zeros(np.asarray(root.n_h).shape, dtype=bool)
    for g in problem.grids[1:]:
        ox, oy, oz = (int(v) for v in g.offset)
        nz, ny, nx = np.asarray(g.n_h).shape
        mask[oz:oz + nz // 2, oy:oy + ny // 2, ox:ox + nx // 2] = True
    return mask


def iterate(problem, tol: float = 1e-6, max_iter: int = 300, damping: float = 0.5, n_threads: int = 1):
    """Damped fixed-point iteration to ionisation equilibrium, from neutral
    gas, over every grid of the problem (covered root cells excluded).

    Returns (x_final, last oracle result, iterations used): x_final is a
    float64 array for a single grid, else a list of arrays, one per grid."""
    p = copy.copy(problem)
    p.grids = [copy.copy(g) for g in problem.grids]
    covered = covered_root_cells(problem)
    xs = [np.ones(np.asarray(g.n_h).shape) for g in p.grids]
    res = None
    done = max_iter
    for it in range(1, max_iter + 1):
        for g, x in zip(p.grids, xs):
            g.x_hi = x.astype(np.float32)
        res = _oracle.trace(p, n_threads=n_threads)
        dx = 0.0
        for q, g in enumerate(p.grids):
            x_new = equilibrium_x(res["k_ph"][q], g.n_h)
            x_next = (1.0 - damping) * xs[q] + damping * x_new
            if q == 0:
                x_next[covered] = xs[0][covered]
            dx = max(dx, float(np.max(np.abs(x_next - xs[q]))))
            xs[q] = x_next
        if dx < tol:
            done = it
            for g, x in zip(p.grids, xs):
                g.x_hi = x.astype(np.float32)
            res = _oracle.trace(p, n_threads=n_threads)
            break
    else:
        for g, x in zip(p.grids, xs):
            g.x_hi = x.astype(np.float32)
    return (xs[0] if len(xs) == 1 else xs), res, done
