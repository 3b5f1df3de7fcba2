"""Comparison helpers shared by the GPU parity tests (no GPU needed to import).

Bars (derived in the design notes from the arithmetic of each path):
* k_ph and heating per cell: relative error <= 1e-4 wherever the oracle's
  value exceeds 1e-6 of its maximum in mixed precision, <= 1e-9 in float64
  (the same expressions in the same order up to atomic summation order and
  libm ulps); below that floor the absolute error is held to the same bar
  times the maximum.
* Photon conservation absorbed + escaped + truncated = emitted to 1e-9.
* The ray ledger seeded + 4 splits = splits + escaped + truncated exactly.
* Ray counts equal the oracle's in float64; in mixed precision they may
  differ only through near-ties of cell corners (1e-5 relative) and flipped
  split decisions (three rays per flip).
"""
import numpy as np
import pytest


def np_(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def field_err(got, want, floor=1e-6):
    """(max relative error over cells above floor * max, max absolute error / max)."""
    got, want = np_(got).ravel(), np.asarray(want).ravel()
    mx = want.max()
    if mx == 0.0:
        return 0.0, float(np.abs(got).max())
    m = want > floor * mx
    rel = float(np.max(np.abs(got[m] - want[m]) / want[m])) if m.any() else 0.0
    absr = float(np.max(np.abs(got - want)) / mx)
    return rel, absr


def check(res, ref, rel_tol, name="", fp64=False, count_rtol=1e-5, conserving=True):
    """Hold one GPU result to the oracle's: fields per cell, totals, ledger and
    counts. Returns the worst relative field error. count_rtol bounds the
    relative difference of the mixed-precision counts (near-ties). With the
    covering factor (conserving=False) the absorbed total is scaled cell by
    cell and no longer balances the photons emitted; it is held to the
    oracle's instead."""
    T = ref["totals"]
    worst = 0.0
    for q in range(len(ref["k_ph"])):
        for f in ("k_ph", "heating"):
            rel, absr = field_err(res[f][q], ref[f][q])
            worst = max(worst, rel)
            print(f"[{name}] grid {q} {f}: max rel {rel:.3e} (cells > 1e-6 max), max abs/max {absr:.3e}", flush=True)
            assert rel <= rel_tol, (name, q, f, rel)
            assert absr <= max(rel_tol, 1e-6), (name, q, f, absr)
    bal = res["absorbed"] + res["escaped"] + res["truncated"] - res["emitted"]
    print(f"[{name}] conservation {bal / res['emitted']:.3e}; segments gpu {res['segments']} oracle {T['segments']}; "
          f"splits {res['splits']}/{T['splits']}", flush=True)
    if conserving:
        assert abs(bal) <= 1e-9 * res["emitted"]
    else:
        assert res["absorbed"] == pytest.approx(T["absorbed"], rel=max(rel_tol, 1e-12), abs=1e-12 * T["emitted"])
    assert res["emitted"] == pytest.approx(T["emitted"], rel=1e-14)
    assert res["rays_seeded"] + 4 * res["splits"] == res["splits"] + res["rays_escaped"] + res["rays_truncated"]
    assert res["escaped"] == pytest.approx(T["escaped"], rel=max(rel_tol, 1e-12), abs=1e-12 * T["emitted"])
    flips = abs(res["splits"] - T["splits"])
    for k in ("segments", "splits", "rays_escaped", "rays_truncated"):
        if fp64:
            assert res[k] == T[k], (k, res[k], T[k])
        else:
            # one flipped split decision turns one ray into four
            assert abs(res[k] - T[k]) <= count_rtol * T[k] + 2 + 3 * flips, (k, res[k], T[k])
    return worst


def inverse_square_deviation(k_ph, problem, r_min=4.0):
    """k_ph / k_exact - 1 over the root cells whose centres lie farther than
    r_min cells from the problem's one source, where k_exact =
    sigma Ndot e^{-kappa r} / (4 pi r^2) is the rate of an unsplit point source
    in a uniform medium (Eqs. flux and kph with the column kappa r of a
    uniform medium). The angular-resolution test takes the standard deviation
    of this field."""
    import math
    g = problem.grids[0]
    n_h, x_hi = float(np.asarray(g.n_h).flat[0]), float(np.asarray(g.x_hi).flat[0])
    nz, ny, nx = np.asarray(g.n_h).shape
    sx, sy, sz, ndot = (float(v) for v in problem.sources[0])
    sigma = float(problem.spectrum.sigma_cm2[0])
    kappa = sigma * n_h * x_hi * g.dx_cm
    R = np.sqrt(((np.arange(nx) + 0.5) - sx)[None, None, :] ** 2 + ((np.arange(ny) + 0.5) - sy)[None, :, None] ** 2 +
                ((np.arange(nz) + 0.5) - sz)[:, None, None] ** 2)
    m = R > r_min
    want = sigma * ndot * np.exp(-kappa * R[m]) / (4.0 * math.pi * (R[m] * g.dx_cm) ** 2)
    return np_(k_ph).reshape(nz, ny, nx)[m] / want - 1.0
