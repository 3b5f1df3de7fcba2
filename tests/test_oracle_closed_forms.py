"""Closed-form pins of the oracle (section 2.2, Eqs. dtau, flux, kph, gamma;
section 2.1 termination rules).

* Axis rays: the four equatorial base pixels point exactly along +-x and +-y,
  so with no splitting a source at a cell centre sends one ray down each grid
  row; its deposits are the Beer-Lambert series P0 e^{-tau_c (k-1/2)} (1 - e^{-tau_c}).
* Escape: with no splitting every seed ray leaves the box with
  P0 exp(-kappa L_p), L_p the distance from the source to the box along it.
* Truncation radius: in a uniform medium a ray is dropped once
  P < 1e-8 P0, i.e. once its path optical depth exceeds ln(1e8), whatever its
  level; nothing is deposited beyond that radius.
* Heating: for one group the heating rate is k_ph (E - E_ion) per absorber.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W

EV = 1.602176634e-12


def _uniform(n, kappa_cell, src, energies=(13.6,), params=None, x_hi=0.75):
    dx = W.DX_C1
    sigma0 = W.hydrogen_spectrum(energies).sigma_cm2[0]
    n_h = kappa_cell / (sigma0 * x_hi * dx)
    g = W.uniform_grid(n, dx, n_h, x_hi)
    return W.Problem([g], np.array([src], dtype=np.float64), W.hydrogen_spectrum(energies),
                     params or W.Params(phi_c=0.0, level_init=0, level_max=14, p_min_frac=0.0))


def test_axis_rays_beer_lambert_series():
    n = 16
    p = _uniform(n, 0.3, [8.5, 8.5, 8.5, 1.2e49])
    g = p.grids[0]
    tau_c = p.spectrum.sigma_cm2[0] * float(g.n_h[0, 0, 0]) * float(g.x_hi[0, 0, 0]) * g.dx_cm
    res = O.trace(p)
    A = res["absorbed"][0]
    P0 = 1.2e49 / 12
    ks = np.arange(1, n - 8)
    want = P0 * np.exp(-tau_c * (ks - 0.5)) * -np.expm1(-tau_c)
    for sgn in (+1, -1):
        got_x = np.array([A[8, 8, 8 + sgn * k] for k in ks])
        got_y = np.array([A[8, 8 + sgn * k, 8] for k in ks])
        np.testing.assert_allclose(got_x, want, rtol=1e-13)
        np.testing.assert_allclose(got_y, want, rtol=1e-13)
    # source cell: four axis rays cross half a cell, eight z=+-2/3 rays leave
    # through a z face after 0.5/(2/3) = 0.75 cells
    want_src = 4 * P0 * -math.expm1(-0.5 * tau_c) + 8 * P0 * -math.expm1(-0.75 * tau_c)
    assert A[8, 8, 8] == pytest.approx(want_src, rel=1e-13)


@pytest.mark.parametrize("level", [1, 2])
def test_escape_totals_closed_form(level):
    n = 16
    s = np.array([5.25, 9.5, 7.0009765625])
    p = _uniform(n, 0.4, list(s) + [1e49],
                 params=W.Params(phi_c=0.0, level_init=level, level_max=14, p_min_frac=1e-8))
    g = p.grids[0]
    kappa = p.spectrum.sigma_cm2[0] * float(g.n_h[0, 0, 0]) * float(g.x_hi[0, 0, 0]) * g.dx_cm
    res = O.trace(p)
    npix = 12 * 4 ** level
    P0 = 1e49 / npix
    tot = 0.0
    for pix in range(npix):
        v = O.pix2vec(level, pix)
        L = min(((n if v[a] > 0 else 0.0) - s[a]) / v[a] for a in range(3) if v[a] != 0.0)
        tot += P0 * math.exp(-kappa * L)
    assert res["totals"]["truncated"] == 0.0
    assert res["escaped_sg"][0, 0] == pytest.approx(tot, rel=1e-12)
    assert res["totals"]["rays_escaped"] == npix


def test_truncation_radius_is_level_independent():
    # kappa = 1 per cell: rays end after an optical depth of ln(1e8) = 18.42 cells
    n = 48
    s = [24.5, 24.5, 24.5, 1e50]
    p = _uniform(n, 1.0, s, params=W.Params(phi_c=5.1, level_init=1, level_max=14, p_min_frac=1e-8))
    res = O.trace(p)
    A = res["absorbed"][0]
    ax = np.arange(n) + 0.5
    R = np.sqrt((ax[None, None, :] - s[0]) ** 2 + (ax[None, :, None] - s[1]) ** 2 + (ax[:, None, None] - s[2]) ** 2)
    r_end = math.log(1e8)
    assert np.all(A[R > r_end + 1.0] == 0.0)             # nothing beyond (cell half-diagonal 0.87)
    assert np.all(A[R < r_end - 1.0] > 0.0)              # everything inside receives photons
    T = res["totals"]
    assert T["escaped"] == 0.0 and T["rays_escaped"] == 0
    assert 0.0 < T["truncated"] <= 1e-8 * T["emitted"]


def test_heating_is_kph_times_excess_energy():
    p = _uniform(12, 0.5, [6.25, 5.5, 6.75, 1e49], energies=(30.0,),
                 params=W.Params(phi_c=5.1, level_init=1, level_max=14, p_min_frac=1e-8))
    res = O.trace(p)
    k, h = res["k_ph"][0], res["heating"][0]
    m = k > 0
    assert m.sum() > 1000
    np.testing.assert_allclose(h[m] / k[m], (30.0 - 13.6) * EV, rtol=1e-14)
    # k_ph is the absorbed rate per absorber: absorbed / (n_H x_HI V)
    g = p.grids[0]
    nabs = g.n_h.astype(np.float64) * g.x_hi.astype(np.float64)
    np.testing.assert_allclose(k * nabs * g.dx_cm ** 3, res["absorbed"][0], rtol=1e-14)


def test_no_absorber_cells_get_no_photons():
    p = _uniform(10, 0.5, [5.5, 5.5, 5.5, 1e49], params=W.Params(phi_c=2.0, level_init=1, level_max=14, p_min_frac=1e-8))
    g = p.grids[0]
    g.x_hi = g.x_hi.copy()
    g.x_hi[:, :, 7] = 0.0                  # a fully ionised slab
    res = O.trace(p)
    assert np.all(res["absorbed"][0][:, :, 7] == 0.0)
    assert np.all(res["k_ph"][0][:, :, 7] == 0.0)
    assert np.all(res["absorbed"][0][:, :, 8] > 0.0)   # photons pass through it
