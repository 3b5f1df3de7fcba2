"""Pins of the oracle's covering-factor correction (section 2.3, Eqs.
midpoint and fc), none of which re-types the oracle's formula:

* Closed form on axis rays. With phi_c = 0 the level-0 base pixels 4 and 6
  point along +x and -x, and a source at a cell centre sends them through
  the centres of the cells on its row: the k-th cell's segment starts at
  R_0 = k - 1/2 and its midpoint is the cell centre, so D_edge = 1/2 and
  f_c = min(1, (1/2 + (1/2) / ((k - 1/2) sqrt(pi/3)))^2) (theta_pix =
  sqrt(4 pi / 12)). A source moved by delta across the row (along y) keeps
  the midpoints delta off the centres: D_edge = 1/2 - delta. No other seed
  ray reaches those cells, so k_ph(corrected) / k_ph(plain) equals f_c.
* Invariants: the correction leaves the attenuation alone, so escaped and
  truncated photons, segments and ray counts are unchanged; per cell the
  corrected rate is between a quarter and all of the plain one.
* The paper's purpose for it: in the optically thin test the corrected k_ph
  scatters less about sigma Ndot e^-tau / (4 pi r^2) than the plain one at low
  phi_c (section 8.1, the improvements from the covering factor).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W

THETA0 = math.sqrt(4.0 * math.pi / 12.0)


def _axis_problem(delta, covering, n=17):
    g = W.uniform_grid(n, W.DX_C1, 1e-3, 1.0)
    c = n // 2 + 0.5
    src = np.array([[c, c + delta, c, 1e48]])
    params = W.Params(phi_c=0.0, level_init=0, level_max=0, p_min_frac=0.0, covering=covering)
    return W.Problem([g], src, W.hydrogen_spectrum([13.6]), params)


@pytest.mark.parametrize("delta", [0.0, 0.2, -0.35])
def test_axis_rays_follow_the_closed_form(delta):
    plain = O.trace(_axis_problem(delta, False))["k_ph"][0]
    cov = O.trace(_axis_problem(delta, True))["k_ph"][0]
    n = plain.shape[0]
    i0 = n // 2
    j = i0 + (1 if delta >= 0.5 else 0)
    for k in range(2, n // 2):
        for sgn in (1, -1):                       # the +x and -x rays
            i = i0 + sgn * k
            want = min(1.0, (0.5 + (0.5 - abs(delta)) / ((k - 0.5) * THETA0)) ** 2)
            got = cov[i0, j, i] / plain[i0, j, i]
            assert got == pytest.approx(want, rel=1e-12, abs=0.0), (delta, k, sgn)


def test_correction_leaves_the_attenuation_alone():
    base = W.lognormal_problem(98, 3, 20, 2, params=W.Params(phi_c=2.0, level_init=1))
    on = W.lognormal_problem(98, 3, 20, 2, params=W.Params(phi_c=2.0, level_init=1, covering=True))
    a, b = O.trace(base), O.trace(on)
    for key in ("segments", "splits", "rays_seeded", "rays_escaped", "rays_truncated"):
        assert a["totals"][key] == b["totals"][key], key
    for key in ("escaped", "truncated", "emitted"):
        assert b["totals"][key] == pytest.approx(a["totals"][key], rel=1e-13), key
    ka, kb = a["k_ph"][0], b["k_ph"][0]
    m = ka > 0
    ratio = kb[m] / ka[m]
    assert np.all(ratio <= 1.0 + 1e-12) and np.all(ratio >= 0.25 - 1e-12)
    assert np.all(kb[~m] == 0)
    assert b["totals"]["absorbed"] < a["totals"]["absorbed"]      # no longer photon-conserving


def _thin_scatter(phi_c, covering, n=32):
    box = 6.6 * W.KPC_CM
    g = W.uniform_grid(n, box / n, 1e-3, 1e-4)
    s = np.array([0.5, 0.5, 0.5])
    p = W.Problem([g], np.array([[*s, 5e48]]), W.hydrogen_spectrum([13.6]),
                  W.Params(phi_c=phi_c, level_init=1, level_max=14, p_min_frac=1e-8, covering=covering))
    k = O.trace(p)["k_ph"][0]
    sigma = p.spectrum.sigma_cm2[0]
    kappa = sigma * 1e-3 * 1e-4 * g.dx_cm
    ax = np.arange(n) + 0.5
    R = np.sqrt((ax[None, None, :] - s[0]) ** 2 + (ax[None, :, None] - s[1]) ** 2 + (ax[:, None, None] - s[2]) ** 2)
    m = R > 4.0
    want = sigma * 5e48 * np.exp(-kappa * R[m]) / (4.0 * math.pi * (R[m] * g.dx_cm) ** 2)
    return float(np.std(k[m] / want - 1.0))


@pytest.mark.parametrize("phi_c", [1.0, 2.0])
def test_correction_reduces_the_anisotropy_of_thin_rays(phi_c):
    plain, cov = _thin_scatter(phi_c, False), _thin_scatter(phi_c, True)
    print(f"phi_c {phi_c}: scatter plain {plain:.3f}, corrected {cov:.3f}")
    assert cov < plain
