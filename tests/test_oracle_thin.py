"""Pins of the oracle's optically-thin approximation (section 2.4, Eq.
optthin, the per-source marker field), none of which re-types the oracle's
arithmetic:

* The thin field is the inverse-square law. In a medium too thin to matter
  every cell away from the source gets sigma Ndot / (4 pi r^2) from each
  (source, group), exactly once, whatever ray reached it first (the paper:
  the field strictly follows 1/r^2 inside the thin radius, section 8.2):
  checked against the closed form for two groups and two sources, with the
  heating k (E - E_ion), and with the rate unchanged by the seed level.
* Thin rays are split against one ray per cell (phi = min(1, phi_c)) and
  remove no photons: an all-thin trace at phi_c = 5.1 walks the same ray
  tree as the general trace at phi_c = 1 and lets every photon escape.
* A vanishing tau_thin leaves the general trace bit for bit.
* In a uniform medium the optical depth from the source is sigma n dx r on
  every ray, so the thin-or-thick decision is r_exit < R_thin = tau_thin /
  (sigma n dx): cells wholly inside R_thin remove no photons and hold the
  closed form, cells wholly outside it get no thin rate.
* Along an axis ray the decision takes the optical depth where the ray
  leaves the cell: the first thick cell is the one it leaves beyond
  tau_thin, and it and the cells after it hold the general deposits of the
  undiminished ray.
* The cell that holds a source at its centre takes the general deposit of
  the seed rays, computed here from the pixel directions and the cell's
  faces.
* Two coincident sources double the rate (one mark per source), and the
  approximation saves ray segments in an ionised medium, its purpose.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W

DX = W.DX_C1


def _problem(n, n_h, sources, energies=(13.6,), tau_thin=1e300, phi_c=5.1, level_init=1, p_min=0.0, x_hi=1.0):
    g = W.uniform_grid(n, DX, n_h, x_hi)
    return W.Problem([g], np.asarray(sources, float), W.hydrogen_spectrum(list(energies)),
                     W.Params(phi_c=phi_c, level_init=level_init, level_max=14, p_min_frac=p_min, tau_thin=tau_thin))


def _centres(n):
    z, y, x = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    return x, y, z


def _holding(n, s):
    """cells whose closed box [c, c+1]^3 contains the point s"""
    x, y, z = _centres(n)
    return ((x - 0.5 <= s[0]) & (s[0] <= x + 0.5) & (y - 0.5 <= s[1]) & (s[1] <= y + 0.5) &
            (z - 0.5 <= s[2]) & (s[2] <= z + 0.5))


def _inverse_square(n, sources, sp):
    """sum over sources and groups of sigma_g f_g Ndot / (4 pi r^2), and the
    heating sum k_g (E_g - E_ion); r from the source to the cell centre (cm)"""
    x, y, z = _centres(n)
    k = np.zeros((n, n, n))
    h = np.zeros((n, n, n))
    erg = O.ev_erg()
    for s in sources:
        r2 = ((x - s[0]) ** 2 + (y - s[1]) ** 2 + (z - s[2]) ** 2) * DX ** 2
        for sig, f, e in zip(sp.sigma_cm2, sp.frac, sp.energy_ev):
            kg = sig * f * s[3] / (4.0 * math.pi * r2)
            k += kg
            h += kg * (e - sp.e_ion_ev) * erg
    return k, h


@pytest.mark.parametrize("level_init", [0, 2])
def test_thin_field_is_the_inverse_square_law(level_init):
    n = 20
    srcs = [[7.3, 11.6, 9.15, 1e48], [12.5, 5.25, 14.0, 3e48]]
    p = _problem(n, 1e-9, srcs, energies=(13.6, 30.0), level_init=level_init)
    r = O.trace(p)
    k, h = r["k_ph"][0], r["heating"][0]
    want_k, want_h = _inverse_square(n, srcs, p.spectrum)
    away = ~(_holding(n, srcs[0]) | _holding(n, srcs[1]))
    # a cell missed by one item's thin rays lacks that item's rate; most are reached by all four
    full = np.isclose(k, want_k, rtol=1e-12, atol=0.0) & away
    assert full.sum() >= 0.97 * away.sum(), (full.sum(), away.sum())
    np.testing.assert_allclose(h[full], want_h[full], rtol=1e-12)
    # every cell's rate is a sum of whole per-item terms: never above the closed form
    assert np.all(k[away] <= want_k[away] * (1 + 1e-12))
    T = r["totals"]
    assert T["absorbed"] == 0.0 and T["escaped"] == pytest.approx(T["emitted"], rel=1e-13)
    assert T["thin_segments"] == T["segments"] and T["thin_marked"] <= 4 * n ** 3


def test_the_rate_does_not_depend_on_the_seed_level():
    n = 16
    srcs = [[5.6, 9.3, 7.8, 1e48]]
    a = O.trace(_problem(n, 1e-9, srcs, level_init=0))["k_ph"][0]
    b = O.trace(_problem(n, 1e-9, srcs, level_init=3))["k_ph"][0]
    both = (a > 0) & (b > 0) & ~_holding(n, srcs[0])
    assert both.sum() > 0.95 * n ** 3
    np.testing.assert_allclose(a[both], b[both], rtol=1e-13)


@pytest.mark.parametrize("phi_c,phi_general", [(5.1, 1.0), (0.5, 0.5)])
def test_thin_rays_split_against_one_ray_per_cell(phi_c, phi_general):
    n = 18
    srcs = [[6.7, 8.2, 9.9, 1e48]]
    thin = O.trace(_problem(n, 1e-6, srcs, phi_c=phi_c))["totals"]
    gen = O.trace(_problem(n, 1e-6, srcs, tau_thin=0.0, phi_c=phi_general))["totals"]
    for key in ("segments", "splits", "rays_seeded", "rays_escaped"):
        assert thin[key] == gen[key], key
    assert thin["absorbed"] == 0.0 and gen["absorbed"] > 0.0
    assert thin["escaped"] == pytest.approx(thin["emitted"], rel=1e-13)


def test_vanishing_tau_thin_is_the_general_trace():
    p = W.config0()
    ref = O.trace(p)
    p.params = W.Params(**{**p.params.__dict__, "tau_thin": 1e-300})
    got = O.trace(p)
    for f in ("k_ph", "heating", "absorbed"):
        for a, b in zip(got[f], ref[f]):
            assert np.array_equal(a, b), f
    for key in ("segments", "splits", "absorbed", "escaped", "truncated"):
        assert got["totals"][key] == ref["totals"][key], key
    assert got["totals"]["thin_segments"] == 0 and got["totals"]["thin_marked"] == 0


def test_uniform_medium_switches_at_the_thin_radius():
    n, n_h, tau_thin = 24, 4.7e-5, 0.1
    sig = W.hydrogen_spectrum([13.6]).sigma_cm2[0]
    r_thin = tau_thin / (sig * n_h * DX)              # root cells
    assert 5.0 < r_thin < 9.0
    s = [11.37, 12.61, 11.92, 1e49]
    r = O.trace(_problem(n, n_h, [s], tau_thin=tau_thin, p_min=1e-8))
    x, y, z = _centres(n)
    d = np.stack([x - s[0], y - s[1], z - s[2]])
    far = np.sqrt(((np.abs(d) + 0.5) ** 2).sum(0))                  # farthest point of the cell
    near = np.sqrt((np.maximum(np.abs(d) - 0.5, 0.0) ** 2).sum(0))  # nearest point
    hold = _holding(n, s)
    inner = (far < r_thin * (1 - 1e-9)) & ~hold
    outer = near > r_thin * (1 + 1e-9)
    absorbed, k = r["absorbed"][0], r["k_ph"][0]
    want_k, _ = _inverse_square(n, [s], W.hydrogen_spectrum([13.6]))
    assert inner.sum() > 300 and outer.sum() > 5000
    assert np.all(absorbed[inner | hold] == 0.0)
    reached = inner & (k > 0)
    assert reached.sum() >= 0.97 * inner.sum()
    np.testing.assert_allclose(k[reached], want_k[reached], rtol=1e-12)
    vol = DX ** 3
    lit = outer & (absorbed > 0)
    assert lit.sum() > 0.9 * outer.sum()
    nab = float(np.float32(n_h))                      # the field is float32
    np.testing.assert_allclose(k[outer], absorbed[outer] / (nab * vol), rtol=1e-13)
    T = r["totals"]
    bal = T["emitted"] - T["absorbed"] - T["escaped"] - T["truncated"]
    assert abs(bal) <= 1e-12 * T["emitted"]
    assert 0.0 < T["thin_margin"] < 1.0


def test_axis_ray_turns_thick_in_the_cell_it_leaves_beyond_tau_thin():
    # level 0, no splits: base pixel 4 points along +x; from a source at a
    # cell centre it leaves the k-th cell of its row at r = k + 1/2, where its
    # optical depth is a (k + 1/2) with a = sigma n dx. With tau_thin = 3 a the
    # cells k = 1, 2 are thin (closed form), the cell k = 3 (entered at 2.5 <
    # 3, left at 3.5) is the first thick one and takes the undiminished
    # P0 (1 - e^-a), the next ones P0 e^-(k-3) a (1 - e^-a).
    assert np.allclose(O.pix2vec(0, 4), [1.0, 0.0, 0.0], atol=1e-15)
    n, n_h = 15, 1e-3
    nab = float(np.float32(n_h))
    sig = W.hydrogen_spectrum([13.6]).sigma_cm2[0]
    a = sig * nab * DX
    s = [4.5, 7.5, 7.5, 1e49]
    r = O.trace(_problem(n, n_h, [s], tau_thin=3.0 * a, level_init=0, phi_c=0.0))
    k = r["k_ph"][0][7, 7, :]
    P0 = s[3] / 12.0
    vol = DX ** 3
    for kk in (1, 2):
        assert k[4 + kk] == pytest.approx(sig * P0 / ((4.0 * math.pi / 12.0) * (kk * DX) ** 2), rel=1e-13)
    for kk in range(3, 10):
        want = P0 * math.exp(-(kk - 3) * a) * -math.expm1(-a) / (nab * vol)
        assert k[4 + kk] == pytest.approx(want, rel=1e-12), kk


def test_cell_holding_a_centred_source_takes_the_seed_deposit():
    n, n_h = 9, 3e-3
    nab = float(np.float32(n_h))
    s = [4.5, 4.5, 4.5, 1e49]
    sp = W.hydrogen_spectrum([13.6])
    r = O.trace(_problem(n, n_h, [s], tau_thin=1.0, level_init=1, phi_c=0.0))   # no splits: only seeds
    P0 = s[3] / 48.0
    tot = 0.0
    for pix in range(48):
        v = O.pix2vec(1, pix)
        t = min((((4 + (1 if v[a] > 0 else 0)) - s[a]) / v[a]) for a in range(3) if v[a] != 0.0)
        tot += P0 * -math.expm1(-sp.sigma_cm2[0] * nab * t * DX)
    assert r["k_ph"][0][4, 4, 4] == pytest.approx(tot / (nab * DX ** 3), rel=1e-13)
    assert r["absorbed"][0][4, 4, 4] == 0.0


def test_each_source_sets_its_own_marks():
    n = 14
    one = [[6.3, 7.1, 5.9, 2e48]]
    two = [[6.3, 7.1, 5.9, 1e48], [6.3, 7.1, 5.9, 1e48]]
    a = O.trace(_problem(n, 1e-9, one))
    b = O.trace(_problem(n, 1e-9, two))
    away = ~_holding(n, one[0])
    np.testing.assert_allclose(b["k_ph"][0][away], a["k_ph"][0][away], rtol=1e-13)
    assert b["totals"]["thin_marked"] == 2 * a["totals"]["thin_marked"]


def test_the_approximation_saves_segments_in_ionised_gas():
    p = W.config0()
    ion = W.Problem([W.Grid(g.n_h, np.full_like(g.x_hi, 1e-4), g.dx_cm, g.parent, g.offset) for g in p.grids],
                    p.sources, p.spectrum, p.params)
    gen = O.trace(ion)["totals"]
    ion.params = W.Params(**{**p.params.__dict__, "tau_thin": 0.1})
    thin = O.trace(ion)["totals"]
    assert thin["segments"] < 0.5 * gen["segments"], (thin["segments"], gen["segments"])
    assert thin["thin_segments"] > 0.5 * thin["segments"]


def test_invalid_and_unsupported_uses_are_rejected():
    p = W.config0()
    for bad in (-0.1, float("nan"), float("inf")):
        p.params = W.Params(**{**W.config0().params.__dict__, "tau_thin": bad})
        with pytest.raises(O.OracleError):
            O.trace(p)
    p.params = W.Params(**{**W.config0().params.__dict__, "tau_thin": 0.1})
    with pytest.raises(O.OracleError):
        O.trace(p, want_accel=True)
    with pytest.raises(O.OracleError):
        O.trace_td(p, 4.0)
