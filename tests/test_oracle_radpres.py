"""Pins of the oracle's radiation-pressure acceleration (section 2.5.4, Eq.
radpres: absorbed photons hand dP E_ph / c along their ray to the cell; the
gas gains a = dp / (rho V), rho = m_H n_H), none of which re-types its sum:

* Axis rays: with phi_c = 0 the level-0 pixels 4 and 6 run along +x and -x
  through the centres of the cells of the source's row, and no other ray
  reaches those cells; there the acceleration is along x, with the ray's
  sign, and equals k_ph x_HI E / (c m_H) (the same dP seen through Eq. kph).
* Mirror symmetry: a source on the centre vertex of a uniform box gives an
  acceleration field odd in x under the x mirror and even in y and z, bit for
  bit from 2.5 cells out, and pushes every lit cell outward.
* Scalings that expose dropped or misplaced factors: twice the photon energy
  gives exactly twice the acceleration; twice n_H at half x_HI (the same
  absorber column, so the same dP) gives exactly half.
* The covering factor (section 2.3) leaves it unchanged: it scales k_ph and
  heating, not the absorbed radiation.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W

C_CMS = 2.99792458e10
M_H = 1.6735575e-24


def _axis_problem(n=17, energy=13.6, covering=False):
    g = W.uniform_grid(n, W.DX_C1, 1e-3, 1.0)
    c = n // 2 + 0.5
    src = np.array([[c, c, c, 1e48]])
    return W.Problem([g], src, W.hydrogen_spectrum([energy]),
                     W.Params(phi_c=0.0, level_init=0, level_max=0, p_min_frac=0.0, covering=covering))


def test_axis_rays_push_along_the_ray():
    p = _axis_problem(energy=20.0)
    r = O.trace(p, want_accel=True)
    a, k = r["accel"][0], r["k_ph"][0]
    x = p.grids[0].x_hi.astype(np.float64)
    e_erg = 20.0 * O.ev_erg()
    n = k.shape[0]
    i0 = n // 2
    for d in range(2, n // 2):
        for sgn in (1, -1):
            i = i0 + sgn * d
            want = sgn * k[i0, i0, i] * x[i0, i0, i] * e_erg / (C_CMS * M_H)
            assert a[0, i0, i0, i] == pytest.approx(want, rel=1e-12), (d, sgn)
            assert abs(a[1, i0, i0, i]) <= 1e-12 * abs(want)
            assert abs(a[2, i0, i0, i]) <= 1e-12 * abs(want)


def test_mirror_symmetry_of_a_centred_source():
    a = O.trace(W.config0(), want_accel=True)["accel"][0]
    n = a.shape[1]
    ax = np.arange(n) + 0.5 - 16.0
    rz, ry, rx = np.meshgrid(ax, ax, ax, indexing="ij")
    # the rays that start on the planes through the source vertex take their
    # first cell by the tie rule (upper cell for a zero component), which is
    # not mirror-symmetric, and those few cells pass it on to their
    # neighbours; from 2.5 cells out the field is mirror-symmetric bit for bit
    near = np.sqrt(rx ** 2 + ry ** 2 + rz ** 2) < 2.5
    assert np.abs(a).max() > 0
    m = a[:, :, :, ::-1]                                  # mirror x
    assert np.array_equal(a[0][~near], -m[0][~near])
    assert np.array_equal(a[1][~near], m[1][~near])
    assert np.array_equal(a[2][~near], m[2][~near])
    scale = np.abs(a).max()
    # every cell away from the source is pushed outward
    far = np.sqrt(rx ** 2 + ry ** 2 + rz ** 2) > 3.0
    radial = a[0] * rx + a[1] * ry + a[2] * rz
    lit = np.linalg.norm(a, axis=0) > 1e-9 * scale
    assert np.all(radial[far & lit] > 0.0)


def test_energy_and_density_scalings_are_exact():
    base = W.lognormal_problem(93, 1, 20, 2)
    a1 = O.trace(base, want_accel=True)["accel"][0]
    twice_e = W.lognormal_problem(93, 1, 20, 2)
    sp = twice_e.spectrum
    twice_e.spectrum = W.Spectrum(energy_ev=2.0 * np.asarray(sp.energy_ev), sigma_cm2=sp.sigma_cm2, frac=sp.frac,
                                  e_ion_ev=sp.e_ion_ev)
    a2 = O.trace(twice_e, want_accel=True)["accel"][0]
    assert np.array_equal(a2, 2.0 * a1)
    dens = W.lognormal_problem(93, 1, 20, 2)
    g = dens.grids[0]
    g.n_h = (2.0 * g.n_h).astype(np.float32)
    g.x_hi = (0.5 * g.x_hi).astype(np.float32)
    a3 = O.trace(dens, want_accel=True)["accel"][0]
    assert np.array_equal(a3, 0.5 * a1)


def test_covering_factor_leaves_the_acceleration_alone():
    plain = O.trace(_axis_problem(), want_accel=True)["accel"][0]
    cov = O.trace(_axis_problem(covering=True), want_accel=True)["accel"][0]
    assert np.array_equal(plain, cov)
