"""Invariant pins of the oracle.

* Photon conservation: photo-ionisations equal absorptions (section 2.2), so
  absorbed + escaped + truncated = emitted, to 1e-12 relative.
* Ray ledger: each seed ray and each split child ends exactly once (escape or
  truncation) or splits, so seeded + 4 splits = splits + escaped + truncated.
* Mirror symmetry: the HEALPix pixel set is symmetric under x -> -x, y -> -y,
  z -> -z and x <-> y; a source at a cell centre in the middle of an odd,
  uniform box must give a k_ph field with the same symmetries.
* Linearity in the sources: fields of disjoint source sets add, and scaling
  every photon rate by 2^k scales every output by exactly 2^k (the truncation
  rule is relative to each ray's own share).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W


def _check_ledger(res, rel=1e-12):
    T = res["totals"]
    bal = T["absorbed"] + T["escaped"] + T["truncated"] - T["emitted"]
    assert abs(bal) <= rel * T["emitted"], bal / T["emitted"]
    assert T["rays_seeded"] + 4 * T["splits"] == T["splits"] + T["rays_escaped"] + T["rays_truncated"]
    assert T["truncated"] <= 1e-8 * T["emitted"]


def _nested_small():
    p = W.lognormal_problem(91, 0, 24, 3)
    rng = W.rng_for(91, 1, 0)
    child = W.Grid(n_h=(10 ** rng.uniform(-2.5, -1.0, (16, 16, 16))).astype(np.float32),
                   x_hi=rng.uniform(0.5, 1.0, (16, 16, 16)).astype(np.float32),
                   dx_cm=p.grids[0].dx_cm / 2, parent=0, offset=(8, 6, 10))
    p.grids.append(child)
    p.sources[1, :3] = [12.25, 9.75, 13.5]          # one source inside the child
    return p


@pytest.mark.parametrize("make", [lambda: W.config0(),
                                  lambda: W.lognormal_problem(91, 2, 24, 4),
                                  _nested_small],
                         ids=["uniform32", "lognormal24", "nested24"])
def test_conservation_and_ledger(make):
    res = O.trace(make())
    _check_ledger(res)
    # the per-(source, group) escaped rates add up to the total
    assert res["escaped_sg"].sum() == pytest.approx(res["totals"]["escaped"], rel=1e-14)


def test_threads_do_not_change_the_result_beyond_rounding():
    p = W.lognormal_problem(91, 3, 24, 3)
    a = O.trace(p, n_threads=1)
    b = O.trace(p, n_threads=5)
    for k in ("segments", "splits", "rays_escaped", "rays_truncated"):
        assert a["totals"][k] == b["totals"][k]
    np.testing.assert_allclose(b["absorbed"][0], a["absorbed"][0], rtol=1e-13, atol=0)


def test_mirror_symmetry_cell_centred_source():
    n = 15
    g = W.uniform_grid(n, W.DX_C1, 1e-2, 0.8)
    p = W.Problem([g], np.array([[7.5, 7.5, 7.5, 1e49]]), W.hydrogen_spectrum([20.0]),
                  W.Params(phi_c=5.1, level_init=1, level_max=14, p_min_frac=1e-8))
    k = O.trace(p)["k_ph"][0]          # indexed [z, y, x]
    scale = k.max()
    for img in (k[::-1, :, :], k[:, ::-1, :], k[:, :, ::-1], np.transpose(k, (0, 2, 1))):
        assert np.max(np.abs(img - k)) <= 1e-13 * scale


def test_superposition_of_disjoint_source_sets():
    p = W.lognormal_problem(91, 4, 20, 5)
    full = O.trace(p)
    a = O.trace(W.subset_sources(p, [0, 2, 4]))
    b = O.trace(W.subset_sources(p, [1, 3]))
    s = full["absorbed"][0]
    np.testing.assert_allclose(a["absorbed"][0] + b["absorbed"][0], s, rtol=1e-13, atol=1e-13 * s.max())
    np.testing.assert_allclose(a["heating"][0] + b["heating"][0], full["heating"][0], rtol=1e-13,
                               atol=1e-13 * full["heating"][0].max())
    for k in ("segments", "splits", "rays_escaped", "rays_truncated", "rays_seeded"):
        assert a["totals"][k] + b["totals"][k] == full["totals"][k]


def test_power_of_two_rate_scaling_is_exact():
    p = W.lognormal_problem(91, 5, 16, 3)
    q = W.Problem(p.grids, p.sources.copy(), p.spectrum, p.params)
    q.sources[:, 3] *= 4.0
    a, b = O.trace(p), O.trace(q)
    for f in ("absorbed", "energy", "k_ph", "heating"):
        assert np.array_equal(b[f][0], 4.0 * a[f][0])
    assert np.array_equal(b["escaped_sg"], 4.0 * a["escaped_sg"])
    assert a["totals"]["segments"] == b["totals"]["segments"]
