"""Seeded workload generators: reproducible, with the stated distributions."""
import numpy as np

from paper_1012_2865_amd import workloads as W


def test_generators_are_deterministic():
    a, b = W.lognormal_problem(7, 3, 24, 5), W.lognormal_problem(7, 3, 24, 5)
    assert np.array_equal(a.grids[0].n_h, b.grids[0].n_h)
    assert np.array_equal(a.grids[0].x_hi, b.grids[0].x_hi)
    assert np.array_equal(a.sources, b.sources)
    c = W.lognormal_problem(7, 4, 24, 5)
    assert not np.array_equal(a.grids[0].n_h, c.grids[0].n_h)


def test_lognormal_statistics():
    n_h = W.lognormal_density(64, 1.0, 1e-2, W.rng_for(9, 0, 0)).astype(np.float64)
    assert n_h.dtype == np.float64 and n_h.min() > 0
    assert abs(n_h.mean() / 1e-2 - 1) < 1e-6
    assert abs(np.log(n_h).std() - 1.0) < 1e-6
    # power concentrated at large scales: neighbouring cells are correlated
    g = np.log(n_h)
    g = (g - g.mean()) / g.std()
    assert np.mean(g * np.roll(g, 1, axis=2)) > 0.3          # white noise gives ~0


def test_config1_shape_and_ranges():
    p = W.config1()
    g = p.grids[0]
    assert g.n_h.shape == (128, 128, 128) and g.n_h.dtype == np.float32
    assert g.x_hi.min() >= 0.5 and g.x_hi.max() < 1.0
    assert p.sources.shape == (16, 4)
    assert np.all((p.sources[:, :3] >= 0) & (p.sources[:, :3] < 128))
    # general float64 positions, not a coarse lattice: no coordinate is a
    # multiple of 2^-20 cell
    q = p.sources[:, :3] * 2.0 ** 20
    assert not np.any(q == np.floor(q))
    assert np.all((p.sources[:, 3] >= 1e48) & (p.sources[:, 3] <= 1e50))
    assert np.allclose(p.spectrum.energy_ev, [13.6, 20, 30, 60])
    np.testing.assert_allclose(p.spectrum.sigma_cm2, 6.3e-18 * (p.spectrum.energy_ev / 13.6) ** -3)
    assert abs(g.dx_cm / W.PC_CM - 15.625) < 1e-12


def test_config2_and_config3_shapes():
    probs = W.config2(8)
    assert all(p.grids[0].n_h.shape[0] in W.C2_EDGES for p in probs)
    assert all(1 <= p.n_sources <= 8 for p in probs)
    reqs = W.config3(100.0, n_requests=20, edges=(32, 64))
    t = [r.arrival_s for r in reqs]
    assert np.all(np.diff(t) > 0)
    assert all(1 <= r.problem.n_sources <= 32 for r in reqs)


def test_config4_nesting():
    p = W.config4(n_clusters=2, per_cluster=5, root_n=64, sub_root_cells=16, sigma_root_cells=4.0)
    root, sub = p.grids
    assert sub.parent == 0 and sub.dx_cm == root.dx_cm / 2
    lo = np.array(sub.offset)
    assert np.all(p.sources[:, :3] >= lo) and np.all(p.sources[:, :3] < lo + sub.n_h.shape[0] // 2)
    c = root.n_h.shape[0] // 2
    assert 95.0 < root.n_h[c, c, c] / 1e-2 <= 100.0      # cell centre is 0.87 cells from the peak
