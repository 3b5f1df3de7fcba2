"""Pins of the oracle's time-dependent rays (orc_trace_td: section 2.1, a ray
halts once it has travelled c dt_P and goes on in the next step; section 3.1
step 3j):

* With c dt_P beyond the box every ray finishes in one step: the step equals
  the single pass bit for bit and holds no ray.
* Photon bookkeeping per step: emitted + held before = absorbed + escaped +
  truncated + held after, to rounding.
* Steady state: with fixed fields and sources, once the oldest rays have had
  time to leave, every step deposits what the single pass deposits (a segment
  cut at a halting radius absorbs P(1 - e^-t1) + P e^-t1 (1 - e^-t2) =
  P(1 - e^-(t1+t2)), and splits are tested at the same cell exits).
* Light front: in the first step no cell whose nearest point lies beyond
  c dt_P of the source is reached, and in a thin uniform box every cell that
  lies wholly within it is.
* A pulse: a source that emits in one step only lights a shell that moves
  out by c dt_P per step; cells wholly inside the shell's inner radius stay
  dark.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import workloads as W


def _thin_uniform(n=20, src=(10.5, 9.5, 10.25)):
    g = W.uniform_grid(n, W.DX_C1, 1e-3, 1e-2)           # tau per cell ~ 3e-3
    return W.Problem([g], np.array([[*src, 1e49]]), W.hydrogen_spectrum([13.6]),
                     W.Params(phi_c=3.0, level_init=1, level_max=10, p_min_frac=1e-8))


def _cell_distances(shape, s):
    nz, ny, nx = shape
    c = [np.arange(m) + 0.5 for m in (nz, ny, nx)]
    dz, dy, dx = np.meshgrid(np.abs(c[0] - s[2]), np.abs(c[1] - s[1]), np.abs(c[2] - s[0]), indexing="ij")
    near = np.sqrt(np.maximum(dx - 0.5, 0) ** 2 + np.maximum(dy - 0.5, 0) ** 2 + np.maximum(dz - 0.5, 0) ** 2)
    far = np.sqrt((dx + 0.5) ** 2 + (dy + 0.5) ** 2 + (dz + 0.5) ** 2)
    return near, far


def test_infinite_speed_of_light_is_the_single_pass():
    p = W.lognormal_problem(94, 1, 20, 2, mean=1e-4)
    ref = O.trace(p)
    res, rays = O.trace_td(p, 1e6)
    assert len(rays) == 0 and res["held"] == 0.0
    assert np.array_equal(res["k_ph"][0], ref["k_ph"][0])
    for k in ("segments", "splits", "rays_escaped", "rays_truncated", "rays_seeded"):
        assert res["totals"][k] == ref["totals"][k], k


def test_bookkeeping_and_steady_state():
    p = W.lognormal_problem(94, 2, 20, 2, mean=1e-4)
    ref = O.trace(p)
    rays, held = None, 0.0
    for step in range(12):                             # 12 * 4 cells > the box diagonal
        res, rays = O.trace_td(p, 4.0, rays)
        T = res["totals"]
        bal = T["emitted"] + held - T["absorbed"] - T["escaped"] - T["truncated"] - res["held"]
        assert abs(bal) <= 1e-13 * T["emitted"], (step, bal)
        held = res["held"]
        if step == 0:
            assert len(rays) > 0 and held > 0.0
    k, kr = res["k_ph"][0], ref["k_ph"][0]
    m = kr > 1e-6 * kr.max()
    assert np.max(np.abs(k[m] - kr[m]) / kr[m]) <= 1e-12
    assert np.all(k[~m] <= 1e-6 * kr.max())
    assert res["totals"]["absorbed"] == pytest.approx(ref["totals"]["absorbed"], rel=1e-12)
    assert res["totals"]["escaped"] == pytest.approx(ref["totals"]["escaped"], rel=1e-12)


def test_first_step_reaches_c_dt():
    p = _thin_uniform()
    cdt = 6.0
    res, rays = O.trace_td(p, cdt)
    k = res["k_ph"][0]
    near, far = _cell_distances(k.shape, p.sources[0, :3])
    assert np.all(k[near > cdt] == 0.0)
    assert np.all(k[far < cdt] > 0.0)
    assert np.all(rays["r"] == cdt) and np.all(rays["age"] == 0)


def test_a_pulse_lights_a_moving_shell():
    p = _thin_uniform()
    cdt = 3.0
    res, rays = O.trace_td(p, cdt)                     # the only step that emits
    held = res["held"]
    for step in range(1, 4):
        res, rays = O.trace_td(p, cdt, rays, emit=False)
        T = res["totals"]
        assert T["emitted"] == 0.0
        assert T["absorbed"] + T["escaped"] + T["truncated"] + res["held"] == pytest.approx(held, rel=1e-13)
        held = res["held"]
        k = res["k_ph"][0]
        near, far = _cell_distances(k.shape, p.sources[0, :3])
        r_in, r_out = step * cdt, (step + 1) * cdt
        assert np.all(k[far < r_in] == 0.0), step      # behind the shell
        assert np.all(k[near > r_out] == 0.0), step    # ahead of it
        assert np.all(k[(near > r_in) & (far < r_out)] > 0.0), step
