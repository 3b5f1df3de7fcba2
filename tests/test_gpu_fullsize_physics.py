"""The optional physics at the benchmark's own size (lognormal 128^3, 16
sources, 4 groups), mixed precision, against the FP64 oracle, per cell to the
mixed path's bar (1e-4 relative wherever the oracle's value exceeds 1e-6 of
its maximum):

* the covering-factor correction (section 2.3) on the whole workload;
* the radiation-pressure acceleration (section 2.5.4) on the whole workload;
* time-dependent rays (section 2.1) on a two-source subset for three steps
  of c dt_P = 32 cells (the oracle's time-dependent step runs on one thread).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def _rel(got, want):
    got, want = _np(got).ravel(), np.asarray(want).ravel()
    m = want > 1e-6 * want.max()
    return float(np.max(np.abs(got[m] - want[m]) / want[m])), float(np.max(np.abs(got - want)) / want.max())


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    c = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    yield c
    M.moray_free(c)


def test_covering_factor_at_full_size(ctx):
    p = W.config1()
    p.params = W.Params(**{**p.params.__dict__, "covering": True})
    res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
    ref = O.trace(p, n_threads=16)
    for f in ("k_ph", "heating"):
        rel, absr = _rel(res[f][0], ref[f][0])
        print(f"[covering 128^3] {f}: max rel {rel:.2e}, max abs/max {absr:.2e}", flush=True)
        assert rel <= 1e-4 and absr <= 1e-4
    assert res["absorbed"] == pytest.approx(ref["totals"]["absorbed"], rel=1e-4)


def test_radiation_pressure_at_full_size(ctx):
    p = W.config1()
    res = M.moray_trace(ctx, [M.problem_to_device(p)], want_accel=True)[0]
    ref = O.trace(p, n_threads=16, want_accel=True)
    a, b = _np(res["accel"][0]), ref["accel"][0]
    norm = np.linalg.norm(b, axis=0)
    diff = np.linalg.norm(a - b, axis=0)
    m = norm > 1e-6 * norm.max()
    rel, absr = float(np.max(diff[m] / norm[m])), float(diff.max() / norm.max())
    print(f"[radiation pressure 128^3] max rel {rel:.2e}, max abs/max {absr:.2e}", flush=True)
    assert rel <= 1e-4 and absr <= 1e-4


def test_time_dependent_rays_at_full_size(ctx):
    p = W.subset_sources(W.config1(), [3, 11])
    dev = M.problem_to_device(p)
    td = M.moray_td_create(ctx, dev, 32.0, 1 << 24)
    try:
        rays = None
        for step in range(3):
            ref, rays = O.trace_td(p, 32.0, rays, out_cap=1 << 24)
            res, held = M.moray_td_step(ctx, td, dev)
            rel, absr = _rel(res["k_ph"][0], ref["k_ph"][0])
            print(f"[td 128^3 sources 3,11 step {step}] k_ph max rel {rel:.2e}; held {held:.4e} "
                  f"(oracle {ref['held']:.4e}), {len(rays)} rays in flight", flush=True)
            assert rel <= 1e-4 and absr <= 1e-4
            assert held == pytest.approx(ref["held"], rel=1e-4)
    finally:
        M.moray_td_free(ctx, td)
