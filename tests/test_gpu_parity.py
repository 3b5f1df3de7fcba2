"""GPU parity: the HIP library against the FP64 CPU oracle on the same seeded
inputs, through the C ABI.

Bars (written here, derived in the design notes):
* k_ph and heating per cell: relative error <= 1e-4 wherever the oracle's
  value exceeds 1e-6 of its maximum, in both precisions; the float64 path is
  also held to 1e-9 (it evaluates the same expressions in the same order up
  to atomic summation order and libm ulps).
* Photon conservation absorbed + escaped + truncated = emitted to 1e-9.
* The ray ledger seeded + 4 splits = splits + escaped + truncated exactly.
* Ray counts match the oracle's exactly in float64; in float32 they may differ
  only through cell-corner near-ties, bounded here by 1e-5 relative.
"""
import numpy as np
import pytest

from checks import check as _check, np_ as _np
from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(precision, **kw):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return M.moray_init(device=0, precision=precision, **kw)


@pytest.fixture(scope="module")
def ctx64():
    c = _ctx(M.MORAY_FP64)
    yield c
    M.moray_free(c)


@pytest.fixture(scope="module")
def ctx32():
    c = _ctx(M.MORAY_FP32_ACC64)
    yield c
    M.moray_free(c)


def _run(ctx, problems, **kw):
    dev = [M.problem_to_device(p) for p in problems]
    return M.moray_trace(ctx, dev, **kw)


def _nested(item, n=24, child_n=16):
    p = W.lognormal_problem(95, item, n, 3)
    rng = W.rng_for(95, 100 + item, 0)
    child = W.Grid(n_h=(10 ** rng.uniform(-2.5, -1.0, (child_n,) * 3)).astype(np.float32),
                   x_hi=rng.uniform(0.5, 1.0, (child_n,) * 3).astype(np.float32),
                   dx_cm=p.grids[0].dx_cm / 2, parent=0, offset=(6, 5, 7))
    p.grids.append(child)
    p.sources[0, :3] = [10.25, 9.5, 11.75]          # inside the child
    return p


CASES = {
    "uniform32_vertex": lambda: W.config0(),
    "lognormal24_s3": lambda: W.lognormal_problem(95, 1, 24, 3),
    "lognormal40_s2_l0": lambda: W.lognormal_problem(95, 2, 40, 2, params=W.Params(level_init=0)),
    "nested24": lambda: _nested(3),
    "thin32_phi2": lambda: W.lognormal_problem(95, 4, 32, 2, mean=1e-5, params=W.Params(phi_c=2.1)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_matches_oracle(ctx64, case):
    p = CASES[case]()
    ref = O.trace(p)
    res = _run(ctx64, [p])[0]
    _check(res, ref, 1e-9, name=f"fp64 {case}", fp64=True)


@pytest.mark.parametrize("case", list(CASES))
def test_fp32_matches_oracle(ctx32, case):
    p = CASES[case]()
    ref = O.trace(p)
    res = _run(ctx32, [p])[0]
    _check(res, ref, 1e-4, name=f"fp32 {case}")


def test_c1_source_subset_both_precisions(ctx32, ctx64):
    p = W.subset_sources(W.config1(), [3, 11])
    ref = O.trace(p, n_threads=8)
    _check(_run(ctx64, [p])[0], ref, 1e-9, name="fp64 c1[3,11]", fp64=True)
    _check(_run(ctx32, [p])[0], ref, 1e-4, name="fp32 c1[3,11]")


def test_host_fields_and_host_outputs(ctx32):
    p = W.lognormal_problem(95, 5, 24, 2)
    ref = O.trace(p)
    res = M.moray_trace(ctx32, [p], out_on_device=False, want_escaped_sg=True)[0]
    _check(res, ref, 1e-4, name="fp32 host-io")
    np.testing.assert_allclose(res["escaped_sg"], ref["escaped_sg"], rtol=1e-4, atol=1e-9 * ref["totals"]["emitted"])


def test_batch_equals_each_alone(ctx32):
    probs = [W.lognormal_problem(96, i, n, s) for i, (n, s) in enumerate([(16, 1), (32, 3), (24, 2), (16, 4)])]
    probs.append(_nested(7))
    together = _run(ctx32, probs)
    for p, t in zip(probs, together):
        alone = _run(ctx32, [p])[0]
        for q in range(len(p.grids)):
            a, b = _np(alone["k_ph"][q]), _np(t["k_ph"][q])
            assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * a.max()), q
        for k in ("segments", "splits", "rays_escaped", "rays_truncated", "rays_seeded"):
            assert alone[k] == t[k], k


def test_invalid_inputs_leave_outputs_untouched(ctx32):
    import torch
    p = W.lognormal_problem(95, 6, 16, 1)
    d = M.problem_to_device(p)
    d.grids[0].x_hi[3, 4, 5] = 1.5                        # neutral fraction above 1
    with pytest.raises(M.MorayError) as e:
        M.moray_trace(ctx32, [d])
    assert e.value.status == M.MORAY_EINVAL
    d = M.problem_to_device(p)
    d.grids[0].n_h[0, 0, 0] = float("nan")
    with pytest.raises(M.MorayError) as e:
        M.moray_trace(ctx32, [d])
    assert e.value.status == M.MORAY_EINVAL
    q = W.lognormal_problem(95, 6, 16, 1)
    q.sources = q.sources.copy()
    q.sources[0, 0] = 16.0                                # on the upper face: outside
    with pytest.raises(M.MorayError) as e:
        M.moray_trace(ctx32, [M.problem_to_device(q)])
    assert e.value.status == M.MORAY_EINVAL
    # the context still works afterwards
    ok = M.moray_trace(ctx32, [M.problem_to_device(p)])[0]
    assert ok["segments"] > 0
    torch.cuda.synchronize()


def test_small_queue_traces_in_chunks():
    # a queue smaller than the sum of the trees' bounds: trees are traced in
    # consecutive chunks that share the accumulators
    big = _ctx(M.MORAY_FP32_ACC64)
    c = _ctx(M.MORAY_FP32_ACC64, queue_capacity=20000)
    try:
        p = W.lognormal_problem(95, 8, 16, 6)
        ref = O.trace(p)
        res = _run(c, [p])[0]
        one = _run(big, [p])[0]
        _check(res, ref, 1e-4, name="fp32 small-queue")
        assert res["peak_level_rays"] <= 20000
        assert res["trace_launches"] > one["trace_launches"]
    finally:
        M.moray_free(c)
        M.moray_free(big)


def test_queue_too_small_for_one_tree_reports_equeue():
    c = _ctx(M.MORAY_FP32_ACC64, queue_capacity=256)
    try:
        p = W.lognormal_problem(95, 9, 16, 1, mean=1e-6)
        with pytest.raises(M.MorayError) as e:
            _run(c, [p])
        assert e.value.status == M.MORAY_EQUEUE
        # a problem without splits still runs on the same context
        q = W.lognormal_problem(95, 9, 16, 1, params=W.Params(phi_c=0.0))
        ref = O.trace(q)
        _check(_run(c, [q])[0], ref, 1e-4, name="fp32 no-split")
    finally:
        M.moray_free(c)


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_direct_atomics_and_lds_cache_agree(precision):
    # deposits combined in the per-wave LDS table and deposits sent one atomic
    # per segment give the same fields (to summation order)
    probs = [W.lognormal_problem(98, 0, 24, 4), _nested(9)]
    outs = {}
    for cache in (0, -1):
        c = _ctx(precision, deposit_cache=cache)
        try:
            outs[cache] = _run(c, probs)
        finally:
            M.moray_free(c)
    for p, a, b in zip(probs, outs[0], outs[-1]):
        ref = O.trace(p)
        for res in (a, b):
            _check(res, ref, 1e-4 if precision == M.MORAY_FP32_ACC64 else 1e-9, name=f"cache p{precision}",
                   fp64=precision == M.MORAY_FP64)
        for q in range(len(p.grids)):
            x, y = _np(a["k_ph"][q]), _np(b["k_ph"][q])
            assert np.allclose(x, y, rtol=1e-12, atol=1e-15 * y.max())
