"""Properties that hold at any size, checked at the benchmark sizes (the
element-wise oracle comparisons of the same workloads are in
test_gpu_bench_configs.py: the whole 128^3 workload, all 64 batched problems,
10-source subsets of the nested workload).

* Nested 256^3 root + 128^3 child, 1000 clustered sources, 4 groups: a
  2-source subset against the FP64 oracle (per-cell bars as elsewhere), and
  at full size photon conservation, the integer ray ledger and linearity in
  the sources -- k_ph of all sources equals the sum over two disjoint halves
  (each cell receives the same deposits, summed in another order). The
  oracle would take minutes on all 1000 sources, so the whole workload is
  checked through these properties.
* Lognormal 128^3, 16 sources: linearity over four disjoint quarters at full
  size, in both precisions.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu


def _np(a):
    return a.detach().cpu().numpy()


def _rel(got, want, floor=1e-6):
    m = want > floor * want.max()
    return float(np.max(np.abs(got[m] - want[m]) / want[m]))


def _invariants(r, name):
    bal = r["absorbed"] + r["escaped"] + r["truncated"] - r["emitted"]
    print(f"[{name}] segments {r['segments']:.4e} conservation {bal / r['emitted']:.2e}", flush=True)
    assert abs(bal) <= 1e-9 * r["emitted"]
    assert r["rays_seeded"] + 4 * r["splits"] == r["splits"] + r["rays_escaped"] + r["rays_truncated"]


def _linearity(ctx, p, parts, name, tol):
    whole = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
    _invariants(whole, name)
    pieces = [M.moray_trace(ctx, [M.problem_to_device(W.subset_sources(p, list(ix)))])[0] for ix in parts]
    assert sum(q["segments"] for q in pieces) == whole["segments"]
    assert sum(q["splits"] for q in pieces) == whole["splits"]
    for g in range(len(whole["k_ph"])):
        want = sum(_np(q["k_ph"][g]) for q in pieces)
        rel = _rel(_np(whole["k_ph"][g]), want)
        print(f"[{name}] grid {g}: whole vs sum of parts max rel {rel:.2e}", flush=True)
        assert rel <= tol


@pytest.fixture(scope="module")
def nested():
    return W.config4()


@pytest.fixture(scope="module")
def nested_ref(nested):
    sub = W.subset_sources(nested, [0, 517])
    return sub, O.trace(sub, n_threads=16)


@pytest.mark.parametrize("precision,tol", [(M.MORAY_FP32_ACC64, 1e-4), (M.MORAY_FP64, 1e-9)])
def test_nested_subset_matches_oracle(nested_ref, precision, tol):
    sub, ref = nested_ref
    ctx = M.moray_init(device=0, precision=precision)
    try:
        r = M.moray_trace(ctx, [M.problem_to_device(sub)])[0]
    finally:
        M.moray_free(ctx)
    _invariants(r, f"nested subset {precision}")
    for g in range(2):
        for f in ("k_ph", "heating"):
            rel = _rel(_np(r[f][g]), ref[f][g])
            print(f"[nested subset {precision}] grid {g} {f} max rel {rel:.2e}", flush=True)
            assert rel <= tol
    T = ref["totals"]
    if precision == M.MORAY_FP64:
        for k in ("segments", "splits", "rays_escaped", "rays_truncated"):
            assert r[k] == T[k]
    else:
        flips = abs(r["splits"] - T["splits"])
        assert abs(r["segments"] - T["segments"]) <= 1e-5 * T["segments"] + 2 + 3 * flips


def test_nested_full_size_linearity(nested):
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        idx = np.arange(nested.n_sources)
        _linearity(ctx, nested, [idx[::2], idx[1::2]], "nested full fp32", 1e-9)
    finally:
        M.moray_free(ctx)


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_lognormal128_full_size_linearity(precision):
    p = W.config1()
    ctx = M.moray_init(device=0, precision=precision)
    try:
        _linearity(ctx, p, [range(0, 4), range(4, 8), range(8, 12), range(12, 16)], f"c1 full {precision}", 1e-9)
    finally:
        M.moray_free(ctx)
