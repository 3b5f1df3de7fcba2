"""Oracle parity at every benchmark configuration, element by element, and on
the input classes the benchmark workloads do not reach.

* The 128^3 workload (16 sources, 4 groups) whole, in both precisions, with
  the launch settings and graph replay of the timed form.
* All 64 problems of the batched workload through a context the autotuner
  tuned, on a graph-replayed batched call (the timed mixed-precision form),
  and through the plain float64 form (one problem per call).
* Three 10-source subsets of the nested 256^3 + 128^3 workload: one cluster's
  first ten sources, another cluster's, and one source from each cluster.
* A serving request of the largest class (256^3, 32 sources, photon rates
  log-uniform in [1e47, 1e51]) submitted asynchronously inside a mix of
  smaller requests, checked on a 4-source subset that runs in the same mix
  and by equality with the same request traced alone.
* Sources at general float64 positions near cell planes, corners and the
  faces of a child grid, in both precisions.
* Rays at HEALPix levels 11 to 15: seeds at level 11, and a narrow column
  whose rays split level by level up to level 15 (the 64-bit ring arithmetic
  of levels 14 and up).

Bars as in the other parity tests (tests/checks.py).
"""
import os

import numpy as np
import pytest

from checks import check, np_
from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
PRECISIONS = [(M.MORAY_FP32_ACC64, 1e-4, False), (M.MORAY_FP64, 1e-9, True)]


def _outputs(dev):
    import torch
    out = []
    for p in dev:
        n = sum(int(g.n_h.numel()) for g in p.grids)
        out.append((torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda")))
    return out


def _replayed(ctx, dev, calls=3):
    """The timed form: repeated calls on one set of result buffers, so the
    last call replays the captured launch sequence."""
    outs = _outputs(dev)
    res = None
    for _ in range(calls):
        res = M.moray_trace(ctx, dev, outputs=outs)
    assert res[0]["from_graph"] == 1
    return res


# ---------------------------------------------------------------------------
# 128^3, 16 sources, 4 groups: the whole workload
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1():
    p = W.config1()
    print(f"[c1] oracle on {THREADS} threads", flush=True)
    return p, O.trace(p, n_threads=THREADS)


@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_c1_whole_matches_oracle(c1, precision, tol, fp64):
    p, ref = c1
    dev = [M.problem_to_device(p)]
    ctx = M.moray_init(device=0, precision=precision)
    try:
        res = _replayed(ctx, dev)[0]
    finally:
        M.moray_free(ctx)
    check(res, ref, tol, name=f"c1 whole p{precision}", fp64=fp64)


# ---------------------------------------------------------------------------
# 64 grids of 32^3..96^3 with 1-8 sources: every problem, tuned and replayed
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2():
    probs = W.config2(64)
    print(f"[c2] oracle on {THREADS} threads, 64 problems", flush=True)
    return probs, [O.trace(p, n_threads=THREADS) for p in probs]


def test_c2_tuned_replayed_batch_matches_oracle(c2):
    probs, refs = c2
    dev = [M.problem_to_device(p) for p in probs]
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        tune = M.moray_autotune(ctx, dev)
        print(f"[c2] tuned settings {tune}", flush=True)
        res = _replayed(ctx, dev)
    finally:
        M.moray_free(ctx)
    worst = max(check(r, ref, 1e-4, name=f"c2 batched #{i}") for i, (r, ref) in enumerate(zip(res, refs)))
    print(f"[c2] batched: worst per-cell relative error over 64 problems {worst:.2e}", flush=True)


def test_c2_plain_fp64_one_per_call_matches_oracle(c2):
    probs, refs = c2
    ctx = M.moray_init(device=0, precision=M.MORAY_FP64)
    try:
        for i, (p, ref) in enumerate(zip(probs, refs)):
            res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
            check(res, ref, 1e-9, name=f"c2 fp64 #{i}", fp64=True)
    finally:
        M.moray_free(ctx)


# ---------------------------------------------------------------------------
# Nested 256^3 + 128^3, 1000 clustered sources: 10-source subsets
# ---------------------------------------------------------------------------
C4_SUBSETS = {
    "cluster0": np.arange(0, 10),
    "cluster6": np.arange(600, 610),
    "one_per_cluster": np.arange(10) * 100 + 37,
}


@pytest.fixture(scope="module")
def c4():
    return W.config4()


@pytest.mark.parametrize("subset", list(C4_SUBSETS))
def test_c4_subset_matches_oracle(c4, subset):
    sub = W.subset_sources(c4, C4_SUBSETS[subset])
    print(f"[c4 {subset}] oracle on {THREADS} threads", flush=True)
    ref = O.trace(sub, n_threads=THREADS)
    dev = [M.problem_to_device(sub)]
    for precision, tol, fp64 in PRECISIONS:
        ctx = M.moray_init(device=0, precision=precision)
        try:
            res = M.moray_trace(ctx, dev)[0]
        finally:
            M.moray_free(ctx)
        check(res, ref, tol, name=f"c4 {subset} p{precision}", fp64=fp64)


# ---------------------------------------------------------------------------
# The serving stream's largest request class, inside a mix
# ---------------------------------------------------------------------------
def test_largest_serving_request_in_a_mix_matches_oracle():
    """The 32-source 256^3 request runs inside a mix that also holds a
    4-source subset of it (its brightest and faintest sources and two more,
    on the same fields) and smaller requests. The subset is held to the
    oracle per cell; the whole request equals the same request traced alone
    (counts exactly, fields to summation order), so both sit on the oracle's
    arithmetic."""
    import time
    big = W.lognormal_problem(3, 424_242, 256, 32, log_ndot=(47.0, 51.0))
    nd = big.sources[:, 3]
    pick = sorted({int(np.argmax(nd)), int(np.argmin(nd)), 5, 17})
    sub = W.subset_sources(big, pick)
    small = [W.lognormal_problem(3, 424_243 + i, n, s, log_ndot=(47.0, 51.0))
             for i, (n, s) in enumerate([(32, 7), (64, 20), (128, 3), (32, 32)])]
    print(f"[c3 big] oracle on {THREADS} threads, sources {pick}", flush=True)
    ref = O.trace(sub, n_threads=THREADS)
    dev_big, dev_sub = M.problem_to_device(big), M.problem_to_device(sub)
    dev_small = [M.problem_to_device(p) for p in small]
    alone_ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        alone = M.moray_trace(alone_ctx, [dev_big])[0]
        tickets = [M.moray_trace_async(ctx, [dev_small[0]]), M.moray_trace_async(ctx, [dev_small[1]])]
        time.sleep(0.001)
        t_big = M.moray_trace_async(ctx, [dev_big])
        t_sub = M.moray_trace_async(ctx, [dev_sub])
        tickets += [M.moray_trace_async(ctx, [p]) for p in dev_small[2:]]
        res = M.moray_query(ctx, t_big, -1)[0]
        res_sub = M.moray_query(ctx, t_sub, -1)[0]
        others = [M.moray_query(ctx, t, -1)[0] for t in tickets]
    finally:
        M.moray_free(ctx)
        M.moray_free(alone_ctx)
    check(res_sub, ref, 1e-4, name="c3 256^3 subset of 4 sources, in the mix")
    for k in ("segments", "splits", "rays_seeded", "rays_escaped", "rays_truncated"):
        assert res[k] == alone[k], (k, res[k], alone[k])
    bal = res["absorbed"] + res["escaped"] + res["truncated"] - res["emitted"]
    assert abs(bal) <= 1e-9 * res["emitted"]
    for f in ("k_ph", "heating"):
        a, b = np_(res[f][0]).ravel(), np_(alone[f][0]).ravel()
        m = b > 1e-6 * b.max()
        rel = float(np.max(np.abs(a[m] - b[m]) / b[m]))
        print(f"[c3 big] 32 sources in the mix vs alone, {f}: max rel {rel:.2e}", flush=True)
        assert rel <= 1e-9
    # the mix really overlapped: some other request was admitted while the big one ran
    assert any(o["t_admit"] < res["t_done"] and o["t_done"] > res["t_admit"] for o in others + [res_sub])


# ---------------------------------------------------------------------------
# Sources anywhere: near planes, corners and child faces, both precisions
# ---------------------------------------------------------------------------
def _off_lattice_root():
    p = W.lognormal_problem(97, 11, 24, 4)
    p.sources = p.sources.copy()
    p.sources[0, :3] = [7.0 + 1e-13, 11.5 + 2.0 ** -30, 3.0 - 1e-12]         # just off two planes
    p.sources[1, :3] = [np.nextafter(12.0, 0.0), np.nextafter(12.0, 24.0), 12.0 + 3e-9]   # at a corner
    p.sources[2, :3] = [0.1234567890123, 23.9876543210987, 17.3141592653589]  # near the faces of the grid
    return p


def _off_lattice_nested():
    p = W.lognormal_problem(97, 12, 24, 4, params=W.Params(level_init=0))
    rng = W.rng_for(97, 112, 0)
    child = W.Grid(n_h=(10 ** rng.uniform(-2.5, -1.0, (16,) * 3)).astype(np.float32),
                   x_hi=rng.uniform(0.5, 1.0, (16,) * 3).astype(np.float32),
                   dx_cm=p.grids[0].dx_cm / 2, parent=0, offset=(6, 5, 7))
    p.grids.append(child)
    p.sources = p.sources.copy()
    p.sources[0, :3] = [6.0 + 1e-11, 9.123456789012345, 10.98765432109876]    # inside the child, at its x face
    p.sources[1, :3] = [10.25 + 2.0 ** -33, 8.75 - 1e-14, 12.5]               # on and near fine-cell planes
    p.sources[2, :3] = rng.uniform([6.0, 5.0, 7.0], [14.0, 13.0, 15.0])       # anywhere in the child
    p.sources[3, :3] = [np.nextafter(6.0, 0.0), 9.0, 11.0]                    # just outside the child
    return p


@pytest.mark.parametrize("case", ["root", "nested"])
@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_off_lattice_sources_match_oracle(case, precision, tol, fp64):
    p = _off_lattice_root() if case == "root" else _off_lattice_nested()
    ref = O.trace(p, n_threads=THREADS)
    ctx = M.moray_init(device=0, precision=precision)
    try:
        res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
    finally:
        M.moray_free(ctx)
    # Sources 1e-15 to 1e-9 cells from a plane (in two axes at the corner
    # source) make every diagonal ray cross pairs of planes closer than the
    # float path resolves (about 2^-36 / |d| cells): each such crossing is a
    # sub-resolution segment, counted or not depending on rounding, with no
    # deposit to speak of. Their number is not unique between the two
    # arithmetics, so in mixed precision it is bounded (2e-3 of the segments),
    # while fields, totals and split counts are held as everywhere.
    check(res, ref, tol, name=f"off-lattice {case} p{precision}", fp64=fp64, count_rtol=2e-3)
    if not fp64:
        assert res["splits"] == ref["totals"]["splits"]


# ---------------------------------------------------------------------------
# HEALPix levels 11-15
# ---------------------------------------------------------------------------
def _seeds_level11():
    """50 million seed rays at level 11 in a 2^3 grid; the rays towards the
    grid's corners travel far enough to split to level 12."""
    g = W.uniform_grid(2, W.DX_C1, 1e-3, 0.6)
    return W.Problem([g], np.array([[1.0173, 0.9741, 1.0089, 1e49]]), W.hydrogen_spectrum([20.0]),
                     W.Params(phi_c=1.56e6, level_init=11, level_max=15))


def _column(level_max=15):
    """A 2 x 2 x 256 column with a source near its bottom: the rays that stay
    in it split once per doubling of their radius, reaching level 14 at about
    200 cells and level 15 beyond."""
    g = W.uniform_grid((2, 2, 256), W.DX_C1, 1e-3, 0.6)
    return W.Problem([g], np.array([[1.0312, 0.9687, 0.5123, 1e49]]), W.hydrogen_spectrum([60.0]),
                     W.Params(phi_c=6.4e3, level_init=0, level_max=level_max))


@pytest.fixture(scope="module")
def deep_refs():
    out = {}
    for name, fn in (("seeds11", _seeds_level11), ("column", _column)):
        print(f"[deep {name}] oracle", flush=True)
        p = fn()
        out[name] = (p, O.trace(p, n_threads=THREADS))
    return out


@pytest.mark.parametrize("case", ["seeds11", "column"])
@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_deep_healpix_levels_match_oracle(deep_refs, case, precision, tol, fp64):
    p, ref = deep_refs[case]
    ctx = M.moray_init(device=0, precision=precision, queue_capacity=1 << 24)
    try:
        res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
    finally:
        M.moray_free(ctx)
    check(res, ref, tol, name=f"deep {case} p{precision}", fp64=fp64)


def test_column_reaches_level_15(deep_refs):
    """Level-14 rays split in the column: capping the levels at 14 removes
    splits, on both sides."""
    _, ref15 = deep_refs["column"]
    p14 = _column(level_max=14)
    ref14 = O.trace(p14, n_threads=THREADS)
    assert ref14["totals"]["splits"] < ref15["totals"]["splits"]
    ctx = M.moray_init(device=0, precision=M.MORAY_FP64, queue_capacity=1 << 24)
    try:
        res = M.moray_trace(ctx, [M.problem_to_device(p14)])[0]
    finally:
        M.moray_free(ctx)
    check(res, ref14, 1e-9, name="deep column l_max 14", fp64=True)
