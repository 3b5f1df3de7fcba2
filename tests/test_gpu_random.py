"""Oracle parity on seeded random problems (section 2.1-2.2, section 3.1
steps 3a-3k), beyond the hand-built cases: root grids of 8-24 cells per
edge, cubic or not, with or without a 2x-refined child at a random aligned
place; 1-3 sources at random float64 positions, some snapped onto a cell
plane, edge or vertex, some inside the child; 1-4 groups; seed levels 0-2;
split thresholds from 1.1 to 25.1 rays per face; level caps 6 or 14;
truncation at 1e-8 or 1e-3 of the seed rate; media from optically thin to
thick. Every problem alone in both precisions, and all of them in one
batched call (mixed precision), each per cell against the oracle; the
covering-factor correction, the radiation-pressure acceleration and
time-dependent rays on subsets of them; all of them through the serving
engine in staggered groups. Bars as
in the other parity tests (tests/checks.py); the mixed-precision counts of
sources on planes may differ by sub-resolution segments (2e-3 of the
segments, as for the off-lattice cases).
"""
import os

import numpy as np
import pytest

from checks import check
from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
N_PROBLEMS = 24


def _problem(k: int) -> W.Problem:
    rng = W.rng_for(90, k, 0)
    nx, ny, nz = (int(rng.choice([8, 12, 16, 24])) for _ in range(3)) if rng.random() < 0.3 else \
        (int(rng.choice([8, 12, 16, 24])),) * 3
    dx = W.DX_C1 * float(rng.choice([0.5, 1.0, 4.0]))
    mean = float(10.0 ** rng.uniform(-4.0, 0.5))
    lg = W.lognormal_density(max(nx, ny, nz), 1.0, mean, rng)[:nz, :ny, :nx]
    root = W.Grid(np.ascontiguousarray(lg, dtype=np.float32),
                  rng.uniform(0.0, 1.0, (nz, ny, nx)).astype(np.float32), dx)
    grids = [root]
    child_box = None
    if rng.random() < 0.4:
        # m root cells per axis, refined 2x, inside the root
        m = [int(rng.integers(1, max(2, n // 2) + 1)) for n in (nx, ny, nz)]
        o = [int(rng.integers(0, n - mm + 1)) for n, mm in zip((nx, ny, nz), m)]
        shape = (2 * m[2], 2 * m[1], 2 * m[0])
        cn = (mean * rng.lognormal(0.0, 0.7, shape)).astype(np.float32)
        grids.append(W.Grid(cn, rng.uniform(0.0, 1.0, shape).astype(np.float32), dx / 2.0, parent=0,
                            offset=(o[0], o[1], o[2])))
        child_box = (o, m)
    n_src = int(rng.integers(1, 4))
    src = np.empty((n_src, 4))
    for s in range(n_src):
        if child_box is not None and rng.random() < 0.5:
            o, m = child_box
            pos = [o[a] + rng.uniform(0.0, m[a]) for a in range(3)]
        else:
            pos = [rng.uniform(0.0, n) for n in (nx, ny, nz)]
        snap = int(rng.integers(0, 4))          # 0: general, 1-3: on that many cell planes
        for a in rng.permutation(3)[:snap]:
            pos[a] = float(np.clip(np.floor(pos[a]), 0.0, (nx, ny, nz)[a] - 1))
        src[s, :3] = np.minimum(pos, np.nextafter(np.array([nx, ny, nz], dtype=np.float64), 0.0))
        src[s, 3] = 10.0 ** rng.uniform(47.0, 50.0)
    n_grp = int(rng.integers(1, 5))
    spec = W.hydrogen_spectrum(sorted(rng.choice([13.6, 16.0, 20.0, 30.0, 45.0, 60.0], n_grp, replace=False)))
    params = W.Params(phi_c=float(rng.choice([1.1, 3.1, 5.1, 10.1, 25.1])), level_init=int(rng.integers(0, 3)),
                      level_max=int(rng.choice([6, 14])), p_min_frac=float(rng.choice([1e-8, 1e-3])))
    return W.Problem(grids, src, spec, params, name=f"random{k}")


@pytest.fixture(scope="module")
def cases():
    out = []
    for k in range(N_PROBLEMS):
        p = _problem(k)
        out.append((p, O.trace(p, n_threads=THREADS)))
    print(f"[random] {len(out)} problems, {sum(r['totals']['segments'] for _, r in out)} oracle segments", flush=True)
    return out


@pytest.mark.parametrize("precision,tol,fp64", [(M.MORAY_FP32_ACC64, 1e-4, False), (M.MORAY_FP64, 1e-9, True)])
def test_random_problems_alone(cases, precision, tol, fp64):
    ctx = M.moray_init(device=0, precision=precision)
    try:
        for p, ref in cases:
            res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
            check(res, ref, tol, name=f"{p.name} p{precision}", fp64=fp64, count_rtol=2e-3)
    finally:
        M.moray_free(ctx)


def test_random_problems_in_one_batch(cases):
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        res = M.moray_trace(ctx, [M.problem_to_device(p) for p, _ in cases])
        for (p, ref), r in zip(cases, res):
            check(r, ref, 1e-4, name=f"{p.name} batched", count_rtol=2e-3)
    finally:
        M.moray_free(ctx)


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def _field_rel(got, want):
    got, want = _np(got).ravel(), np.asarray(want).ravel()
    mx = want.max()
    if mx == 0.0:
        return 0.0, float(np.abs(got).max())
    m = want > 1e-6 * mx
    return float(np.max(np.abs(got[m] - want[m]) / want[m])), float(np.max(np.abs(got - want)) / mx)


PRECISIONS = [(M.MORAY_FP32_ACC64, 1e-4, False), (M.MORAY_FP64, 1e-9, True)]


@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_random_problems_with_covering_factor(precision, tol, fp64):
    """The covering-factor correction (section 2.3) on the first 12 random
    problems: k_ph and heating per cell, escaped photons and (float64)
    every count; the corrected deposit is not photon-conserving, so the
    ledger is not held."""
    ctx = M.moray_init(device=0, precision=precision)
    try:
        for k in range(12):
            p = _problem(k)
            p.params = W.Params(**{**p.params.__dict__, "covering": True})
            ref = O.trace(p, n_threads=THREADS)
            res = M.moray_trace(ctx, [M.problem_to_device(p)])[0]
            for q in range(len(p.grids)):
                for f in ("k_ph", "heating"):
                    rel, absr = _field_rel(res[f][q], ref[f][q])
                    assert rel <= tol and absr <= max(tol, 1e-6), (p.name, q, f, rel, absr)
            T = ref["totals"]
            assert res["absorbed"] == pytest.approx(T["absorbed"], rel=tol)
            assert res["escaped"] == pytest.approx(T["escaped"], rel=max(tol, 1e-12), abs=1e-12 * T["emitted"])
            if fp64:
                for c in ("segments", "splits", "rays_escaped", "rays_truncated"):
                    assert res[c] == T[c], (p.name, c)
    finally:
        M.moray_free(ctx)


@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_random_problems_with_radiation_pressure(precision, tol, fp64):
    """The radiation-pressure acceleration (section 2.5.4) on the first 12
    random problems: per cell the vector against the oracle's."""
    ctx = M.moray_init(device=0, precision=precision)
    try:
        for k in range(12):
            p = _problem(k)
            ref = O.trace(p, n_threads=THREADS, want_accel=True)
            res = M.moray_trace(ctx, [M.problem_to_device(p)], want_accel=True)[0]
            for q in range(len(p.grids)):
                a, b = _np(res["accel"][q]), np.asarray(ref["accel"][q])
                norm = np.linalg.norm(b, axis=0)
                if norm.max() == 0.0:
                    assert np.abs(a).max() == 0.0
                    continue
                diff = np.linalg.norm(a - b, axis=0)
                m = norm > 1e-6 * norm.max()
                rel, absr = float(np.max(diff[m] / norm[m])), float(diff.max() / norm.max())
                assert rel <= tol and absr <= max(tol, 1e-6), (p.name, q, rel, absr)
    finally:
        M.moray_free(ctx)


@pytest.mark.parametrize("precision,tol,fp64", PRECISIONS)
def test_random_problems_time_dependent(precision, tol, fp64):
    """Time-dependent rays (section 2.1, c dt_P of 1.5-8 root cells) on six
    random problems, four steps each with a random emission pattern (a
    pulsed source emits in some steps only): k_ph per cell, the photons
    held by the rays in flight, and (float64) every count."""
    ctx = M.moray_init(device=0, precision=precision)
    try:
        for k in range(6):
            p = _problem(k)
            rng = W.rng_for(90, k, 1)
            cdt = float(rng.uniform(1.5, 8.0))
            emits = [True] + [bool(rng.random() < 0.6) for _ in range(3)]
            dev = M.problem_to_device(p)
            td = M.moray_td_create(ctx, dev, cdt, 1 << 20)
            try:
                rays, held_prev = None, 0.0
                for step, emit in enumerate(emits):
                    ref, rays = O.trace_td(p, cdt, rays, emit=emit)
                    res, held = M.moray_td_step(ctx, td, dev, emit=emit)
                    T = ref["totals"]
                    for q in range(len(p.grids)):
                        rel, absr = _field_rel(res["k_ph"][q], ref["k_ph"][q])
                        assert rel <= tol and absr <= max(tol, 1e-6), (p.name, step, q, rel, absr)
                    scale = max(T["emitted"], held_prev, 1.0)
                    assert held == pytest.approx(ref["held"], rel=tol, abs=1e-12 * scale), (p.name, step)
                    if fp64:
                        for c in ("segments", "splits", "rays_escaped", "rays_truncated", "rays_seeded"):
                            assert res[c] == T[c], (p.name, step, c, res[c], T[c])
                    held_prev = held
            finally:
                M.moray_td_free(ctx, td)
    finally:
        M.moray_free(ctx)


def test_random_problems_served(cases):
    """All 24 random problems submitted to the serving engine (continuous
    batching) in staggered groups of one to four while earlier ones run;
    every result against the oracle, mixed precision."""
    import time
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        dev = [M.problem_to_device(p) for p, _ in cases]
        rng = np.random.default_rng(91)
        tickets, i = [], 0
        while i < len(dev):
            n = int(rng.integers(1, 5))
            tickets.append((i, M.moray_trace_async(ctx, dev[i:i + n])))
            i += n
            time.sleep(float(rng.uniform(0.0, 0.004)))
        for first, t in tickets:
            res = M.moray_query(ctx, t, -1)
            for j, r in enumerate(res):
                p, ref = cases[first + j]
                check(r, ref, 1e-4, name=f"{p.name} served", count_rtol=2e-3)
    finally:
        M.moray_free(ctx)
