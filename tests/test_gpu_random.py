"""Oracle parity on seeded random problems (section 2.1-2.2, section 3.1
steps 3a-3k), beyond the hand-built cases: root grids of 8-24 cells per
edge, cubic or not, with or without a 2x-refined child at a random aligned
place; 1-3 sources at random float64 positions, some snapped onto a cell
plane, edge or vertex, some inside the child; 1-4 groups; seed levels 0-2;
split thresholds from 1.1 to 25.1 rays per face; level caps 6 or 14;
truncation at 1e-8 or 1e-3 of the seed rate; media from optically thin to
thick. Every problem alone in both precisions, and all of them in one
batched call (mixed precision), each per cell against the oracle. Bars as
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
