"""moray_trace_noalloc, the entry point that allocates no device memory,
against moray_trace on the same inputs, through the C ABI: two calls in a
row, the second with a smaller batch (the fixed scratch array keeps the first
call's contents, so anything left over would show), in both precisions, and
a batch too large for the array rejected with MORAY_ENOMEM, and batches
with the optically-thin approximation (its marks and float64 columns live in
the array as well). Results must
equal moray_trace's to summation order: counts exactly, k_ph and heating to
1e-9 relative (1e-4 is the oracle bar of the mixed path; both calls run the
same kernels on the same inputs)."""
import numpy as np
import pytest

from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTS = ("segments", "thin_segments", "splits", "rays_seeded", "rays_escaped", "rays_truncated")


def _outputs(problems, device=True):
    import torch
    out = []
    for p in problems:
        n = sum(int(np.prod(g.n_h.shape)) for g in p.grids)
        if device:
            out.append((torch.full((n,), -1.0, dtype=torch.float64, device="cuda"),
                        torch.full((n,), -1.0, dtype=torch.float64, device="cuda")))
        else:
            out.append((np.full(n, -1.0), np.full(n, -1.0)))
    return out


def _same(got, want, name):
    for k in COUNTS:
        assert got[k] == want[k], (name, k, got[k], want[k])
    for k in ("emitted", "absorbed", "escaped", "truncated"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-12 * want["emitted"]), (name, k)
    for q in range(len(want["k_ph"])):
        for f in ("k_ph", "heating"):
            a = got[f][q].detach().cpu().numpy().ravel() if hasattr(got[f][q], "detach") else np.ravel(got[f][q])
            b = want[f][q].detach().cpu().numpy().ravel() if hasattr(want[f][q], "detach") else np.ravel(want[f][q])
            m = b > 1e-6 * b.max()
            rel = float(np.max(np.abs(a[m] - b[m]) / b[m]))
            print(f"[{name}] grid {q} {f}: max rel vs moray_trace {rel:.2e}", flush=True)
            assert rel <= 1e-9, (name, q, f, rel)
            assert np.all(np.abs(a[~m] - b[~m]) <= 1e-9 * b.max()), (name, q, f)


def _nested():
    p = W.lognormal_problem(93, 3, 24, 3)
    rng = W.rng_for(93, 103, 0)
    p.grids.append(W.Grid(n_h=(10 ** rng.uniform(-2.5, -1.0, (16,) * 3)).astype(np.float32),
                          x_hi=rng.uniform(0.5, 1.0, (16,) * 3).astype(np.float32),
                          dx_cm=p.grids[0].dx_cm / 2, parent=0, offset=(6, 5, 7)))
    return p


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_noalloc_equals_trace_twice_second_smaller(precision):
    first = [W.lognormal_problem(93, 0, 64, 6), W.lognormal_problem(93, 1, 48, 3), _nested()]
    second = [W.lognormal_problem(93, 2, 24, 2)]
    ctx = M.moray_init(device=0, precision=precision)
    ref = M.moray_init(device=0, precision=precision)
    try:
        for call, probs in enumerate((first, second)):
            dev = [M.problem_to_device(p) for p in probs]
            print(f"[noalloc p{precision}] call {call}: {len(probs)} problems", flush=True)
            got = M.moray_trace_noalloc(ctx, dev, _outputs(probs))
            want = M.moray_trace(ref, dev)
            for i, (g, w) in enumerate(zip(got, want)):
                _same(g, w, f"noalloc p{precision} call {call} problem {i}")
        # host fields and host results go through the array too
        probs = [W.lognormal_problem(93, 4, 32, 2)]
        got = M.moray_trace_noalloc(ctx, probs, _outputs(probs, device=False), out_on_device=False)
        want = M.moray_trace(ref, probs, out_on_device=False)
        _same(got[0], want[0], f"noalloc p{precision} host io")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)


def _thin(item, n, n_src):
    """ionised lognormal gas with the optically-thin approximation: its marks
    and float64 columns come from the scratch array too"""
    p = W.lognormal_problem(93, item, n, n_src)
    g = p.grids[0]
    p.grids[0] = W.Grid(g.n_h, (g.x_hi * np.float32(0.05)).astype(np.float32), g.dx_cm)
    p.params = W.Params(**{**p.params.__dict__, "tau_thin": 0.1})
    return p


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_noalloc_optically_thin_twice_second_smaller(precision):
    ctx = M.moray_init(device=0, precision=precision)
    ref = M.moray_init(device=0, precision=precision)
    try:
        for call, probs in enumerate(([_thin(7, 32, 3), W.lognormal_problem(93, 8, 24, 2)], [_thin(9, 24, 2)])):
            dev = [M.problem_to_device(p) for p in probs]
            print(f"[noalloc thin p{precision}] call {call}: {len(probs)} problems", flush=True)
            got = M.moray_trace_noalloc(ctx, dev, _outputs(probs))
            want = M.moray_trace(ref, dev)
            assert want[0]["thin_segments"] > 0
            for i, (g, w) in enumerate(zip(got, want)):
                _same(g, w, f"noalloc thin p{precision} call {call} problem {i}")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)


def test_noalloc_rejects_a_batch_beyond_the_array_and_recovers():
    big = [M.problem_to_device(W.lognormal_problem(93, 5, 256, 1))]   # 16.8 M cells x 4 groups of accumulators
    small = [M.problem_to_device(W.lognormal_problem(93, 6, 24, 2))]
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ref = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        with pytest.raises(M.MorayError) as e:
            M.moray_trace_noalloc(ctx, big, _outputs(big))
        assert e.value.status == M.MORAY_ENOMEM
        assert "scratch array" in str(e.value)
        got = M.moray_trace_noalloc(ctx, small, _outputs(small))
        _same(got[0], M.moray_trace(ref, small)[0], "after a rejected batch")
        # the context's own moray_trace still works, with its own buffers
        _same(M.moray_trace(ctx, small)[0], M.moray_trace(ref, small)[0], "moray_trace on the same context")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)
