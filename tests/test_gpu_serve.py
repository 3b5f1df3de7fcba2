"""Serving engine (moray_trace_async / moray_query) on the GPU.

* Every problem's results in a running mix equal its results traced alone by
  moray_trace: ray and segment counts exactly, k_ph and heating to 1e-9
  relative wherever they exceed 1e-6 of their maximum (only the order of the
  float64 additions into a cell differs), in both precisions.
* Problems submitted while others run are admitted into the running launch
  sequence (their admission time precedes the earlier problems' completion).
* One asynchronous result is checked against the FP64 oracle directly.
* Invalid field values fail only their own ticket; host fields and host
  outputs work; tickets report MORAY_EBUSY until done and are then forgotten.
* A problem that overflows the ray queue while running alone fails with
  MORAY_EQUEUE on its own ticket, and the engine goes on with the next one.
"""
import ctypes
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTS = ("segments", "splits", "rays_seeded", "rays_escaped", "rays_truncated")


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def _same(got, want, tol, name):
    for k in COUNTS:
        assert got[k] == want[k], (name, k, got[k], want[k])
    for k in ("emitted", "absorbed", "escaped", "truncated"):
        assert got[k] == pytest.approx(want[k], rel=tol, abs=1e-12 * want["emitted"]), (name, k)
    for q in range(len(want["k_ph"])):
        for f in ("k_ph", "heating"):
            a, b = _np(got[f][q]).ravel(), _np(want[f][q]).ravel()
            m = b > 1e-6 * b.max() if b.max() > 0 else np.zeros_like(b, bool)
            rel = float(np.max(np.abs(a[m] - b[m]) / b[m])) if m.any() else 0.0
            print(f"[{name}] grid {q} {f}: max rel vs alone {rel:.2e}", flush=True)
            assert rel <= tol, (name, q, f, rel)
            assert np.all(a[~m] <= 1e-6 * b.max() * (1 + 1e-6) + 1e-300), (name, q, f)


def _mix():
    return [
        W.lognormal_problem(96, 0, 128, 16),                     # long-running anchor (~10 ms)
        W.lognormal_problem(96, 1, 24, 3),
        W.lognormal_problem(96, 2, 40, 2, params=W.Params(level_init=0)),
        W.lognormal_problem(96, 3, 32, 5, mean=1e-4),
        W.lognormal_problem(96, 4, 48, 1, params=W.Params(phi_c=2.1)),
    ]


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_mix_equals_alone(precision):
    probs = [M.problem_to_device(p) for p in _mix()]
    alone_ctx = M.moray_init(device=0, precision=precision)
    serve_ctx = M.moray_init(device=0, precision=precision)
    try:
        alone = [M.moray_trace(alone_ctx, [p])[0] for p in probs]
        print(f"[precision {precision}] submitting {len(probs)} problems, staggered", flush=True)
        tickets = [M.moray_trace_async(serve_ctx, [probs[0]])]
        time.sleep(0.002)
        tickets.append(M.moray_trace_async(serve_ctx, probs[1:3]))
        time.sleep(0.001)
        tickets += [M.moray_trace_async(serve_ctx, [p]) for p in probs[3:]]
        got = []
        for t in tickets:
            r = M.moray_query(serve_ctx, t, -1)
            assert r is not None
            got += r
        for i, (g, a) in enumerate(zip(got, alone)):
            _same(g, a, 1e-9, f"p{i}")
            assert g["t_done"] >= g["t_admit"] > 0.0
        # the later problems joined while the anchor was still on the device
        assert min(g["t_admit"] for g in got[1:]) < got[0]["t_done"]
    finally:
        M.moray_free(serve_ctx)
        M.moray_free(alone_ctx)


def test_async_matches_oracle():
    p = W.lognormal_problem(96, 5, 24, 2)
    ref = O.trace(p)
    ctx = M.moray_init(device=0, precision=M.MORAY_FP64)
    try:
        t = M.moray_trace_async(ctx, [M.problem_to_device(p)])
        res = M.moray_query(ctx, t, -1)[0]
    finally:
        M.moray_free(ctx)
    T = ref["totals"]
    for k in ("segments", "splits", "rays_escaped", "rays_truncated"):
        assert res[k] == T[k], (k, res[k], T[k])
    k_ref = ref["k_ph"][0]
    k_got = _np(res["k_ph"][0])
    m = k_ref > 1e-6 * k_ref.max()
    rel = float(np.max(np.abs(k_got[m] - k_ref[m]) / k_ref[m]))
    print(f"[async fp64 vs oracle] k_ph max rel {rel:.2e}", flush=True)
    assert rel <= 1e-9
    bal = res["absorbed"] + res["escaped"] + res["truncated"] - res["emitted"]
    assert abs(bal) <= 1e-9 * res["emitted"]


def test_host_io_and_bad_fields_fail_alone():
    good = W.lognormal_problem(96, 6, 24, 2)
    bad = W.lognormal_problem(96, 7, 24, 2)
    bad.grids[0].n_h[3, 4, 5] = np.nan
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ref_ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        alone = M.moray_trace(ref_ctx, [good], out_on_device=False)[0]
        tb = M.moray_trace_async(ctx, [bad], out_on_device=False)
        tg = M.moray_trace_async(ctx, [good], out_on_device=False)
        with pytest.raises(M.MorayError) as e:
            M.moray_query(ctx, tb, -1)
        assert e.value.status == M.MORAY_EINVAL
        _same(M.moray_query(ctx, tg, -1)[0], alone, 1e-9, "host-io")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref_ctx)


def test_ticket_semantics():
    lib = M.load_library()
    big = M.problem_to_device(W.lognormal_problem(96, 8, 96, 16))
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        t = M.moray_trace_async(ctx, [big])
        early = M.moray_query(ctx, t, 0)
        busy = None
        if early is None:
            # the context refuses one-shot solves while serving
            try:
                M.moray_trace(ctx, [big])
            except M.MorayError as e:
                busy = e.status
        res = M.moray_query(ctx, t, -1)
        assert res is not None and res[0]["segments"] > 0
        if early is None and busy is not None:
            assert busy == M.MORAY_EBUSY
        # a finished ticket is forgotten
        assert lib.moray_query(ctx, ctypes.c_ulonglong(t.handle), 0) == M.MORAY_EINVAL
        assert lib.moray_query(ctx, ctypes.c_ulonglong(987654321), 0) == M.MORAY_EINVAL
        # the context serves one-shot solves again once idle
        assert M.moray_trace(ctx, [M.problem_to_device(W.lognormal_problem(96, 9, 16, 1))])[0]["segments"] > 0
    finally:
        M.moray_free(ctx)


def test_overflow_alone_fails_only_its_ticket():
    # a 4096-ray queue: the 32^3 problem (16 trees) cannot fit even alone,
    # the 8^3 one (1 tree, phi_c 0.5: at most 12 * 4^4 = 3072 rays per level) can
    big = M.problem_to_device(W.lognormal_problem(98, 0, 32, 4))
    small = M.problem_to_device(W.lognormal_problem(98, 1, 8, 1, energies=(13.6,),
                                                    params=W.Params(level_init=0, phi_c=0.5)))
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64, queue_capacity=4096)
    ref = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        alone = M.moray_trace(ref, [small])[0]
        tb = M.moray_trace_async(ctx, [big])
        ts = M.moray_trace_async(ctx, [small])
        with pytest.raises(M.MorayError) as e:
            M.moray_query(ctx, tb, -1)
        assert e.value.status == M.MORAY_EQUEUE
        _same(M.moray_query(ctx, ts, -1)[0], alone, 1e-9, "after overflow")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)


def test_cancel_and_deadline_leave_other_requests_intact():
    """A long anchor request cancelled from the host, and another that passes
    its deadline, leave at a launch boundary with MORAY_ECANCELED and
    MORAY_ETIMEOUT; small requests running beside them complete with their
    solo results, and the engine serves new requests afterwards (on the tree
    slots and memory the removed requests gave back)."""
    anchor = M.problem_to_device(W.lognormal_problem(96, 20, 256, 32))
    small = [M.problem_to_device(W.lognormal_problem(96, 21 + i, 32, 3)) for i in range(3)]
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ref = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        alone = [M.moray_trace(ref, [p])[0] for p in small]
        t_anchor = M.moray_trace_async(ctx, [anchor])
        t_small = M.moray_trace_async(ctx, [small[0]])
        time.sleep(0.003)
        M.moray_cancel(ctx, t_anchor)
        _same(M.moray_query(ctx, t_small, -1)[0], alone[0], 1e-9, "beside a cancelled request")
        with pytest.raises(M.MorayError) as e:
            M.moray_query(ctx, t_anchor, -1)
        assert e.value.status == M.MORAY_ECANCELED
        t_anchor = M.moray_trace_async(ctx, [anchor])
        M.moray_set_deadline(ctx, t_anchor, 0.002)
        t_small = M.moray_trace_async(ctx, [small[1]])
        _same(M.moray_query(ctx, t_small, -1)[0], alone[1], 1e-9, "beside a timed-out request")
        with pytest.raises(M.MorayError) as e:
            M.moray_query(ctx, t_anchor, -1)
        assert e.value.status == M.MORAY_ETIMEOUT
        # a finished ticket keeps its status when cancelled late; unknown tickets are rejected
        t_small = M.moray_trace_async(ctx, [small[2]])
        got = M.moray_query(ctx, t_small, -1)
        _same(got[0], alone[2], 1e-9, "after the removed requests")
        lib = M.load_library()
        assert lib.moray_cancel(ctx, ctypes.c_ulonglong(987654321)) == M.MORAY_EINVAL
        assert lib.moray_set_deadline(ctx, ctypes.c_ulonglong(987654321), 1.0) == M.MORAY_EINVAL
        t_late = M.moray_trace_async(ctx, [small[0]])
        time.sleep(0.5)                                   # a 32^3 solve takes a few milliseconds
        assert lib.moray_cancel(ctx, ctypes.c_ulonglong(t_late.handle)) == M.MORAY_OK
        _same(M.moray_query(ctx, t_late, -1)[0], alone[0], 1e-9, "cancelled after it finished")
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)


def test_admission_share_recovers_after_an_overflow(monkeypatch):
    """An overflow (injected into the first launch that runs several problems)
    restarts them with half the queue share, so fewer are admitted at once;
    clean launches restore the share, and a later burst is admitted together
    again. Every result equals its solo run."""
    probs = [M.problem_to_device(W.lognormal_problem(96, 30 + i, 24, 3)) for i in range(8)]
    # the admission estimate of one such problem is 12006 rays per tree x 12
    # trees; a queue where four fit in 0.75 of it but not in half of that
    bound = 12006 * 12
    monkeypatch.setenv("MORAY_INJECT_SERVE_OVERFLOW", "1")
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64, queue_capacity=int(4 * bound / 0.6))
    monkeypatch.delenv("MORAY_INJECT_SERVE_OVERFLOW")
    ref = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        alone = [M.moray_trace(ref, [p])[0] for p in probs]
        first = M.moray_query(ctx, M.moray_trace_async(ctx, probs[:4]), -1)
        second = M.moray_query(ctx, M.moray_trace_async(ctx, probs[4:]), -1)
        for i, r in enumerate(first + second):
            _same(r, alone[i], 1e-9, f"overflow recovery p{i}")
        admits1 = sorted({r["t_admit"] for r in first})
        admits2 = sorted({r["t_admit"] for r in second})
        print(f"admission times after the overflow: {len(admits1)} distinct; later burst: {len(admits2)}", flush=True)
        assert len(admits1) >= 2          # the restart admitted them in smaller groups
        assert len(admits2) == 1          # the later burst went in together
    finally:
        M.moray_free(ctx)
        M.moray_free(ref)
