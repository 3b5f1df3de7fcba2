"""Captured launch sequences and the autotuner, on the GPU.

* Repeated one-shot solves of the same descriptors (device fields and
  results): the second call captures the launch sequence in a HIP graph, the
  later ones replay it. Every replay is checked against an eager solve of the
  same inputs on another context (counts exactly, k_ph to 1e-9), with eager
  torch work and synchronisations between replays, and with the field values
  changed in place between replays.
* moray_autotune picks settings from its candidate lists, and solves with
  them still match the oracle-checked default settings exactly in counts.
* a PreparedBatch (descriptors built once) replays the captured sequence
  and returns what moray_trace returns for the same inputs.
* moray_autotune_cached: a miss tunes and appends one line; a new context
  (a later process) takes the same settings from the file without timing;
  another batch shape misses; malformed or out-of-range lines are ignored;
  an unwritable path fails before anything changes.
"""
import numpy as np
import pytest
import torch

from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

COUNTS = ("segments", "splits", "rays_seeded", "rays_escaped", "rays_truncated")


def _cmp(got, want, name, tol=1e-9):
    for k in COUNTS:
        assert got[k] == want[k], (name, k, got[k], want[k])
    for f in ("k_ph", "heating"):
        a = got[f][0].detach().cpu().numpy().ravel()
        b = want[f][0].detach().cpu().numpy().ravel()
        m = b > 1e-6 * b.max()
        rel = float(np.max(np.abs(a[m] - b[m]) / b[m]))
        print(f"[{name}] {f} max rel vs eager {rel:.2e}", flush=True)
        assert rel <= tol, (name, f, rel)


@pytest.mark.parametrize("precision", [M.MORAY_FP32_ACC64, M.MORAY_FP64])
def test_graph_replays_match_eager(precision):
    p = M.problem_to_device(W.lognormal_problem(97, 0, 40, 3))
    ncell = 40 ** 3
    outs = [(torch.empty(ncell, dtype=torch.float64, device="cuda"),
             torch.empty(ncell, dtype=torch.float64, device="cuda"))]
    ctx = M.moray_init(device=0, precision=precision)
    eager = M.moray_init(device=0, precision=precision)
    try:
        seen = []
        for call in range(6):
            if call == 4:
                # new field values, same pointers: the replay must read them
                p.grids[0].n_h.mul_(1.5)
                p.grids[0].x_hi.mul_(0.9)
            junk = torch.randn(1 << 20, device="cuda")
            float(junk.square().sum())
            torch.cuda.synchronize()
            got = M.moray_trace(ctx, [p], outputs=outs)[0]
            seen.append(got["from_graph"])
            want = M.moray_trace(eager, [p])[0]
            _cmp(got, want, f"prec {precision} call {call}")
        print(f"from_graph per call: {seen}", flush=True)
        assert seen[:2] == [0, 0] and all(seen[2:])
        # another descriptor set drops the graph; coming back captures again
        other = M.problem_to_device(W.lognormal_problem(97, 1, 24, 1))
        assert M.moray_trace(ctx, [other])[0]["from_graph"] == 0
        assert M.moray_trace(ctx, [p], outputs=outs)[0]["from_graph"] == 0
    finally:
        M.moray_free(ctx)
        M.moray_free(eager)


def test_autotune_settings_and_results():
    probs = [M.problem_to_device(W.lognormal_problem(97, 2 + i, n, s))
             for i, (n, s) in enumerate([(48, 3), (32, 2), (64, 1)])]
    base = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        want = M.moray_trace(base, probs)
        r = M.moray_autotune(ctx, probs)
        print(f"autotune: {r}", flush=True)
        assert r["chunk_rays"] in (128, 256, 512, 1024)
        assert r["refill_lanes"] in (8, 16, 24, 64)
        assert r["reserve_rays"] in (0, 64, 128, 256)
        assert r["waves_per_cu"] % 4 == 0 and r["waves_per_cu"] >= 4
        assert 0.0 < r["best_ms"] <= r["first_ms"] and r["trials"] >= 1
        got = M.moray_trace(ctx, probs)
        for i in range(len(probs)):
            _cmp(got[i], want[i], f"tuned p{i}")
    finally:
        M.moray_free(ctx)
        M.moray_free(base)


def test_prepared_batch_equals_moray_trace():
    probs = [M.problem_to_device(W.lognormal_problem(97, 20 + i, n, s)) for i, (n, s) in enumerate([(32, 2), (24, 1)])]
    outs = [(torch.empty(int(p.grids[0].n_h.numel()), dtype=torch.float64, device="cuda"),
             torch.empty(int(p.grids[0].n_h.numel()), dtype=torch.float64, device="cuda")) for p in probs]
    eager = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        want = M.moray_trace(eager, probs)
        batch = M.PreparedBatch(probs, outputs=outs)
        for call in range(3):
            got = M.moray_trace_prepared(ctx, batch)
            assert got[0]["from_graph"] == (1 if call == 2 else 0)
            for i in range(len(probs)):
                _cmp(got[i], want[i], f"prepared call {call} p{i}")
                assert got[i]["k_ph"][0].data_ptr() == outs[i][0].data_ptr()
    finally:
        M.moray_free(ctx)
        M.moray_free(eager)


def test_autotune_cache_file(tmp_path):
    probs = [M.problem_to_device(W.lognormal_problem(97, 2 + i, n, s))
             for i, (n, s) in enumerate([(48, 3), (32, 2)])]
    other = [M.problem_to_device(W.lognormal_problem(97, 9, 40, 1))]
    path = tmp_path / "tune.txt"
    path.write_text("not a tuning line\n")
    ctxs = [M.moray_init(device=0, precision=M.MORAY_FP32_ACC64) for _ in range(3)]
    try:
        a = M.moray_autotune(ctxs[0], probs, max_trials=4, cache_path=str(path))
        assert a["from_cache"] is False and 1 <= a["trials"] <= 4
        lines = path.read_text().splitlines()
        assert len(lines) == 2 and lines[1].startswith("moray-tune-1 ")
        b = M.moray_autotune(ctxs[1], probs, cache_path=str(path))
        assert b["from_cache"] is True
        for k in ("chunk_rays", "refill_lanes", "reserve_rays", "waves_per_cu", "trials"):
            assert b[k] == a[k], k
        assert b["best_ms"] == pytest.approx(a["best_ms"], rel=1e-5)
        # the cached settings are the ones the context now runs with: same counts as the tuned context
        want, got = M.moray_trace(ctxs[0], probs), M.moray_trace(ctxs[1], probs)
        for i in range(len(probs)):
            _cmp(got[i], want[i], f"cached p{i}")
        # an out-of-range line with the same key appended later is ignored
        f = lines[1].split(" ")
        bad = " ".join(f[:7] + ["512", "99", "0", "12"] + f[11:])
        with open(path, "a") as fh:
            fh.write(bad + "\n")
        c = M.moray_autotune(ctxs[1], probs, cache_path=str(path))
        assert c["from_cache"] is True and c["refill_lanes"] == a["refill_lanes"]
        # another shape misses and appends its own line
        d = M.moray_autotune(ctxs[2], other, max_trials=2, cache_path=str(path))
        assert d["from_cache"] is False
        assert len(path.read_text().splitlines()) == 4
        with pytest.raises(M.MorayError) as e:
            M.moray_autotune(ctxs[2], other, cache_path=str(tmp_path / "no_such_dir" / "t.txt"))
        assert e.value.status == M.MORAY_EINVAL
    finally:
        for c in ctxs:
            M.moray_free(c)


def test_failed_capture_falls_back_to_eager(monkeypatch):
    """A capture that fails (injected at the second call, where the library
    would capture) still returns MORAY_OK with the eager results; later calls
    capture and replay as usual."""
    p = M.problem_to_device(W.lognormal_problem(97, 3, 32, 2))
    outs = [(torch.empty(32 ** 3, dtype=torch.float64, device="cuda"),
             torch.empty(32 ** 3, dtype=torch.float64, device="cuda"))]
    monkeypatch.setenv("MORAY_INJECT_CAPTURE_FAILURE", "1")
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    monkeypatch.delenv("MORAY_INJECT_CAPTURE_FAILURE")
    eager = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        want = M.moray_trace(eager, [p])[0]
        seen = []
        for call in range(6):
            got = M.moray_trace(ctx, [p], outputs=outs)[0]
            seen.append(got["from_graph"])
            _cmp(got, want, f"injected capture failure, call {call}")
        print(f"from_graph per call: {seen}", flush=True)
        assert seen[1] == 0                      # the failed capture ran eagerly
        assert seen[-1] == 1                     # and graphs work again afterwards
    finally:
        M.moray_free(ctx)
        M.moray_free(eager)
