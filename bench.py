#!/usr/bin/env python3
"""Throughput benchmark of the adaptive ray tracer on one MI355X.

A step is one full single-pass trace (absorber columns, seeding, every
HEALPix level's march/split/deposit, finalize) of one synthetic batch whose
fields are already resident in HBM. The headline workload is the batched one:
64 independent lognormal grids (edges 32-96, 1-8 sources each) traced in one
call, in the float32-geometry / float64-accumulate mode, with launch settings
chosen by the library's autotuner for this batch and the launch sequence
replayed from its HIP graph. `value` is ray-cell segments per second over the
timed steps (wall clock around the steps, including each call's read-back of
its totals). Beside it: the plain float64 form (the same 64 problems, one
problem per call, planned and launched anew every call, no graph), the
trace kernel's roofline, the CPU oracle on all 64 problems, the 128^3
single-problem workload, the nested 256^3 + 128^3 workload, a serving sweep
over arrival rates, and the optional physics rows.

  python bench.py [--steps K] [--warmup W] [--workload c2|c1|c4] [--settings C,R,S,W]
  python bench.py --serve-only [--serve-rates 10,50,...] [--serve-requests N]
  python bench.py --equilibrium-only | --evolve-only | --covering-only | --radpres-only | --td-only | --thin-only
  python bench.py --counter-pass [--workload c2] [--counter-variant plain|radpres|td]   (under rocprofv3 --pmc)
  python bench.py --read-atomics ATOMIC_DIR LAUNCHES
  python bench.py --write-traffic FETCH_DIR WRITE_DIR LAUNCHES [--workload c2]
  python bench.py --write-atomics ATOMIC_DIR LAUNCHES [--workload c2] [--counter-variant radpres|td]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-cell segments/s on 1 MI355X (batched FP32 vs plain FP64); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SEGMENT = {"fp32": 36, "fp64": 40}     # absorber read + two float64 read-modify-writes
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_trace_level.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1012_2865_amd", "csrc", "moray_kernels.hip")
COPY_BYTES = 1 << 30                              # calibration copy of the counter pass
MICROBENCH_LIB = os.path.join(ROOT, "paper_1012_2865_amd", "libmoray_microbench.so")


MB_KINDS = {"atomics": 0, "copy": 1, "copy_nt": 2, "read": 3, "read_nt": 4}
MB_MIB = 1 << 20


def _microbench():
    import ctypes
    if not os.path.exists(MICROBENCH_LIB):
        return None
    lib = ctypes.CDLL(MICROBENCH_LIB)
    lib.moray_microbench.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.moray_microbench.restype = ctypes.c_int
    lib.moray_microbench_case.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.moray_microbench_case.restype = ctypes.c_int
    return lib


def _microbench_sweep(lib):
    """Every point of the device-peak sweep: float64 atomics over array sizes
    128 MiB - 1 GiB, 2-32 blocks per CU, 16-256 adds per thread, with every
    lane scattered (runs of 1) and with each wave one run of 64 cells, then
    the run length 1-64 at the best scattered shape; streaming copies and
    reads of 512 MiB - 4 GiB (beyond the 256 MiB last-level cache) with 1-16
    blocks per CU and 1-8 16-byte loads in flight per lane, plain and
    non-temporal. Returns a list of dicts."""
    import ctypes
    rows = []

    def one(kind, size, bpc, per, group=1):
        r = ctypes.c_double(0.0)
        rc = lib.moray_microbench_case(0, MB_KINDS[kind], size, bpc, per, group, ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"microbenchmark case {kind} {size} {bpc} {per} {group}: error {rc}")
        rows.append({"kind": kind, "MiB": size // MB_MIB, "blocks_per_cu": bpc, "per_thread": per,
                     "group": group, "rate": r.value})
        return r.value

    for group in (1, 64):
        for size in (128, 256, 512, 1024):
            for bpc in (2, 4, 8, 16, 32):
                for per in (16, 64, 256):
                    one("atomics", size * MB_MIB, bpc, per, group)
    best = max((r for r in rows if r["group"] == 1), key=lambda r: r["rate"])
    for group in (2, 4, 8, 16, 32):
        one("atomics", best["MiB"] * MB_MIB, best["blocks_per_cu"], best["per_thread"], group)
    for kind in ("copy", "copy_nt", "read", "read_nt"):
        for size in (512, 1024, 2048, 4096):
            for bpc in (1, 2, 4, 8, 16):
                for per in (1, 2, 4, 8):
                    one(kind, size * MB_MIB, bpc, per)
    return rows


def _device_peaks(sweep=True):
    """Float64 atomic rates and streaming bandwidths measured on the device
    by the project's microbenchmark: with `sweep`, the maximum of every
    pattern over the sweep and the shape that reached it (the fixed shape of
    `moray_microbench` is reported beside it); None when it is not built."""
    import ctypes
    lib = _microbench()
    if lib is None:
        return None
    out = (ctypes.c_double * 3)()
    if lib.moray_microbench(0, out) != 0:
        return None
    fixed = {"atomics_scattered": out[0], "atomics_coherent": out[1], "copy_GBs": out[2]}
    if not sweep:
        return fixed
    rows = _microbench_sweep(lib)

    def top(pred):
        r = max((r for r in rows if pred(r)), key=lambda r: r["rate"])
        return r["rate"], {k: r[k] for k in ("MiB", "blocks_per_cu", "per_thread", "group")}

    sc, sc_at = top(lambda r: r["kind"] == "atomics" and r["group"] == 1)
    co, co_at = top(lambda r: r["kind"] == "atomics")
    cp, cp_at = top(lambda r: r["kind"] in ("copy", "copy_nt"))
    rd, rd_at = top(lambda r: r["kind"] in ("read", "read_nt"))
    return {"atomics_scattered": sc, "atomics_coherent": co, "copy_GBs": cp, "read_GBs": rd,
            "at": {"atomics_scattered": sc_at, "atomics_coherent": co_at, "copy_GBs": cp_at, "read_GBs": rd_at},
            "fixed_shape": fixed, "sweep_points": len(rows),
            "source": "maxima of the microbenchmark sweep run in this process"}


def _microbench_table():
    """The sweep condensed to markdown (what profiles/ keeps): the best rate of
    every pattern and the shape that reached it, the scattered-atomic rate by
    array size and blocks per CU, and each streaming pattern by blocks per CU
    and loads in flight."""
    lib = _microbench()
    if lib is None:
        raise SystemExit("libmoray_microbench.so is not built")
    rows = _microbench_sweep(lib)

    def best(pred):
        sel = [r for r in rows if pred(r)]
        return max(sel, key=lambda r: r["rate"]) if sel else None

    out = [f"{len(rows)} sweep points.", "", "| pattern | best rate | MiB | blocks/CU | per thread | run |",
           "|---|---:|---:|---:|---:|---:|"]
    for run in (1, 2, 4, 8, 16, 32, 64):
        b = best(lambda r: r["kind"] == "atomics" and r["group"] == run)
        if b:
            out.append(f"| float64 atomics, runs of {run} | {b['rate']:.3e}/s | {b['MiB']} | {b['blocks_per_cu']} | "
                       f"{b['per_thread']} | {run} |")
    for kind in ("copy", "copy_nt", "read", "read_nt"):
        b = best(lambda r: r["kind"] == kind)
        out.append(f"| {kind} | {b['rate']:.0f} GB/s | {b['MiB']} | {b['blocks_per_cu']} | {b['per_thread']} | |")
    sizes = sorted({r["MiB"] for r in rows if r["kind"] == "atomics"})
    bpcs = sorted({r["blocks_per_cu"] for r in rows if r["kind"] == "atomics"})
    out += ["", "Scattered float64 atomics (runs of 1), best over adds per thread, 1e10/s:", "",
            "| MiB \\ blocks/CU | " + " | ".join(str(b) for b in bpcs) + " |", "|---|" + "---:|" * len(bpcs)]
    for m in sizes:
        cells = [best(lambda r: r["kind"] == "atomics" and r["group"] == 1 and r["MiB"] == m and
                      r["blocks_per_cu"] == b) for b in bpcs]
        out.append(f"| {m} | " + " | ".join(f"{c['rate'] / 1e10:.2f}" if c else "" for c in cells) + " |")
    for kind in ("copy", "copy_nt", "read", "read_nt"):
        pers = sorted({r["per_thread"] for r in rows if r["kind"] == kind})
        bp = sorted({r["blocks_per_cu"] for r in rows if r["kind"] == kind})
        out += ["", f"{kind}, best over array sizes, GB/s (rows: blocks per CU; columns: 16-byte loads in flight "
                    f"per lane):", "", "| blocks/CU \\ loads | " + " | ".join(str(p) for p in pers) + " |",
                "|---|" + "---:|" * len(pers)]
        for b in bp:
            cells = [best(lambda r: r["kind"] == kind and r["blocks_per_cu"] == b and r["per_thread"] == p)
                     for p in pers]
            out.append(f"| {b} | " + " | ".join(f"{c['rate']:.0f}" for c in cells) + " |")
    print("\n".join(out))


def _workload(name):
    from paper_1012_2865_amd import workloads as W
    common = {"groups": [13.6, 20.0, 30.0, 60.0], "phi_c": 5.1, "level_init": 1, "level_max": 14, "p_min_frac": 1e-8}
    if name == "c1":
        return [W.config1()], {"workload": "lognormal128_16src_4grp", "grid": "128^3", "box_kpc": 2.0,
                               "sources": 16, **common}
    if name == "c2":
        probs = W.config2(64)
        return probs, {"workload": "batched64_lognormal_32-96", "problems": 64,
                       "cells": int(sum(p.n_cells for p in probs)),
                       "sources": int(sum(p.n_sources for p in probs)), **common}
    if name == "c4":
        p = W.config4()
        return [p], {"workload": "nested256+128_1000src_4grp", "grids": "256^3 root + 128^3 child (2x)",
                     "box_kpc": 4.0, "sources": 1000, "clusters": 10, **common}
    raise ValueError(name)


def _parse_settings(text):
    """--settings chunk,refill,reserve,waves (launch settings to use instead
    of running the autotuner)."""
    c, r, s, w = (int(x) for x in text.split(","))
    return {"chunk_rays": c, "refill_lanes": r, "reserve_rays": s, "waves_per_cu": w, "source": "--settings"}


def _outputs(dev):
    """Result buffers per problem (k_ph, heating), flat float64 on the device."""
    import torch
    out = []
    for p in dev:
        n = sum(int(g.n_h.numel()) for g in p.grids)
        out.append((torch.empty(n, dtype=torch.float64, device="cuda"),
                    torch.empty(n, dtype=torch.float64, device="cuda")))
    return out


def _time_steps(M, ctx, dev, steps, warmup, graph=True):
    """Seconds per step. graph=True reuses one set of result buffers, so from
    the third call on the library replays its captured launch sequence;
    graph=False alternates two sets, so every call plans and launches anew."""
    import torch
    sets = [_outputs(dev), _outputs(dev)] if not graph else [_outputs(dev)]
    # the descriptors are built once per buffer set, as a caller that steps the
    # same batch repeatedly does (fields stay resident; nothing is skipped)
    batches = [M.PreparedBatch(dev, outputs=o) for o in sets]
    res = None
    for i in range(warmup):
        res = M.moray_trace_prepared(ctx, batches[i % len(batches)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        res = M.moray_trace_prepared(ctx, batches[(warmup + i) % len(batches)])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    segs = sum(r["segments"] for r in res)
    return dt / steps, segs, res


def _tuned(M, precision, dev, settings=None):
    """A context whose launch settings the autotuner chose for this batch
    (or the given settings)."""
    if settings:
        ctx = M.moray_init(device=0, precision=precision, chunk_rays=settings["chunk_rays"],
                           refill_lanes=settings["refill_lanes"], reserve_rays=settings["reserve_rays"],
                           waves_per_cu=settings["waves_per_cu"])
        return ctx, dict(settings)
    ctx = M.moray_init(device=0, precision=precision)
    tune = M.moray_autotune(ctx, dev)
    tune["source"] = "moray_autotune"
    return ctx, tune


def _kernel_time(M, precision, dev, tune, reps=3):
    """Summed trace-kernel device time per step, measured with HIP events on
    the library's stream, with the launch settings of the timed form."""
    ctx = M.moray_init(device=0, precision=precision, profile=True, chunk_rays=tune["chunk_rays"],
                       refill_lanes=tune["refill_lanes"], waves_per_cu=tune["waves_per_cu"],
                       reserve_rays=tune["reserve_rays"])
    try:
        M.moray_trace(ctx, dev)
        ms, launches, segs = 0.0, 0, 0
        for _ in range(reps):
            res = M.moray_trace(ctx, dev)
            ms += res[0]["trace_ms"]
            launches += res[0]["trace_launches"]
            segs += sum(r["segments"] for r in res)
        return ms / reps, launches / reps, segs / reps
    finally:
        M.moray_free(ctx)


def _traffic(workload, precision):
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    key = f"{workload}/{precision}"
    if rec.get("kernel_sha256") != sha or key not in rec.get("per_launch_bytes", {}):
        return None
    return rec["per_launch_bytes"][key]


def _counter_pass(workload, variant="plain", settings=None):
    """One warm-up and one measured fp32 trace of the workload (with the
    given launch settings, else the autotuner's for it, else for "c1" the
    library defaults), then a 1 GiB device-to-device copy whose counter
    readings calibrate FETCH_SIZE and WRITE_SIZE, and the device-peak
    microbenchmark whose known atomic count calibrates TCC_EA0_ATOMIC. Meant
    to run under `rocprofv3 --pmc`. The variant "radpres" traces with the
    radiation-pressure sums; "td" runs six time-dependent steps (c dt_P = 32
    cells), the last of which is the measured one; "thin" traces the 128^3
    workload in ionised gas with the optically-thin approximation."""
    import torch
    from paper_1012_2865_amd import moray as M
    from paper_1012_2865_amd import workloads as W
    problems, config = _workload(workload)
    if variant == "thin":
        if workload != "c1":
            raise SystemExit("the thin variant's counter pass runs on the 128^3 workload (--workload c1)")
        problems = [W.config1_ionised(0.1)]
        config = {"workload": problems[0].name}
    dev = [M.problem_to_device(p) for p in problems]
    if settings is None and workload == "c1":
        ctx, settings = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64), {"source": "library defaults"}
    else:
        ctx, settings = _tuned(M, M.MORAY_FP32_ACC64, dev, settings)
    try:
        if variant == "td":
            td = M.moray_td_create(ctx, dev[0], 32.0, 1 << 25)
            try:
                for _ in range(6):
                    res = [M.moray_td_step(ctx, td, dev[0])[0]]
            finally:
                M.moray_td_free(ctx, td)
        else:
            accel = variant == "radpres"
            M.moray_trace(ctx, dev, want_accel=accel)
            res = M.moray_trace(ctx, dev, want_accel=accel)
    finally:
        M.moray_free(ctx)
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    peaks = _device_peaks(sweep=False)     # its scattered-atomics kernel calibrates the atomic counter
    print(json.dumps({"counter_pass": config["workload"], "variant": variant, "settings": settings,
                      "segments": sum(r["segments"] for r in res),
                      "launches_per_trace": res[0]["trace_launches"], "copy_bytes": COPY_BYTES,
                      "peaks": peaks}), flush=True)


def _read_counter_csv(folder, counter):
    """Per-dispatch values of one counter from a rocprofv3 --pmc output folder,
    in dispatch order: list of (kernel name, value in KiB)."""
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def _write_traffic(fetch_dir, write_dir, workload, launches, variant="plain"):
    """Turn two counter passes into HBM bytes per trace-kernel launch. The
    trace kernel's dispatches of the second (measured) trace are averaged; the
    1 GiB copy's reading calibrates KiB per byte moved."""
    rec = {"kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest(), "per_launch_bytes": {}}
    if os.path.exists(TRAFFIC_FILE):
        old = json.load(open(TRAFFIC_FILE))
        if old.get("kernel_sha256") == rec["kernel_sha256"]:
            rec = old
    out = {}
    for name, folder, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _read_counter_csv(folder, counter)
        trace = [v for k, v in rows if "trace_level_kernel" in k]
        if len(trace) < 2 * launches:
            raise SystemExit(f"{folder}: {len(trace)} trace dispatches, expected {2 * launches}")
        measured = trace[len(trace) - launches:]
        other = [v for k, v in rows if "moray" not in k]
        copy_kib = max(other)
        factor = COPY_BYTES / (copy_kib * 1024.0)
        out[name] = {"kib_per_launch": sum(measured) / launches, "copy_kib": copy_kib, "bytes_per_byte": factor,
                     "bytes_per_launch": sum(measured) / launches * 1024.0 * factor}
    key = f"{workload}/fp32" if variant == "plain" else f"{workload}/fp32/{variant}"
    rec["per_launch_bytes"][key] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    rec.setdefault("detail", {})[key] = out
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(out, indent=1))


def _atomic_calibration(atomic_dir):
    """Atomics per count of TCC_EA0_ATOMIC_sum, from the microbenchmark's
    scattered-atomics dispatch (64 float64 atomics per thread of its grid)."""
    import csv
    import glob
    scattered = [v for k, v in _read_counter_csv(atomic_dir, "TCC_EA0_ATOMIC_sum") if "atomics_scattered" in k]
    grid = 0
    for f in glob.glob(os.path.join(atomic_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if "atomics_scattered" in r["Kernel_Name"]:
                grid = int(r["Grid_Size"])
    known = grid * 64
    return (known / scattered[-1] if (scattered and known) else 1.0), (scattered[-1] if scattered else None), known


def _read_atomics(atomic_dir, launches):
    """Float64 atomics per trace-kernel launch over the last `launches`
    trace dispatches of a TCC_EA0_ATOMIC_sum pass (no record is written)."""
    trace = [v for k, v in _read_counter_csv(atomic_dir, "TCC_EA0_ATOMIC_sum") if "trace_level_kernel" in k]
    if len(trace) < launches:
        raise SystemExit(f"{atomic_dir}: {len(trace)} trace dispatches, expected at least {launches}")
    factor, _, _ = _atomic_calibration(atomic_dir)
    last = trace[len(trace) - launches:]
    return {"atomics_per_trace": sum(last) * factor, "per_launch": [v * factor for v in last],
            "atomics_per_count": factor}


def _write_atomics(atomic_dir, workload, launches, variant="plain"):
    """Float64 atomics per trace-kernel launch from a TCC_EA0_ATOMIC_sum pass.
    The microbenchmark's timed scattered-atomics dispatch (64 atomics per
    thread of its grid) calibrates the counter."""
    import csv
    import glob
    rows = _read_counter_csv(atomic_dir, "TCC_EA0_ATOMIC_sum")
    trace = [v for k, v in rows if "trace_level_kernel" in k]
    if len(trace) < 2 * launches:
        raise SystemExit(f"{atomic_dir}: {len(trace)} trace dispatches, expected {2 * launches}")
    scattered = [v for k, v in rows if "atomics_scattered" in k]
    grid = 0          # threads of the scattered-atomics dispatch; each issues 64 atomics
    for f in glob.glob(os.path.join(atomic_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if "atomics_scattered" in r["Kernel_Name"]:
                grid = int(r["Grid_Size"])
    known = grid * 64
    factor = known / scattered[-1] if (scattered and known) else 1.0
    per_launch = sum(trace[len(trace) - launches:]) / launches * factor
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != sha:
        raise SystemExit("the traffic record belongs to another kernel source; write the traffic first")
    key = f"{workload}/fp32" if variant == "plain" else f"{workload}/fp32/{variant}"
    rec.setdefault("atomics_per_launch", {})[key] = per_launch
    rec.setdefault("detail", {}).setdefault(key, {})["atomics"] = {
        "counter_per_launch": sum(trace[len(trace) - launches:]) / launches,
        "microbench_counter": scattered[-1] if scattered else None, "microbench_atomics": known,
        "atomics_per_count": factor}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"atomics_per_launch": per_launch, "atomics_per_count": factor}))


def _atomics_per_launch(workload, precision):
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != sha:
        return None
    return rec.get("atomics_per_launch", {}).get(f"{workload}/{precision}")


def _equilibrium_c1(M, updates=20, oracle_threads=0):
    """Photo-ionisation equilibrium iteration (moray_equilibrate) on the 128^3
    workload from neutral gas: `updates` damped updates, each a full trace plus
    the per-cell update, then the final trace. With oracle_threads, the
    oracle's harness is timed beside it on the first two updates."""
    import numpy as np
    import torch
    from paper_1012_2865_amd import workloads as W
    p = W.config1()
    p.grids[0].x_hi = np.ones_like(p.grids[0].x_hi)
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        M.moray_equilibrate(ctx, M.problem_to_device(p), tol=1e-30, max_iter=2)      # warm-up
        pd = M.problem_to_device(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.moray_equilibrate(ctx, pd, tol=1e-30, max_iter=2)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0
        pd = M.problem_to_device(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, done, _ = M.moray_equilibrate(ctx, pd, tol=1e-30, max_iter=updates)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        x = pd.grids[0].x_hi
    finally:
        M.moray_free(ctx)
    out = {"workload": "lognormal128_16src_4grp from neutral gas", "updates": done, "ms_total": dt * 1e3,
           "ms_per_trace": dt * 1e3 / (done + 1), "segments_final_trace": res["segments"],
           "ionised_fraction_final": float(1.0 - x.double().mean()), "dtype": "f32+f64acc"}
    if oracle_threads:
        from oracle import equilibrium as E
        t0 = time.perf_counter()
        E.iterate(p, tol=1e-30, max_iter=2, n_threads=oracle_threads)
        dto = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": dto / 2.0, "unit": "s per update (trace + update)", "cores": oracle_threads,
                             "kind": "oracle", "sample": f"the first two updates from neutral gas in {dto:.1f} s",
                             "gpu_same_sample_s_per_update": dt2 / 3.0, "gpu_speedup": dto / 2.0 / (dt2 / 3.0)}
    return out


def _covering_c1(M, steps, oracle_threads=0):
    """The 128^3 workload with the covering-factor correction of k_ph and
    heating switched on (section 2.3), mixed precision, beside the plain
    trace under the same launch settings."""
    import torch
    from paper_1012_2865_amd import workloads as W
    plain = W.config1()
    cov = W.config1()
    cov.params = W.Params(**{**cov.params.__dict__, "covering": True})
    dp, dc = [M.problem_to_device(plain)], [M.problem_to_device(cov)]
    torch.cuda.synchronize()
    ctx, _ = _tuned(M, M.MORAY_FP32_ACC64, dp)
    try:
        sp, segp, _ = _time_steps(M, ctx, dp, steps, 2)
        sc, segc, res = _time_steps(M, ctx, dc, steps, 2)
    finally:
        M.moray_free(ctx)
    out = {"workload": "lognormal128_16src_4grp with covering factor", "ms_per_step": sc * 1e3,
           "segments_per_s": segc / sc, "plain_ms_per_step": sp * 1e3, "overhead": sc / sp - 1.0,
           "absorbed_over_plain_emitted": res[0]["absorbed"] / res[0]["emitted"], "dtype": "f32+f64acc"}
    if oracle_threads:
        from oracle import oracle as O
        t0 = time.perf_counter()
        segs = O.trace(cov, n_threads=oracle_threads)["totals"]["segments"]
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": segs / dt, "unit": "segments/s", "cores": oracle_threads, "kind": "oracle",
                             "sample": f"full workload with the correction: {segs} segments in {dt:.1f} s",
                             "gpu_speedup": (segc / sc) / (segs / dt)}
    return out


def _evolve_test1(M, oracle_threads=0):
    """The paper's Test 1 (section 4.1) end to end on the device: a 5e48 ph/s
    source at the corner of a 6.6 kpc, 64^3 box of n_H = 1e-3, evolved for
    500 Myr with moray_evolve (eps_ion = 0.1, steps of at most t_rec / 400),
    mixed precision; the ionised volume's equivalent radius against
    R_s (1 - e^{-t/t_rec})^{1/3}."""
    import math
    import numpy as np
    import torch
    from paper_1012_2865_amd import workloads as W
    n, box, alpha = 64, 6.6 * W.KPC_CM, M.ALPHA_B
    t_rec, myr = 1.0 / (alpha * 1e-3), 3.15576e13

    def problem():
        g = W.uniform_grid(n, box / n, 1e-3, 1.0 - 1.2e-3)
        return M.problem_to_device(W.Problem([g], np.array([[0.0, 0.0, 0.0, 5e48]]), W.hydrogen_spectrum([13.6]),
                                             W.Params()))
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        M.moray_evolve(ctx, problem(), 10 * myr, dt_max=t_rec / 400)               # warm-up
        pd = problem()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, steps10, _, _, _ = M.moray_evolve(ctx, pd, 10 * myr, dt_max=t_rec / 400)
        torch.cuda.synchronize()
        dt10 = time.perf_counter() - t0
        pd = problem()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, steps, t, x64, _ = M.moray_evolve(ctx, pd, 500 * myr, dt_max=t_rec / 400, want_x64=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        x = x64.cpu().numpy()
    finally:
        M.moray_free(ctx)
    r = (6.0 * float(np.sum(1.0 - x)) * (box / n) ** 3 / math.pi) ** (1.0 / 3.0)
    rs = (3.0 * 5e48 / (4.0 * math.pi * alpha * 1e-6)) ** (1.0 / 3.0) * (1.0 - math.exp(-t / t_rec)) ** (1.0 / 3.0)
    out = {"workload": "Test 1 (64^3, 6.6 kpc, 5e48 ph/s) to 500 Myr", "steps": steps, "s_total": dt,
           "ms_per_step": dt * 1e3 / steps, "front_over_analytic": r / rs, "dtype": "f32+f64acc"}
    if oracle_threads:
        from oracle import evolve as EV
        g = W.uniform_grid(n, box / n, 1e-3, 1.0 - 1.2e-3)
        ph = W.Problem([g], np.array([[0.0, 0.0, 0.0, 5e48]]), W.hydrogen_spectrum([13.6]), W.Params())
        t0 = time.perf_counter()
        _, _, osteps, _, _ = EV.evolve(ph, 10 * myr, eps=0.1, dt_max=t_rec / 400, n_threads=oracle_threads)
        dto = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": dto * 1e3 / osteps, "unit": "ms per step", "cores": oracle_threads,
                             "kind": "oracle", "sample": f"the first 10 Myr: {osteps} steps in {dto:.1f} s",
                             "gpu_same_sample_ms_per_step": dt10 * 1e3 / steps10,
                             "gpu_speedup": (dto / osteps) / (dt10 / steps10)}
    return out


def _radpres_c1(M, steps, oracle_threads=0):
    """The 128^3 workload with the radiation-pressure acceleration (section
    2.5.4) asked for, mixed precision, beside the plain trace under the same
    launch settings and result buffers."""
    import torch
    from paper_1012_2865_amd import workloads as W
    dev = [M.problem_to_device(W.config1())]
    n = dev[0].grids[0].n_h.numel()
    outs = [(torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
             torch.empty(3 * n, dtype=torch.float64, device="cuda"))]
    torch.cuda.synchronize()
    ctx, _ = _tuned(M, M.MORAY_FP32_ACC64, dev)
    try:
        sp, _, _ = _time_steps(M, ctx, dev, steps, 2)
        res = None
        for i in range(2):
            res = M.moray_trace(ctx, dev, outputs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            res = M.moray_trace(ctx, dev, outputs=outs)
        torch.cuda.synchronize()
        sr = (time.perf_counter() - t0) / steps
    finally:
        M.moray_free(ctx)
    segs = res[0]["segments"]
    out = {"workload": "lognormal128_16src_4grp with radiation pressure", "ms_per_step": sr * 1e3,
           "segments_per_s": segs / sr, "plain_ms_per_step": sp * 1e3, "overhead": sr / sp - 1.0,
           "dtype": "f32+f64acc"}
    if oracle_threads:
        from oracle import oracle as O
        t0 = time.perf_counter()
        osegs = O.trace(W.config1(), n_threads=oracle_threads, want_accel=True)["totals"]["segments"]
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": osegs / dt, "unit": "segments/s", "cores": oracle_threads, "kind": "oracle",
                             "sample": f"full workload with the acceleration: {osegs} segments in {dt:.1f} s",
                             "gpu_speedup": (segs / sr) / (osegs / dt)}
    return out


THIN_BYTES_PER_SEGMENT = 5    # a thin segment: absorber read (4 B) + the mark (a 1 B store)


def _with_tau(p, tau):
    from paper_1012_2865_amd import workloads as W
    return W.Problem(p.grids, p.sources, p.spectrum, W.Params(**{**p.params.__dict__, "tau_thin": tau}), p.name)


def _thin_workloads(M, steps, peaks=None, oracle_threads=0):
    """The workloads of the optically-thin approximation (section 2.4): the
    128^3 lognormal workload with its neutral fractions scaled by 1e-3
    (ionised gas, thin out to tens of cells around each source) and the thin
    box of the angular-resolution test (section 7.2, 128^3), each traced with
    the approximation (tau_thin = 0.1) and without it, mixed precision,
    library defaults, graph replay; the thin launch sequence's roofline from
    HIP-event launch times (36 B per thick segment, 5 B per thin one)."""
    import torch
    out = {}
    settings = {"chunk_rays": 256, "refill_lanes": 64, "reserve_rays": 0, "waves_per_cu": 0}
    from paper_1012_2865_amd import workloads as W
    for p in (W.config1_ionised(), W.thin_box()):
        name = p.name
        thin, plain = [M.problem_to_device(_with_tau(p, 0.1))], [M.problem_to_device(p)]
        torch.cuda.synchronize()
        ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
        try:
            sp, segp, _ = _time_steps(M, ctx, plain, steps, 2)
            st, segt, res = _time_steps(M, ctx, thin, steps, 2)
        finally:
            M.moray_free(ctx)
        kms, launches, ksegs = _kernel_time(M, M.MORAY_FP32_ACC64, thin, settings)
        tsegs = res[0]["thin_segments"]
        algo = BYTES_PER_SEGMENT["fp32"] * (ksegs - tsegs) + THIN_BYTES_PER_SEGMENT * tsegs
        achieved = algo / (kms * 1e-3) / 1e9
        traffic = _traffic("c1", "fp32/thin") if name.startswith("ionised") else None
        apl = _atomics_per_launch("c1", "fp32/thin") if name.startswith("ionised") else None
        rec = {"workload": name, "ms_per_step": st * 1e3, "segments_per_step": segt, "thin_segments": tsegs,
               "segments_per_s": segt / st, "plain_ms_per_step": sp * 1e3, "plain_segments_per_step": segp,
               "speedup_over_plain": sp / st, "absorbed_over_emitted": res[0]["absorbed"] / res[0]["emitted"],
               "dtype": "f32+f64acc",
               "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                            "traffic_source": "FETCH_SIZE + WRITE_SIZE counter passes of this kernel source "
                                              "(--counter-variant thin), per launch, read from "
                                              "profiles/traffic_trace_level.json (null: none for this workload "
                                              "or kernel changed since)",
                            "float64_atomics_per_launch": apl,
                            "kernel": "trace_level_kernel<float, true, kPhysThin>", "launches_per_step": launches,
                            "avg_launch_ms": kms / launches if launches else None,
                            "algorithmic_bytes_per_launch": algo / launches if launches else None}}
        if oracle_threads:
            from oracle import oracle as O
            t0 = time.perf_counter()
            osegs = O.trace(_with_tau(p, 0.1), n_threads=oracle_threads)["totals"]["segments"]
            dt = time.perf_counter() - t0
            rec["cpu_oracle"] = {"value": osegs / dt, "unit": "segments/s", "cores": oracle_threads, "kind": "oracle",
                                 "sample": f"full workload with the approximation: {osegs} segments in {dt:.1f} s",
                                 "gpu_speedup": (segt / st) / (osegs / dt)}
        out[name] = rec
    return out


def _td_c1(M, steps=10, c_dt=32.0, oracle=False):
    """Time-dependent rays on the 128^3 workload (section 2.1): rays halt after
    c dt_P = 32 root cells per step and continue in the next; `steps` steps
    from an empty box, mixed precision, each timed on its own. The steps from
    the fifth on have every emission batch in flight."""
    import torch
    from paper_1012_2865_amd import workloads as W
    dev = M.problem_to_device(W.config1())
    n = dev.grids[0].n_h.numel()
    outs = [(torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"))]
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    td = None
    try:
        td = M.moray_td_create(ctx, dev, c_dt, 1 << 25)
        ms, segs, held = [], [], 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, held = M.moray_td_step(ctx, td, dev, outputs=outs)
            ms.append((time.perf_counter() - t0) * 1e3)
            segs.append(res["segments"])
    finally:
        if td:
            M.moray_td_free(ctx, td)
        M.moray_free(ctx)
    late = slice(4, steps)
    out = {"workload": "lognormal128_16src_4grp, time-dependent rays, c dt_P = 32 cells", "steps": steps,
           "ms_per_step": ms, "segments_per_step": segs, "held_after_last": held,
           "segments_per_s_late": sum(segs[late]) / (sum(ms[late]) * 1e-3), "dtype": "f32+f64acc"}
    if oracle:
        # the oracle's time-dependent step runs on one thread: three steps of two of the sources,
        # beside the GPU on the same sample
        from oracle import oracle as O
        sub = W.subset_sources(W.config1(), [3, 11])
        t0 = time.perf_counter()
        rays, osegs = None, 0
        for _ in range(3):
            ref, rays = O.trace_td(sub, c_dt, rays, out_cap=1 << 24)
            osegs += ref["totals"]["segments"]
        dt = time.perf_counter() - t0
        dsub = M.problem_to_device(sub)
        ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
        td = None
        try:
            td = M.moray_td_create(ctx, dsub, c_dt, 1 << 24)
            torch.cuda.synchronize()
            g0, gsegs = time.perf_counter(), 0
            for _ in range(3):
                gsegs += M.moray_td_step(ctx, td, dsub)[0]["segments"]
            torch.cuda.synchronize()
            gdt = time.perf_counter() - g0
        finally:
            if td:
                M.moray_td_free(ctx, td)
            M.moray_free(ctx)
        out["cpu_oracle"] = {"value": osegs / dt, "unit": "segments/s", "cores": 1, "kind": "oracle",
                             "sample": f"sources 3 and 11, steps 1-3: {osegs} segments in {dt:.1f} s",
                             "gpu_same_sample": gsegs / gdt, "gpu_speedup": (gsegs / gdt) / (osegs / dt)}
    return out


def _roofline(M, workload, dev, tune, peaks):
    """Roofline of the dominant kernel (trace_level_kernel<float>) under the
    timed form's launch settings: algorithmic bytes per launch (36 B per
    segment) over the average launch duration measured with HIP events on
    the library's stream. traffic and atomics come from the committed counter
    passes of the same kernel source (profiles/traffic_trace_level.json), or
    null when the kernel has changed since."""
    kms, launches, ksegs = _kernel_time(M, M.MORAY_FP32_ACC64, dev, tune)
    algo_bytes = BYTES_PER_SEGMENT["fp32"] * ksegs
    achieved = algo_bytes / (kms * 1e-3) / 1e9
    traffic = _traffic(workload, "fp32")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_source": "FETCH_SIZE + WRITE_SIZE counter passes of this kernel source, per launch, read from "
                              "profiles/traffic_trace_level.json (null: kernel changed since)",
            "kernel": "trace_level_kernel<float>", "launches_per_step": launches,
            "avg_launch_ms": kms / launches if launches else None,
            "algorithmic_bytes_per_launch": algo_bytes / launches if launches else None,
            "segments_per_step": ksegs}
    # the deposits' second bound: float64 atomics that reach the memory side
    # (evicted LDS sums), against the device's measured atomic peak
    apl = _atomics_per_launch(workload, "fp32")
    if peaks:
        rate = apl / (kms * 1e-3 / launches) if (apl and launches) else None
        roof["atomics"] = {"unit": "float64 atomics/s", "per_launch": apl,
                           "per_segment": apl * launches / ksegs if apl else None, "achieved": rate,
                           "peak": peaks["atomics_scattered"], "peak_coherent": peaks["atomics_coherent"],
                           "frac": rate / peaks["atomics_scattered"] if rate else None,
                           "source": "TCC_EA0_ATOMIC counter pass read from profiles/traffic_trace_level.json"}
        roof["copy_GBs_measured"] = peaks["copy_GBs"]
    return roof


def _plain_fp64(M, dev, steps):
    """The plain form: float64 path, one problem per call, every call planned
    and launched anew (alternating result buffers, so nothing replays)."""
    import torch
    ctx = M.moray_init(device=0, precision=M.MORAY_FP64)
    try:
        sets = [_outputs(dev), _outputs(dev)]
        for i, p in enumerate(dev[:4]):
            M.moray_trace(ctx, [p], outputs=[sets[0][i]])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seg64 = 0
        for rep in range(steps):
            seg64 = 0
            for i, p in enumerate(dev):
                seg64 += M.moray_trace(ctx, [p], outputs=[sets[rep % 2][i]])[0]["segments"]
        torch.cuda.synchronize()
        s64 = (time.perf_counter() - t0) / steps
    finally:
        M.moray_free(ctx)
    return {"value": seg64 / s64, "unit": "segments/s", "ms_per_step": s64 * 1e3, "segments": seg64,
            "dtype": "f64", "form": "one problem per call, no graph" if len(dev) > 1 else "one solve per call, no graph"}


def _single_workload(M, name, steps, peaks, cpu_threads=0):
    """A workload traced as one problem: the mixed form (default settings,
    graph replay) beside the float64 form, with its own roofline."""
    import torch
    problems, config = _workload(name)
    dev = [M.problem_to_device(p) for p in problems]
    torch.cuda.synchronize()
    settings = {"chunk_rays": 256, "refill_lanes": 64, "reserve_rays": 0, "waves_per_cu": 0,
                "source": "library defaults"}
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        s32, seg32, res = _time_steps(M, ctx, dev, steps, 2)
    finally:
        M.moray_free(ctx)
    out = {"workload": config["workload"], "config": config, "value": seg32 / s32, "unit": "segments/s",
           "ms_per_step": s32 * 1e3, "segments_per_step": seg32, "graph_replay": bool(res[0]["from_graph"]),
           "dtype": "f32+f64acc", "settings": settings,
           "plain_fp64": _plain_fp64(M, dev, max(1, steps // 2)),
           "roofline": _roofline(M, name, dev, settings, peaks)}
    out["fp32_over_fp64"] = out["value"] / out["plain_fp64"]["value"]
    if cpu_threads:
        v, dt, segs = _cpu_baseline(problems, cpu_threads)
        out["cpu_oracle"] = {"value": v, "unit": "segments/s", "cores": cpu_threads, "kind": "oracle",
                             "sample": f"full workload: {segs} segments in {dt:.1f} s"}
    return out


def _serving_c3(M, rate_hz, n_requests, horizon_s):
    """Config 3: Poisson arrivals of requests (edges 32-256, 1-32 sources,
    Ndot log-U[1e47, 1e51]) on device-resident pooled fields, submitted in
    real time to the serving engine. Latency = completion - arrival."""
    import numpy as np
    import torch
    from paper_1012_2865_amd import workloads as W
    pool, reqs = W.config3_pool(rate_hz, n_requests, horizon_s)
    dev_pool = {e: [M.problem_to_device(W.Problem([g], np.zeros((0, 4)), None, None)).grids[0] for g in gs]
                for e, gs in pool.items()}
    torch.cuda.synchronize()
    ctx = M.moray_init(device=0, precision=M.MORAY_FP32_ACC64)
    try:
        # the engine's pools are created by the first request
        M.moray_query(ctx, M.moray_trace_async(ctx, [W.pooled_problem(dev_pool, reqs[0])]), -1)
        t0 = time.monotonic()
        tickets = []
        for r in reqs:
            delay = t0 + r.arrival_s - time.monotonic()
            if delay > 0:
                time.sleep(delay)
            tickets.append((r, M.moray_trace_async(ctx, [W.pooled_problem(dev_pool, r)])))
        lat, segs, done = [], 0, []
        for r, t in tickets:
            res = M.moray_query(ctx, t, -1)[0]
            lat.append(res["t_done"] - (t0 + r.arrival_s))
            done.append(res["t_done"])
            segs += res["segments"]
        span = max(done) - t0
    finally:
        M.moray_free(ctx)
    lat = np.sort(np.asarray(lat)) * 1e3
    return {"rate_hz": rate_hz, "requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "segments_per_s": segs / span, "makespan_s": span, "dtype": "f32+f64acc",
            "fields": "device-resident pool, 2 per edge"}


def _host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"logical_cpus": os.cpu_count(), "model": model}


def _cpu_baseline(problems, threads):
    from oracle import oracle as O
    t0 = time.perf_counter()
    segs = 0
    for p in problems:
        segs += O.trace(p, n_threads=threads)["totals"]["segments"]
    dt = time.perf_counter() - t0
    return segs / dt, dt, segs


def _serving_sweep(M, rates, n_requests):
    out = []
    for rate in rates:
        r = _serving_c3(M, rate, n_requests, 60.0)
        print(f"# serving {rate:g} req/s: p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms "
              f"{r['segments_per_s']:.3e} segments/s", file=sys.stderr, flush=True)
        out.append(r)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["c2", "c1", "c4"], default="c2")
    ap.add_argument("--settings", type=str, default=None,
                    help="chunk,refill,reserve,waves launch settings for the timed form instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("MORAY_CPU_THREADS", "16")))
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-problem, nested, serving and physics measurements")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-only", action="store_true",
                    help="print one serving JSON line per --serve-rates value and exit")
    ap.add_argument("--serve-rates", type=str, default="10,50,100,200,500")
    ap.add_argument("--equilibrium-only", action="store_true",
                    help="print the photo-ionisation equilibrium measurement as one JSON line and exit")
    ap.add_argument("--evolve-only", action="store_true",
                    help="print the time-stepped Test 1 measurement (64^3 to 500 Myr) as one JSON line and exit")
    ap.add_argument("--td-only", action="store_true",
                    help="print the time-dependent-ray measurement (128^3 workload) as one JSON line and exit")
    ap.add_argument("--radpres-only", action="store_true",
                    help="print the radiation-pressure measurement (128^3 workload) as one JSON line and exit")
    ap.add_argument("--covering-only", action="store_true",
                    help="print the covering-factor measurement (128^3 workload) as one JSON line and exit")
    ap.add_argument("--thin-only", action="store_true",
                    help="print the optically-thin measurements (two 128^3 workloads) as one JSON line and exit")
    ap.add_argument("--no-microbench", action="store_true",
                    help="skip the device-peak sweep (no atomic or copy peaks in the line)")
    ap.add_argument("--microbench-table", action="store_true",
                    help="run the device-peak microbenchmark sweep, print its summary as markdown and exit")
    ap.add_argument("--counter-pass", action="store_true",
                    help="run one traced workload and a 1 GiB copy for rocprofv3 --pmc, then exit")
    ap.add_argument("--counter-variant", choices=("plain", "radpres", "td", "thin"), default="plain",
                    help="with --counter-pass: trace with radiation pressure, time-dependent steps or the "
                         "optically-thin approximation (ionised 128^3 workload)")
    ap.add_argument("--read-atomics", nargs=2, metavar=("ATOMIC_DIR", "LAUNCHES"),
                    help="host only: print the float64 atomics per launch of the last LAUNCHES trace "
                         "dispatches of a TCC_EA0_ATOMIC_sum pass, calibrated like --write-atomics")
    ap.add_argument("--write-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "LAUNCHES"),
                    help="host only: turn FETCH_SIZE / WRITE_SIZE pass folders into the traffic record")
    ap.add_argument("--write-atomics", nargs=2, metavar=("ATOMIC_DIR", "LAUNCHES"),
                    help="host only: add the float64 atomics per launch from a TCC_EA0_ATOMIC_sum pass")
    args = ap.parse_args()
    settings = _parse_settings(args.settings) if args.settings else None
    if args.write_traffic:
        _write_traffic(args.write_traffic[0], args.write_traffic[1], args.workload, int(args.write_traffic[2]),
                       args.counter_variant)
        return
    if args.write_atomics:
        _write_atomics(args.write_atomics[0], args.workload, int(args.write_atomics[1]), args.counter_variant)
        return
    if args.read_atomics:
        print(json.dumps(_read_atomics(args.read_atomics[0], int(args.read_atomics[1]))))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this tracer shards by request or by source; "
              f"--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)

    if args.microbench_table:
        _microbench_table()
        return
    if args.counter_pass:
        _counter_pass(args.workload, args.counter_variant, settings)
        return
    import torch
    from paper_1012_2865_amd import moray as M
    if args.equilibrium_only:
        print(json.dumps(_equilibrium_c1(M)), flush=True)
        return
    if args.evolve_only:
        print(json.dumps(_evolve_test1(M)), flush=True)
        return
    if args.covering_only:
        print(json.dumps(_covering_c1(M, args.steps)), flush=True)
        return
    if args.td_only:
        print(json.dumps(_td_c1(M)), flush=True)
        return
    if args.radpres_only:
        print(json.dumps(_radpres_c1(M, args.steps)), flush=True)
        return
    if args.thin_only:
        print(json.dumps(_thin_workloads(M, args.steps, oracle_threads=0 if args.no_cpu_baseline
                                         else args.cpu_threads)), flush=True)
        return
    if args.serve_only:
        for rate in (float(x) for x in args.serve_rates.split(",")):
            print(json.dumps(_serving_c3(M, rate, args.serve_requests, 60.0)), flush=True)
        return

    threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
    peaks = None if args.no_microbench else _device_peaks()
    problems, config = _workload(args.workload)
    dev = [M.problem_to_device(p) for p in problems]
    torch.cuda.synchronize()
    print(f"# workload {config['workload']} on {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)

    # the timed form: mixed precision, one call per step over the whole
    # batch, launch settings from the autotuner (or --settings), graph replay
    ctx32, tune = _tuned(M, M.MORAY_FP32_ACC64, dev, settings)
    try:
        s32, seg32, res32 = _time_steps(M, ctx32, dev, args.steps, max(2, args.warmup))
    finally:
        M.moray_free(ctx32)
    print(f"# fp32 batched: {s32 * 1e3:.2f} ms/step, {seg32} segments, graph replay {bool(res32[0]['from_graph'])}, "
          f"settings {tune}", file=sys.stderr, flush=True)
    plain = None
    if not args.no_fp64:
        plain = _plain_fp64(M, dev, max(1, args.steps // 2))
        print(f"# fp64 plain: {plain['ms_per_step']:.2f} ms/step, {plain['segments']} segments", file=sys.stderr,
              flush=True)
    roofline = _roofline(M, args.workload, dev, tune, peaks)

    cpu = None
    if not args.no_cpu_baseline:
        v, dt, segs = _cpu_baseline(problems, threads)
        what = f"all {len(problems)} problems" if len(problems) > 1 else "full workload"
        cpu = {"value": v, "unit": "segments/s", "cores": threads, "kind": "oracle",
               "sample": f"{what}: {segs} segments in {dt:.1f} s", "host": _host_cpu()}
        # the plain single-threaded oracle on a bounded sample of the same workload
        from paper_1012_2865_amd import workloads as W
        one = problems[:1] if len(problems) > 1 else [W.subset_sources(problems[0], [0, 1])]
        v1, dt1, segs1 = _cpu_baseline(one, 1)
        cpu["one_thread"] = {"value": v1, "unit": "segments/s", "cores": 1, "kind": "oracle",
                             "sample": f"{'the first problem' if len(problems) > 1 else 'sources 0-1'}: "
                                       f"{segs1} segments in {dt1:.1f} s"}
        cpu["gpu_speedup"] = {"over_all_cores": (seg32 / s32) / v, "over_one_thread": (seg32 / s32) / v1}
        print(f"# cpu oracle ({threads} threads): {v:.3e} segments/s", file=sys.stderr, flush=True)

    extras = {}
    if not args.no_extras:
        oth = 0 if args.no_cpu_baseline else threads
        for name, steps in (("c1", args.steps), ("c4", 2)):
            if name != args.workload:
                extras[name] = _single_workload(M, name, steps, peaks, oth if name == "c1" else 0)
                print(f"# {name}: {extras[name]['ms_per_step']:.2f} ms/step, {extras[name]['value']:.3e} segments/s, "
                      f"roofline {extras[name]['roofline']['frac']:.3f}", file=sys.stderr, flush=True)
        extras["serving_c3"] = {"sweep": _serving_sweep(M, [float(x) for x in args.serve_rates.split(",")],
                                                        args.serve_requests)}
        extras["equilibrium"] = _equilibrium_c1(M, oracle_threads=oth)
        print(f"# equilibrium: {extras['equilibrium']['ms_per_trace']:.2f} ms per trace + update", file=sys.stderr,
              flush=True)
        extras["covering"] = _covering_c1(M, max(2, args.steps // 2), oth)
        print(f"# covering factor: {extras['covering']['ms_per_step']:.2f} ms per step "
              f"({100 * extras['covering']['overhead']:+.1f}%)", file=sys.stderr, flush=True)
        extras["radpres"] = _radpres_c1(M, max(2, args.steps // 2), oth)
        print(f"# radiation pressure: {extras['radpres']['ms_per_step']:.2f} ms per step "
              f"({100 * extras['radpres']['overhead']:+.1f}%)", file=sys.stderr, flush=True)
        extras["thin"] = _thin_workloads(M, max(2, args.steps // 2), oracle_threads=oth)
        for nm, rec in extras["thin"].items():
            print(f"# optically thin, {nm}: {rec['ms_per_step']:.2f} ms per step, "
                  f"{rec['speedup_over_plain']:.2f}x the general trace", file=sys.stderr, flush=True)
        extras["td_rays"] = _td_c1(M, oracle=not args.no_cpu_baseline)
        print(f"# time-dependent rays: {extras['td_rays']['segments_per_s_late']:.3e} segments/s", file=sys.stderr,
              flush=True)
        extras["evolve_test1"] = _evolve_test1(M, oracle_threads=oth)
        print(f"# Test 1 to 500 Myr: {extras['evolve_test1']['steps']} steps in "
              f"{extras['evolve_test1']['s_total']:.2f} s", file=sys.stderr, flush=True)

    # the radiation-pressure trace and the time-dependent step against the
    # measured atomic peak (their counts come from their own counter passes on
    # the 128^3 workload)
    if peaks:
        c1_launches = extras["c1"]["roofline"]["launches_per_step"] if "c1" in extras else None
        for name, variant in (("radpres", "radpres"), ("td_rays", "td")):
            ob = extras.get(name)
            apv = _atomics_per_launch("c1", "fp32/" + variant)
            if not ob or not apv or not c1_launches:
                continue
            ms = ob["ms_per_step"][-1] if isinstance(ob["ms_per_step"], list) else ob["ms_per_step"]
            segs = ob["segments_per_step"][-1] if name == "td_rays" else ob["segments_per_s"] * ms * 1e-3
            per_step = apv * c1_launches        # the same level launches as the plain trace
            ob["atomics"] = {"unit": "float64 atomics/s", "per_step": per_step, "per_segment": per_step / segs,
                             "achieved": per_step / (ms * 1e-3), "peak": peaks["atomics_scattered"],
                             "frac": per_step / (ms * 1e-3) / peaks["atomics_scattered"],
                             "source": "TCC_EA0_ATOMIC counter pass read from profiles/traffic_trace_level.json"}

    out = {"metric": METRIC, "value": seg32 / s32, "unit": "segments/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": s32 * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64acc", "data": "synthetic", "config": config,
           "segments_per_step": seg32, "graph_replay": bool(res32[0]["from_graph"]), "settings": tune,
           "plain_fp64": plain, "batched_over_plain": (seg32 / s32) / plain["value"] if plain else None,
           "roofline": roofline, "cpu_baseline": cpu, "device_peaks": peaks, **extras}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
