"""Python binding of libmoray.so (the C ABI in include/moray.h).

Argument marshalling only: every step of a trace runs in the HIP library.
Fields may be torch CUDA tensors (device-resident, passed by pointer) or
numpy arrays (copied by the library); outputs are float64 torch CUDA tensors
by default. PyTorch provides device memory and the stream, nothing else.
The library must be built (python -m paper_1012_2865_amd.build); importing
this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmoray.so")

MORAY_OK, MORAY_EINVAL, MORAY_ENOMEM, MORAY_EDEVICE, MORAY_EQUEUE, MORAY_EBUSY = 0, -1, -2, -3, -4, -5
MORAY_ETIMEOUT, MORAY_EINTERNAL, MORAY_ECANCELED = -6, -7, -8
STATUS_NAMES = {0: "MORAY_OK", -1: "MORAY_EINVAL", -2: "MORAY_ENOMEM", -3: "MORAY_EDEVICE", -4: "MORAY_EQUEUE",
                -5: "MORAY_EBUSY", -6: "MORAY_ETIMEOUT", -7: "MORAY_EINTERNAL", -8: "MORAY_ECANCELED"}
MORAY_FP64, MORAY_FP32_ACC64 = 0, 1
MORAY_FIELDS_ON_DEVICE, MORAY_OUT_ON_DEVICE = 1, 2


class MorayError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class InitParams(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("precision", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("queue_capacity", ctypes.c_size_t), ("waves_per_cu", ctypes.c_int), ("refill_lanes", ctypes.c_int),
                ("chunk_rays", ctypes.c_int), ("hip_stream", ctypes.c_void_p), ("profile", ctypes.c_int),
                ("deposit_cache", ctypes.c_int), ("reserve_rays", ctypes.c_int)]


class Source(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double), ("ndot", ctypes.c_double)]


class Spectrum(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int), ("energy_ev", ctypes.POINTER(ctypes.c_double)),
                ("sigma_cm2", ctypes.POINTER(ctypes.c_double)), ("photon_frac", ctypes.POINTER(ctypes.c_double)),
                ("e_ion_ev", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx_cm", ctypes.c_double),
                ("parent", ctypes.c_int), ("offset", ctypes.c_int * 3), ("n_h", ctypes.c_void_p),
                ("x_hi", ctypes.c_void_p)]


class TraceParams(ctypes.Structure):
    _fields_ = [("phi_c", ctypes.c_double), ("level_init", ctypes.c_int), ("level_max", ctypes.c_int),
                ("p_min_frac", ctypes.c_double), ("covering", ctypes.c_int), ("tau_thin", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("grids", ctypes.POINTER(Grid)), ("n_grids", ctypes.c_int), ("sources", ctypes.POINTER(Source)),
                ("n_sources", ctypes.c_int), ("spectrum", ctypes.POINTER(Spectrum)), ("params", TraceParams)]


class Result(ctypes.Structure):
    _fields_ = [("k_ph", ctypes.c_void_p), ("heating", ctypes.c_void_p), ("escaped_sg", ctypes.POINTER(ctypes.c_double)),
                ("accel", ctypes.c_void_p), ("emitted", ctypes.c_double), ("absorbed", ctypes.c_double), ("escaped", ctypes.c_double),
                ("truncated", ctypes.c_double), ("segments", ctypes.c_ulonglong), ("rays_seeded", ctypes.c_ulonglong),
                ("splits", ctypes.c_ulonglong), ("rays_escaped", ctypes.c_ulonglong),
                ("rays_truncated", ctypes.c_ulonglong), ("peak_level_rays", ctypes.c_ulonglong),
                ("trace_ms", ctypes.c_double), ("trace_launches", ctypes.c_int), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("from_graph", ctypes.c_int), ("thin_segments", ctypes.c_ulonglong)]


class EquilibriumParams(ctypes.Structure):
    _fields_ = [("alpha_b", ctypes.c_double), ("damping", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int)]


ALPHA_B = 2.59e-13   # case-B recombination coefficient at 1e4 K, cm^3/s (section 2.2)


class EvolveParams(ctypes.Structure):
    _fields_ = [("alpha_b", ctypes.c_double), ("eps_ion", ctypes.c_double), ("tau_front", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("t_end", ctypes.c_double), ("max_steps", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("chunk_rays", ctypes.c_int), ("refill_lanes", ctypes.c_int), ("reserve_rays", ctypes.c_int),
                ("waves_per_cu", ctypes.c_int), ("first_ms", ctypes.c_double), ("best_ms", ctypes.c_double),
                ("trials", ctypes.c_int)]


ABI_FUNCTIONS = ("moray_init", "moray_trace", "moray_autotune", "moray_autotune_cached", "moray_equilibrate",
                 "moray_evolve",
                 "moray_td_create", "moray_td_step", "moray_td_free", "moray_trace_async", "moray_query",
                 "moray_set_deadline", "moray_cancel", "moray_trace_noalloc", "moray_free", "moray_last_error",
                 "moray_version")

_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1012_2865_amd.build`")
        # PyTorch carries its own HIP runtime. Loaded first, it also serves the
        # library (same soname); loaded after the library's runtime it brings a
        # second one into the process, and whichever initialises last finds no
        # device. So torch, when it is installed, is imported before the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        lib.moray_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(InitParams)]
        lib.moray_init.restype = ctypes.c_int
        lib.moray_trace.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_uint,
                                    ctypes.POINTER(Result)]
        lib.moray_trace.restype = ctypes.c_int
        lib.moray_trace_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_uint,
                                            ctypes.POINTER(Result)]
        lib.moray_trace_noalloc.restype = ctypes.c_int
        lib.moray_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_uint,
                                       ctypes.c_int, ctypes.POINTER(TuneResult)]
        lib.moray_autotune.restype = ctypes.c_int
        lib.moray_autotune_cached.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(Problem), ctypes.c_int,
                                              ctypes.c_uint, ctypes.c_int, ctypes.POINTER(TuneResult),
                                              ctypes.POINTER(ctypes.c_int)]
        lib.moray_autotune_cached.restype = ctypes.c_int
        lib.moray_equilibrate.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_uint,
                                          ctypes.POINTER(EquilibriumParams), ctypes.c_void_p, ctypes.POINTER(Result),
                                          ctypes.POINTER(ctypes.c_int)]
        lib.moray_equilibrate.restype = ctypes.c_int
        lib.moray_evolve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_uint,
                                     ctypes.POINTER(EvolveParams), ctypes.c_void_p, ctypes.POINTER(Result),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        lib.moray_evolve.restype = ctypes.c_int
        lib.moray_td_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_double, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_void_p)]
        lib.moray_td_create.restype = ctypes.c_int
        lib.moray_td_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_uint,
                                      ctypes.c_int, ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_double)]
        lib.moray_td_step.restype = ctypes.c_int
        lib.moray_td_free.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.moray_td_free.restype = None
        lib.moray_trace_async.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_uint,
                                          ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_ulonglong)]
        lib.moray_trace_async.restype = ctypes.c_int
        lib.moray_query.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong, ctypes.c_int]
        lib.moray_query.restype = ctypes.c_int
        lib.moray_set_deadline.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong, ctypes.c_double]
        lib.moray_set_deadline.restype = ctypes.c_int
        lib.moray_cancel.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong]
        lib.moray_cancel.restype = ctypes.c_int
        lib.moray_free.argtypes = [ctypes.c_void_p]
        lib.moray_free.restype = None
        lib.moray_last_error.argtypes = [ctypes.c_void_p]
        lib.moray_last_error.restype = ctypes.c_char_p
        lib.moray_version.argtypes = []
        lib.moray_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def moray_version() -> str:
    return load_library().moray_version().decode()


def moray_last_error(ctx) -> str:
    return load_library().moray_last_error(ctx).decode()


def moray_init(device: int = 0, precision: int = MORAY_FP32_ACC64, hbm_budget_bytes: int = 0,
               queue_capacity: int = 0, waves_per_cu: int = 0, refill_lanes: int = 0, chunk_rays: int = 0,
               hip_stream=None, profile: bool = False, deposit_cache: int = 0, reserve_rays: int = 0):
    """Create a context; returns an opaque handle. hip_stream: an int handle
    (torch.cuda.Stream.cuda_stream) or None for torch's current stream."""
    lib = load_library()
    if hip_stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                hip_stream = torch.cuda.current_stream(device).cuda_stream
        except Exception:
            hip_stream = None
    p = InitParams(device, precision, hbm_budget_bytes, queue_capacity, waves_per_cu, refill_lanes, chunk_rays,
                   ctypes.c_void_p(hip_stream or 0), int(bool(profile)), int(deposit_cache), int(reserve_rays))
    h = ctypes.c_void_p()
    rc = lib.moray_init(ctypes.byref(h), ctypes.byref(p))
    if rc != MORAY_OK:
        raise MorayError(rc, "moray_init: " + moray_last_error(None))
    return h


def moray_free(ctx) -> None:
    if ctx is not None:
        load_library().moray_free(ctx)


def _is_torch_cuda(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, dtype_np, keep: list):
    if _is_torch_cuda(a):
        assert a.is_contiguous(), "device fields must be contiguous"
        keep.append(a)
        return a.data_ptr()
    arr = np.ascontiguousarray(a, dtype=dtype_np)
    keep.append(arr)
    return arr.ctypes.data


def _marshal(problems: Sequence, out_on_device: bool, want_escaped_sg: bool, outputs=None, want_accel: bool = False):
    """C structs for a list of problems, plus everything they point into.
    outputs: optional list of (k_ph, heating) or (k_ph, heating, accel) flat
    float64 buffers per problem (torch CUDA tensors when out_on_device, else
    numpy arrays); want_accel asks for the radiation-pressure acceleration."""
    keep: list = []
    n = len(problems)
    cprobs = (Problem * n)()
    results = (Result * n)()
    on_dev = None
    outs = []
    for i, pb in enumerate(problems):
        grids = (Grid * len(pb.grids))()
        keep.append(grids)
        n_cells = 0
        shapes = []
        for q, g in enumerate(pb.grids):
            dev = _is_torch_cuda(g.n_h)
            if on_dev is None:
                on_dev = dev
            if dev != on_dev or _is_torch_cuda(g.x_hi) != dev:
                raise ValueError("all fields of one call must be on the device, or all on the host")
            shape = tuple(g.n_h.shape)
            nz, ny, nx = shape
            grids[q].nx, grids[q].ny, grids[q].nz = nx, ny, nz
            grids[q].dx_cm = float(g.dx_cm)
            grids[q].parent = int(g.parent)
            for a in range(3):
                grids[q].offset[a] = int(g.offset[a])
            grids[q].n_h = _ptr(g.n_h, np.float32, keep)
            grids[q].x_hi = _ptr(g.x_hi, np.float32, keep)
            shapes.append(shape)
            n_cells += nx * ny * nz
        S = np.asarray(pb.sources, dtype=np.float64).reshape(-1, 4)
        srcs = (Source * max(1, len(S)))()
        for k, row in enumerate(S):
            srcs[k].x, srcs[k].y, srcs[k].z, srcs[k].ndot = (float(v) for v in row)
        keep.append(srcs)
        sp = pb.spectrum
        e = np.ascontiguousarray(sp.energy_ev, dtype=np.float64)
        sg = np.ascontiguousarray(sp.sigma_cm2, dtype=np.float64)
        fr = np.ascontiguousarray(sp.frac, dtype=np.float64)
        keep += [e, sg, fr]
        dp = ctypes.POINTER(ctypes.c_double)
        cspec = Spectrum(len(e), e.ctypes.data_as(dp), sg.ctypes.data_as(dp), fr.ctypes.data_as(dp), float(sp.e_ion_ev))
        keep.append(cspec)
        pr = pb.params
        cprobs[i] = Problem(grids, len(pb.grids), srcs, len(S), ctypes.pointer(cspec),
                            TraceParams(float(pr.phi_c), int(pr.level_init), int(pr.level_max), float(pr.p_min_frac),
                                        1 if getattr(pr, "covering", False) else 0,
                                        float(getattr(pr, "tau_thin", 0.0))))
        acc = None
        if outputs is not None:
            kph, heat = outputs[i][0], outputs[i][1]
            acc = outputs[i][2] if len(outputs[i]) > 2 else None
            assert (kph.numel() if hasattr(kph, "numel") else kph.size) >= n_cells
            if out_on_device:
                assert _is_torch_cuda(kph) and _is_torch_cuda(heat) and kph.is_contiguous() and heat.is_contiguous()
                results[i].k_ph, results[i].heating = kph.data_ptr(), heat.data_ptr()
            else:
                results[i].k_ph, results[i].heating = kph.ctypes.data, heat.ctypes.data
        elif out_on_device:
            import torch
            kph = torch.empty(n_cells, dtype=torch.float64, device="cuda")
            heat = torch.empty(n_cells, dtype=torch.float64, device="cuda")
            results[i].k_ph, results[i].heating = kph.data_ptr(), heat.data_ptr()
        else:
            kph, heat = np.empty(n_cells), np.empty(n_cells)
            results[i].k_ph, results[i].heating = kph.ctypes.data, heat.ctypes.data
        if want_accel and acc is None:
            if out_on_device:
                import torch
                acc = torch.empty(3 * n_cells, dtype=torch.float64, device="cuda")
            else:
                acc = np.empty(3 * n_cells)
        if acc is not None:
            assert (acc.numel() if hasattr(acc, "numel") else acc.size) >= 3 * n_cells
            results[i].accel = acc.data_ptr() if out_on_device else acc.ctypes.data
        esc = np.zeros(max(1, len(S) * len(e)))
        if want_escaped_sg:
            results[i].escaped_sg = esc.ctypes.data_as(dp)
        outs.append((kph, heat, shapes, esc, len(S), len(e), acc, n_cells))
    flags = (MORAY_FIELDS_ON_DEVICE if on_dev else 0) | (MORAY_OUT_ON_DEVICE if out_on_device else 0)
    return cprobs, results, keep, outs, flags


def _unpack(results, outs, want_escaped_sg: bool) -> List[dict]:
    out = []
    for i in range(len(outs)):
        kph, heat, shapes, esc, ns, ng, acc, n_cells = outs[i]
        kl, hl, al, o = [], [], [], 0
        for shp in shapes:
            m = int(np.prod(shp))
            kl.append(kph[o:o + m].reshape(shp))
            hl.append(heat[o:o + m].reshape(shp))
            if acc is not None:
                al.append(acc[:3 * n_cells].reshape(3, n_cells)[:, o:o + m].reshape((3,) + tuple(shp)))
            o += m
        R = results[i]
        d = {name: getattr(R, name) for name, _ in Result._fields_
             if name not in ("k_ph", "heating", "escaped_sg", "accel")}
        d["k_ph"], d["heating"] = kl, hl
        if acc is not None:
            d["accel"] = al
        if want_escaped_sg:
            d["escaped_sg"] = esc[:ns * ng].reshape(ns, ng)
        out.append(d)
    return out


def moray_trace(ctx, problems: Sequence, out_on_device: bool = True, want_escaped_sg: bool = False,
                outputs=None, want_accel: bool = False) -> List[dict]:
    """Trace a batch of problems in one call.

    Each problem is duck-typed: ``grids`` (``n_h``, ``x_hi`` as torch CUDA
    tensors or numpy arrays of shape (nz, ny, nx); ``dx_cm``, ``parent``,
    ``offset``), ``sources`` (S x 4), ``spectrum`` (``energy_ev``, ``sigma_cm2``,
    ``frac``, ``e_ion_ev``), ``params`` (``phi_c``, ``level_init``,
    ``level_max``, ``p_min_frac``). Returns one dict per problem with ``k_ph``
    and ``heating`` (lists per grid) and the totals. ``outputs`` optionally
    names the result buffers (see _marshal); reusing them across calls lets
    the library replay its captured launch sequence. want_accel adds
    ``accel``, the radiation-pressure acceleration per grid, shaped
    (3, nz, ny, nx)."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal(problems, out_on_device, want_escaped_sg, outputs, want_accel)
    rc = lib.moray_trace(ctx, cprobs, len(problems), flags, results)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return _unpack(results, outs, want_escaped_sg)


class PreparedBatch:
    """A batch's C descriptors, built once for repeated moray_trace calls on
    the same problems and result buffers (the time-stepping, serving-loop and
    benchmark pattern): grid shapes and nesting, field and result pointers,
    sources, spectra and parameters are fixed when the batch is prepared;
    field and result values may change between calls. The per-grid views of
    the results are built once too. Building the descriptors of 64 problems
    takes about a millisecond of Python per call otherwise."""

    def __init__(self, problems: Sequence, outputs=None, out_on_device: bool = True, want_escaped_sg: bool = False,
                 want_accel: bool = False):
        self.n = len(problems)
        self.want_escaped_sg = want_escaped_sg
        self.cprobs, self.results, self.keep, self.outs, self.flags = _marshal(
            problems, out_on_device, want_escaped_sg, outputs, want_accel)
        views = _unpack(self.results, self.outs, want_escaped_sg)
        self.views = [{k: d[k] for k in ("k_ph", "heating", "accel", "escaped_sg") if k in d} for d in views]
        self.fields = [name for name, _ in Result._fields_ if name not in ("k_ph", "heating", "escaped_sg", "accel")]


def moray_trace_prepared(ctx, batch: PreparedBatch) -> List[dict]:
    """moray_trace on a PreparedBatch: the same call, without rebuilding the
    descriptors. Returns one dict per problem as moray_trace does."""
    lib = load_library()
    rc = lib.moray_trace(ctx, batch.cprobs, batch.n, batch.flags, batch.results)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    out = []
    for R, v in zip(batch.results, batch.views):
        d = {name: getattr(R, name) for name in batch.fields}
        d.update(v)
        out.append(d)
    return out


def moray_trace_noalloc(ctx, problems: Sequence, outputs, out_on_device: bool = True,
                        want_escaped_sg: bool = False) -> List[dict]:
    """moray_trace through the entry point that allocates no device memory
    (its scratch comes from the library's fixed array). ``outputs`` names the
    caller's result buffers, as in moray_trace (required: the call itself
    must not allocate them)."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal(problems, out_on_device, want_escaped_sg, outputs)
    rc = lib.moray_trace_noalloc(ctx, cprobs, len(problems), flags, results)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return _unpack(results, outs, want_escaped_sg)


def moray_autotune(ctx, problems: Sequence, max_trials: int = 0, cache_path: Optional[str] = None) -> dict:
    """Pick the fastest launch settings for this batch and keep them in the
    context. With `cache_path`, through the persistent cache file
    (moray_autotune_cached): the result then has "from_cache"."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal(problems, True, False)
    r = TuneResult()
    if cache_path is None:
        rc = lib.moray_autotune(ctx, cprobs, len(problems), flags, int(max_trials), ctypes.byref(r))
        hit = None
    else:
        h = ctypes.c_int(0)
        rc = lib.moray_autotune_cached(ctx, os.fsencode(cache_path), cprobs, len(problems), flags, int(max_trials),
                                       ctypes.byref(r), ctypes.byref(h))
        hit = bool(h.value)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    out = {name: getattr(r, name) for name, _ in TuneResult._fields_}
    if hit is not None:
        out["from_cache"] = hit
    return out


def _x64_buffer(problem):
    """Flat float64 device buffer for the iterate of every grid, in grid order."""
    import torch
    return torch.empty(sum(int(g.n_h.numel()) for g in problem.grids), dtype=torch.float64, device="cuda")


def _x64_views(problem, x64):
    """The iterate shaped like the grid (single grid) or one view per grid."""
    if x64 is None:
        return None
    views, o = [], 0
    for g in problem.grids:
        m = int(g.n_h.numel())
        views.append(x64[o:o + m].view(tuple(g.n_h.shape)))
        o += m
    return views[0] if len(views) == 1 else views


def moray_equilibrate(ctx, problem, alpha_b: float = ALPHA_B, damping: float = 0.5, tol: float = 1e-6,
                      max_iter: int = 300, out_on_device: bool = True, want_escaped_sg: bool = False,
                      want_x64: bool = False):
    """Photo-ionisation equilibrium of one single-grid problem whose fields
    are torch CUDA tensors (see moray.h). The problem's x_hi tensor is updated
    in place. Returns (result dict of the final trace, updates made, float64 x
    as a torch tensor or None)."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal([problem], out_on_device, want_escaped_sg)
    x64 = _x64_buffer(problem) if want_x64 else None
    it = ctypes.c_int(0)
    ep = EquilibriumParams(float(alpha_b), float(damping), float(tol), int(max_iter))
    rc = lib.moray_equilibrate(ctx, cprobs, flags, ctypes.byref(ep), x64.data_ptr() if x64 is not None else None,
                               results, ctypes.byref(it))
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return _unpack(results, outs, want_escaped_sg)[0], it.value, _x64_views(problem, x64)


def moray_evolve(ctx, problem, t_end: float, eps_ion: float = 0.1, tau_front: float = 0.5,
                 dt_max: float | None = None, max_steps: int = 100000, alpha_b: float = ALPHA_B,
                 out_on_device: bool = True, want_escaped_sg: bool = False, want_x64: bool = False,
                 want_dts: bool = False):
    """Time-stepped photo-ionisation of one single-grid problem whose fields
    are torch CUDA tensors (see moray.h), for t_end seconds; dt_max defaults
    to t_end. The problem's x_hi tensor is updated in place. Returns (result
    dict of the final trace, steps taken, time reached, float64 x as a torch
    tensor or None, numpy array of the steps' dt or None)."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal([problem], out_on_device, want_escaped_sg)
    x64 = _x64_buffer(problem) if want_x64 else None
    dts = np.zeros(max(1, int(max_steps)), dtype=np.float64) if want_dts else None
    steps, t = ctypes.c_int(0), ctypes.c_double(0.0)
    ep = EvolveParams(float(alpha_b), float(eps_ion), float(tau_front), float(t_end if dt_max is None else dt_max),
                      float(t_end), int(max_steps))
    rc = lib.moray_evolve(ctx, cprobs, flags, ctypes.byref(ep), x64.data_ptr() if x64 is not None else None,
                          results, ctypes.byref(steps), ctypes.byref(t),
                          dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if dts is not None else None)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return (_unpack(results, outs, want_escaped_sg)[0], steps.value, t.value, _x64_views(problem, x64),
            dts[:steps.value].copy() if dts is not None else None)


def moray_td_create(ctx, problem, c_dt: float, pool_rays: int = 1 << 22):
    """Device state of time-dependent rays for problems shaped like this one
    (see moray.h); c_dt is c dt_P in root cells. Returns the handle."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal([problem], True, False)
    h = ctypes.c_void_p()
    rc = lib.moray_td_create(ctx, cprobs, float(c_dt), int(pool_rays), ctypes.byref(h))
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return h.value


def moray_td_step(ctx, td, problem, emit: bool = True, want_escaped_sg: bool = False, outputs=None):
    """One step of time-dependent rays for a problem with torch CUDA fields.
    Returns (result dict of the step, photon rate of the rays in flight)."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal([problem], True, want_escaped_sg, outputs)
    held = ctypes.c_double(0.0)
    rc = lib.moray_td_step(ctx, td, cprobs, flags, 1 if emit else 0, results, ctypes.byref(held))
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return _unpack(results, outs, want_escaped_sg)[0], held.value


def moray_td_free(ctx, td) -> None:
    if td:
        load_library().moray_td_free(ctx, td)


class Ticket:
    """A pending asynchronous solve: owns the C structs and buffers the
    library writes into until the ticket is done."""

    def __init__(self, handle: int, cprobs, results, keep, outs, want_escaped_sg: bool):
        self.handle = handle
        self._c = (cprobs, results, keep)
        self._results, self._outs, self._want = results, outs, want_escaped_sg
        self.results = None


def moray_trace_async(ctx, problems: Sequence, out_on_device: bool = True, want_escaped_sg: bool = False) -> Ticket:
    """Queue problems on the context's serving engine; returns at once."""
    lib = load_library()
    cprobs, results, keep, outs, flags = _marshal(problems, out_on_device, want_escaped_sg)
    t = ctypes.c_ulonglong()
    rc = lib.moray_trace_async(ctx, cprobs, len(problems), flags, results, ctypes.byref(t))
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    return Ticket(t.value, cprobs, results, keep, outs, want_escaped_sg)


def moray_query(ctx, ticket: Ticket, wait_ms: int = -1):
    """Results of a ticket (a list of dicts like moray_trace's), or None while
    it is still running after wait_ms milliseconds (-1: wait until done)."""
    if ticket.results is not None:
        return ticket.results
    rc = load_library().moray_query(ctx, ticket.handle, int(wait_ms))
    if rc == MORAY_EBUSY:
        return None
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))
    ticket.results = _unpack(ticket._results, ticket._outs, ticket._want)
    return ticket.results


def moray_set_deadline(ctx, ticket: Ticket, seconds: float) -> None:
    """The ticket fails with MORAY_ETIMEOUT unless done `seconds` from now
    (checked at the serving engine's next launch boundary)."""
    rc = load_library().moray_set_deadline(ctx, ticket.handle, float(seconds))
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))


def moray_cancel(ctx, ticket: Ticket) -> None:
    """The ticket fails with MORAY_ECANCELED at the serving engine's next
    launch boundary (unless it is done by then)."""
    rc = load_library().moray_cancel(ctx, ticket.handle)
    if rc != MORAY_OK:
        raise MorayError(rc, moray_last_error(ctx))


def problem_to_device(problem, device: str = "cuda"):
    """Copy a problem's fields into torch CUDA tensors (the device-resident form)."""
    import copy

    import torch
    p = copy.copy(problem)
    p.grids = []
    for g in problem.grids:
        h = copy.copy(g)
        h.n_h = torch.from_numpy(np.ascontiguousarray(g.n_h, dtype=np.float32)).to(device)
        h.x_hi = torch.from_numpy(np.ascontiguousarray(g.x_hi, dtype=np.float32)).to(device)
        p.grids.append(h)
    return p
