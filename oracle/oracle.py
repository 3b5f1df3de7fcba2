"""ctypes front end of the plain FP64 CPU oracle (moray_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline call this to check the GPU library against; the product path never
imports it. It imports nothing from the GPU package: a problem is any object
with the attributes ``grids`` (each with ``n_h``, ``x_hi``, ``dx_cm``,
``parent``, ``offset``), ``sources`` (S x 4: x, y, z in root cells, ndot),
``spectrum`` (``energy_ev``, ``sigma_cm2``, ``frac``, ``e_ion_ev``) and
``params`` (``phi_c``, ``level_init``, ``level_max``, ``p_min_frac``, and
optionally ``covering`` and ``tau_thin``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "moray_oracle.c")
_LIB_PATH = os.environ.get("MORAY_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx_cm", ctypes.c_double),
                ("n_h", ctypes.POINTER(ctypes.c_float)), ("x_hi", ctypes.POINTER(ctypes.c_float)),
                ("parent", ctypes.c_int), ("offset", ctypes.c_int * 3)]


class _Source(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double), ("ndot", ctypes.c_double)]


class _Spectrum(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int), ("energy_ev", ctypes.POINTER(ctypes.c_double)),
                ("sigma_cm2", ctypes.POINTER(ctypes.c_double)), ("frac", ctypes.POINTER(ctypes.c_double)),
                ("e_ion_ev", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("phi_c", ctypes.c_double), ("level_init", ctypes.c_int), ("level_max", ctypes.c_int),
                ("p_min_frac", ctypes.c_double), ("covering", ctypes.c_int), ("tau_thin", ctypes.c_double)]


class _Totals(ctypes.Structure):
    _fields_ = [("emitted", ctypes.c_double), ("absorbed", ctypes.c_double), ("escaped", ctypes.c_double),
                ("truncated", ctypes.c_double), ("segments", ctypes.c_uint64), ("rays_seeded", ctypes.c_uint64),
                ("splits", ctypes.c_uint64), ("rays_escaped", ctypes.c_uint64), ("rays_truncated", ctypes.c_uint64),
                ("thin_segments", ctypes.c_uint64), ("thin_marked", ctypes.c_uint64), ("thin_margin", ctypes.c_double)]


def _params(pr) -> _Params:
    return _Params(float(pr.phi_c), int(pr.level_init), int(pr.level_max), float(pr.p_min_frac),
                   1 if getattr(pr, "covering", False) else 0, float(getattr(pr, "tau_thin", 0.0)))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_trace.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.POINTER(_Source), ctypes.c_int,
                                  ctypes.POINTER(_Spectrum), ctypes.POINTER(_Params), ctypes.c_int,
                                  dp, dp, dp, dp, dp, ctypes.POINTER(_Totals)]
        lib.orc_trace.restype = ctypes.c_int
        lib.orc_trace_accel.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.POINTER(_Source), ctypes.c_int,
                                        ctypes.POINTER(_Spectrum), ctypes.POINTER(_Params), ctypes.c_int,
                                        dp, dp, dp, dp, dp, dp, ctypes.POINTER(_Totals)]
        lib.orc_trace_accel.restype = ctypes.c_int
        sz = ctypes.c_size_t
        lib.orc_trace_td.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.POINTER(_Source), ctypes.c_int,
                                     ctypes.POINTER(_Spectrum), ctypes.POINTER(_Params), ctypes.c_double, ctypes.c_int,
                                     ctypes.c_void_p, sz, ctypes.c_void_p, sz, ctypes.POINTER(sz), dp,
                                     dp, dp, dp, dp, ctypes.POINTER(_Totals)]
        lib.orc_trace_td.restype = ctypes.c_int
        lib.orc_pix2vec_nest.argtypes = [ctypes.c_int, ctypes.c_uint64, dp]
        lib.orc_pix2vec_nest.restype = None
        lib.orc_const_ev_erg.restype = ctypes.c_double
        _lib = lib
    return _lib


def ev_erg() -> float:
    return _load().orc_const_ev_erg()


def pix2vec(level: int, pix: int) -> np.ndarray:
    v = np.zeros(3)
    _load().orc_pix2vec_nest(int(level), int(pix), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return v


def pix2vec_all(level: int) -> np.ndarray:
    return np.array([pix2vec(level, p) for p in range(12 * 4 ** level)])


class OracleError(ValueError):
    pass


TRAY = np.dtype([("src", "<i4"), ("grp", "<i4"), ("level", "<i4"), ("age", "<i4"), ("pix", "<u8"),
                 ("r", "<f8"), ("P", "<f8"), ("P0", "<f8")])


def trace_td(problem, c_dt: float, rays_in=None, emit: bool = True, out_cap: int = 1 << 22):
    """One step of the time-dependent trace (orc_trace_td): the rays in
    flight (a TRAY array, or None) continue one step older, the sources emit
    when `emit`, every ray halts at (age + 1) c_dt root cells. Returns the
    result dict (fields of this step, totals, plus "held": the photon rate
    of the halted rays) and the TRAY array of the halted rays."""
    lib = _load()
    args, keep, n_cells, shapes = _c_problem(problem)
    grids, n_grids, srcs, n_src, spec, par = args
    rin = np.ascontiguousarray(rays_in if rays_in is not None else np.zeros(0, TRAY), dtype=TRAY)
    rout = np.zeros(out_cap, TRAY)
    n_out = ctypes.c_size_t(0)
    held = ctypes.c_double(0.0)
    absorbed, energy, k_ph, heating = (np.zeros(n_cells) for _ in range(4))
    dp = ctypes.POINTER(ctypes.c_double)
    tot = _Totals()
    rc = lib.orc_trace_td(grids, n_grids, srcs, n_src, ctypes.byref(spec), ctypes.byref(par), float(c_dt),
                          1 if emit else 0, rin.ctypes.data if rin.size else None, rin.size, rout.ctypes.data,
                          out_cap, ctypes.byref(n_out), ctypes.byref(held), absorbed.ctypes.data_as(dp),
                          energy.ctypes.data_as(dp), k_ph.ctypes.data_as(dp), heating.ctypes.data_as(dp),
                          ctypes.byref(tot))
    if rc != 0:
        raise OracleError("oracle rejected the step" if rc == -1 else "too many rays in flight")
    split = _splitter(shapes)
    totals = {name: getattr(tot, name) for name, _ in _Totals._fields_}
    res = {"absorbed": split(absorbed), "energy": split(energy), "k_ph": split(k_ph), "heating": split(heating),
           "totals": totals, "held": held.value}
    return res, rout[:n_out.value].copy()


def _splitter(shapes):
    def split(a):
        out, o = [], 0
        for shp in shapes:
            n = int(np.prod(shp))
            out.append(a[o:o + n].reshape(shp))
            o += n
        return out
    return split


def _c_problem(problem):
    """C structs of one problem and the arrays they point into."""
    keep = []
    grids = (_Grid * len(problem.grids))()
    shapes = []
    for q, g in enumerate(problem.grids):
        n_h = np.ascontiguousarray(g.n_h, dtype=np.float32)
        x_hi = np.ascontiguousarray(g.x_hi, dtype=np.float32)
        keep += [n_h, x_hi]
        nz, ny, nx = n_h.shape
        shapes.append(n_h.shape)
        grids[q].nx, grids[q].ny, grids[q].nz = nx, ny, nz
        grids[q].dx_cm = float(g.dx_cm)
        grids[q].n_h = n_h.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        grids[q].x_hi = x_hi.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        grids[q].parent = int(g.parent)
        for a in range(3):
            grids[q].offset[a] = int(g.offset[a])
    S = np.asarray(problem.sources, dtype=np.float64).reshape(-1, 4)
    srcs = (_Source * max(1, len(S)))()
    for i, row in enumerate(S):
        srcs[i].x, srcs[i].y, srcs[i].z, srcs[i].ndot = (float(v) for v in row)
    sp = problem.spectrum
    e = np.ascontiguousarray(sp.energy_ev, dtype=np.float64)
    sg = np.ascontiguousarray(sp.sigma_cm2, dtype=np.float64)
    fr = np.ascontiguousarray(sp.frac, dtype=np.float64)
    keep += [e, sg, fr, grids, srcs]
    dp = ctypes.POINTER(ctypes.c_double)
    spec = _Spectrum(len(e), e.ctypes.data_as(dp), sg.ctypes.data_as(dp), fr.ctypes.data_as(dp), float(sp.e_ion_ev))
    pr = problem.params
    par = _params(pr)
    keep += [spec, par]
    n_cells = sum(int(np.prod(shp)) for shp in shapes)
    return (grids, len(problem.grids), srcs, len(S), spec, par), keep, n_cells, shapes


def trace(problem, n_threads: int = 1, want_accel: bool = False) -> dict:
    """Run the oracle on one problem; returns per-grid fields and totals, and
    with want_accel the radiation-pressure acceleration per grid, shaped
    (3, nz, ny, nx) in cm/s^2."""
    lib = _load()
    keep = []
    grids = (_Grid * len(problem.grids))()
    for q, g in enumerate(problem.grids):
        n_h = np.ascontiguousarray(g.n_h, dtype=np.float32)
        x_hi = np.ascontiguousarray(g.x_hi, dtype=np.float32)
        keep += [n_h, x_hi]
        nz, ny, nx = n_h.shape
        grids[q].nx, grids[q].ny, grids[q].nz = nx, ny, nz
        grids[q].dx_cm = float(g.dx_cm)
        grids[q].n_h = n_h.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        grids[q].x_hi = x_hi.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        grids[q].parent = int(g.parent)
        for a in range(3):
            grids[q].offset[a] = int(g.offset[a])
    S = np.asarray(problem.sources, dtype=np.float64).reshape(-1, 4)
    srcs = (_Source * max(1, len(S)))()
    for i, row in enumerate(S):
        srcs[i].x, srcs[i].y, srcs[i].z, srcs[i].ndot = (float(v) for v in row)
    sp = problem.spectrum
    e = np.ascontiguousarray(sp.energy_ev, dtype=np.float64)
    sg = np.ascontiguousarray(sp.sigma_cm2, dtype=np.float64)
    fr = np.ascontiguousarray(sp.frac, dtype=np.float64)
    keep += [e, sg, fr]
    dp = ctypes.POINTER(ctypes.c_double)
    spec = _Spectrum(len(e), e.ctypes.data_as(dp), sg.ctypes.data_as(dp), fr.ctypes.data_as(dp), float(sp.e_ion_ev))
    pr = problem.params
    par = _params(pr)
    n_cells = sum(int(np.asarray(g.n_h).size) for g in problem.grids)
    absorbed = np.zeros(n_cells)
    energy = np.zeros(n_cells)
    k_ph = np.zeros(n_cells)
    heating = np.zeros(n_cells)
    esc = np.zeros(max(1, len(S) * len(e)))
    accel = np.zeros(3 * n_cells) if want_accel else None
    tot = _Totals()
    rc = lib.orc_trace_accel(grids, len(problem.grids), srcs, len(S), ctypes.byref(spec), ctypes.byref(par),
                             int(n_threads), absorbed.ctypes.data_as(dp), energy.ctypes.data_as(dp),
                             k_ph.ctypes.data_as(dp), heating.ctypes.data_as(dp), esc.ctypes.data_as(dp),
                             accel.ctypes.data_as(dp) if accel is not None else None, ctypes.byref(tot))
    if rc != 0:
        raise OracleError("oracle rejected the problem")

    def split(a):
        out, o = [], 0
        for g in problem.grids:
            n = int(np.asarray(g.n_h).size)
            out.append(a[o:o + n].reshape(np.asarray(g.n_h).shape))
            o += n
        return out

    totals = {name: getattr(tot, name) for name, _ in _Totals._fields_}
    out = {"absorbed": split(absorbed), "energy": split(energy), "k_ph": split(k_ph), "heating": split(heating),
           "escaped_sg": esc[:len(S) * len(e)].reshape(len(S), len(e)), "totals": totals}
    if accel is not None:
        planes = [split(accel[k * n_cells:(k + 1) * n_cells]) for k in range(3)]
        out["accel"] = [np.stack([planes[k][q] for k in range(3)]) for q in range(len(problem.grids))]
    return out
