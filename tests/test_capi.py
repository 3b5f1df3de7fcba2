"""The C-ABI library loads, exports every function include/moray.h declares,
fails cleanly without a GPU, and the Python binding's struct layouts match
the header as compiled by a C compiler."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1012_2865_amd import moray as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "moray.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(moray_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    assert _declared_functions() == sorted(M.ABI_FUNCTIONS)


def test_library_exports_every_declared_function():
    lib = M.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (moray_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_version_string():
    assert re.fullmatch(r"\d+\.\d+\.\d+", M.moray_version())


def test_init_without_gpu_reports_edevice():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    with pytest.raises(M.MorayError) as e:
        M.moray_init(device=0, hip_stream=0)
    assert e.value.status == M.MORAY_EDEVICE


def test_init_rejects_bad_parameters_before_touching_the_device():
    lib = M.load_library()
    h = ctypes.c_void_p()
    p = M.InitParams(0, 7, 0, 0, 0, 0, 0, None, 0, 0, 0)        # unknown precision
    assert lib.moray_init(ctypes.byref(h), ctypes.byref(p)) == M.MORAY_EINVAL
    p = M.InitParams(0, 1, 0, 0, 0, 65, 0, None, 0, 0, 0)       # more idle lanes than a wave has
    assert lib.moray_init(ctypes.byref(h), ctypes.byref(p)) == M.MORAY_EINVAL
    assert lib.moray_init(None, ctypes.byref(p)) == M.MORAY_EINVAL
    assert not h.value
    assert M.moray_last_error(None) == "context pointer is NULL"
    lib.moray_free(None)


_LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "moray.h"
#define S(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  S(moray_init_params) O(moray_init_params, hip_stream) O(moray_init_params, profile) O(moray_init_params, deposit_cache) O(moray_init_params, reserve_rays)
  S(moray_source) S(moray_spectrum) O(moray_spectrum, e_ion_ev)
  S(moray_grid) O(moray_grid, offset) O(moray_grid, n_h) O(moray_grid, x_hi)
  S(moray_trace_params) O(moray_trace_params, p_min_frac) O(moray_trace_params, covering) O(moray_trace_params, tau_thin)
  S(moray_problem) O(moray_problem, params)
  S(moray_result) O(moray_result, accel) O(moray_result, emitted) O(moray_result, segments) O(moray_result, peak_level_rays)
  O(moray_result, trace_ms) O(moray_result, trace_launches) O(moray_result, t_admit) O(moray_result, t_done) O(moray_result, from_graph) O(moray_result, thin_segments)
  S(moray_equilibrium_params) O(moray_equilibrium_params, tol) O(moray_equilibrium_params, max_iter)
  S(moray_evolve_params) O(moray_evolve_params, tau_front) O(moray_evolve_params, t_end) O(moray_evolve_params, max_steps)
  return 0;
}
"""


def test_binding_struct_layout_matches_header():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write(_LAYOUT_C)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        got = dict(line.split() for line in subprocess.check_output([exe], text=True).splitlines())
    py = {"moray_init_params": M.InitParams, "moray_source": M.Source, "moray_spectrum": M.Spectrum,
          "moray_grid": M.Grid, "moray_trace_params": M.TraceParams, "moray_problem": M.Problem,
          "moray_result": M.Result, "moray_equilibrium_params": M.EquilibriumParams,
          "moray_evolve_params": M.EvolveParams}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(py[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(py[key]) == int(val), key


def test_equilibrate_rejects_null_context():
    lib = M.load_library()
    ep = M.EquilibriumParams(M.ALPHA_B, 0.5, 1e-6, 10)
    assert lib.moray_equilibrate(None, None, 1, ctypes.byref(ep), None, None, None) == M.MORAY_EINVAL


def test_evolve_rejects_null_context():
    lib = M.load_library()
    ep = M.EvolveParams(M.ALPHA_B, 0.1, 0.5, 1e13, 1e14, 10)
    assert lib.moray_evolve(None, None, 1, ctypes.byref(ep), None, None, None, None, None) == M.MORAY_EINVAL


def test_time_dependent_entry_points_reject_null_context():
    lib = M.load_library()
    h = ctypes.c_void_p()
    assert lib.moray_td_create(None, None, 4.0, 1 << 16, ctypes.byref(h)) == M.MORAY_EINVAL
    assert not h.value
    held = ctypes.c_double(0.0)
    assert lib.moray_td_step(None, None, None, 3, 1, None, ctypes.byref(held)) == M.MORAY_EINVAL
    lib.moray_td_free(None, None)


def test_async_entry_points_reject_null_context():
    lib = M.load_library()
    t = ctypes.c_ulonglong(0)
    assert lib.moray_trace_async(None, None, 1, 0, None, ctypes.byref(t)) == M.MORAY_EINVAL
    assert lib.moray_query(None, ctypes.c_ulonglong(1), 0) == M.MORAY_EINVAL


def test_c_caller_compiles_against_the_header():
    with tempfile.TemporaryDirectory() as d:
        here = os.path.dirname(os.path.abspath(__file__))
        libdir = os.path.dirname(M.LIB_PATH)
        subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                               os.path.join(here, "capi_host_demo.c"), "-L", libdir, "-lmoray",
                               "-o", os.path.join(d, "demo")])


def test_microbenchmark_library_exports_its_entry_point():
    # the device-peak microbenchmark that bench.py prices the rooflines against
    path = os.path.join(ROOT, "paper_1012_2865_amd", "libmoray_microbench.so")
    if not os.path.exists(path):
        pytest.skip("libmoray_microbench.so is not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    assert re.search(r" T moray_microbench$", out, flags=re.M)
    assert re.search(r" T moray_microbench_case$", out, flags=re.M)


def test_prepared_batch_descriptors_match_a_fresh_marshal():
    """The descriptors a PreparedBatch keeps are those moray_trace builds for
    the same host problems and buffers (pointers, shapes, sources, spectrum),
    and its per-grid result views alias the caller's buffers."""
    import numpy as np
    from paper_1012_2865_amd import workloads as W
    probs = [W.config0(), W.lognormal_problem(97, 1, 16, 2)]
    outs = [(np.zeros(p.grids[0].n_h.size), np.zeros(p.grids[0].n_h.size)) for p in probs]
    b = M.PreparedBatch(probs, outputs=outs, out_on_device=False)
    cp, res, keep, o, flags = M._marshal(probs, False, False, outs)
    assert b.n == 2 and b.flags == flags == 0
    for i in range(2):
        P, Q = b.cprobs[i], cp[i]
        assert (P.n_grids, P.n_sources) == (Q.n_grids, Q.n_sources)
        assert (P.grids[0].nx, P.grids[0].ny, P.grids[0].nz) == (Q.grids[0].nx, Q.grids[0].ny, Q.grids[0].nz)
        assert ctypes.cast(P.grids[0].n_h, ctypes.c_void_p).value == ctypes.cast(Q.grids[0].n_h, ctypes.c_void_p).value
        for k in range(P.n_sources):
            assert (P.sources[k].x, P.sources[k].ndot) == (Q.sources[k].x, Q.sources[k].ndot)
        assert P.spectrum[0].n_groups == Q.spectrum[0].n_groups
        assert b.results[i].k_ph == res[i].k_ph == outs[i][0].ctypes.data
        view = b.views[i]["k_ph"][0]
        assert view.shape == probs[i].grids[0].n_h.shape and np.shares_memory(view, outs[i][0])


def test_binding_loads_torch_before_the_library():
    """PyTorch's HIP runtime must be in the process before the library's, so
    that the library shares it (a second runtime leaves one without a device)."""
    code = "import sys; from paper_1012_2865_amd import moray as M; M.load_library(); print('torch' in sys.modules)"
    out = subprocess.check_output(["python", "-c", code], cwd=ROOT, text=True).strip().splitlines()[-1]
    assert out == "True"
