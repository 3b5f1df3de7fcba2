"""The device-peak microbenchmark on the GPU: its measured scattered and
coherent float64 atomic rates and its copy bandwidth are positive, ordered as
the memory system makes them (coherent lanes share lines, so they are at
least as fast as scattered ones) and below what the hardware can do (a copy
under the 8 TB/s HBM peak); single sweep points reject arguments outside
their documented ranges and agree in order of magnitude with the fixed
shape."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MIB = 1 << 20


def _lib():
    path = os.path.join(ROOT, "paper_1012_2865_amd", "libmoray_microbench.so")
    assert os.path.exists(path), "build libmoray_microbench.so first"
    lib = ctypes.CDLL(path)
    lib.moray_microbench.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.moray_microbench.restype = ctypes.c_int
    lib.moray_microbench_case.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.moray_microbench_case.restype = ctypes.c_int
    return lib


def test_microbenchmark_rates_are_plausible():
    lib = _lib()
    out = (ctypes.c_double * 3)()
    assert lib.moray_microbench(0, out) == 0
    scattered, coherent, copy_gbs = out[0], out[1], out[2]
    print(f"scattered {scattered:.3e}/s coherent {coherent:.3e}/s copy {copy_gbs:.0f} GB/s", flush=True)
    assert 1e8 < scattered <= coherent * 1.05
    assert coherent < 1e12
    assert 100.0 < copy_gbs < 8000.0


def test_sweep_points():
    lib = _lib()
    r = ctypes.c_double(0.0)
    # arguments outside the documented ranges are rejected before any launch
    for args in ((0, 100 * MIB, 8, 64, 1), (0, 128 * MIB, 0, 64, 1), (0, 128 * MIB, 8, 64, 3), (0, 128 * MIB, 8, 0, 1),
                 (1, 1000, 8, 4, 1), (1, 1 << 30, 8, 3, 1), (5, 1 << 30, 8, 4, 1), (3, 1 << 34, 8, 4, 1)):
        assert lib.moray_microbench_case(0, *args, ctypes.byref(r)) == -1, args
    rates = {}
    for name, args in (("scattered", (0, 128 * MIB, 8, 64, 1)), ("runs64", (0, 128 * MIB, 8, 64, 64)),
                       ("copy", (1, 1 << 30, 4, 4, 1)), ("copy_nt", (2, 1 << 30, 4, 4, 1)),
                       ("read", (3, 1 << 30, 4, 4, 1)), ("read_nt", (4, 1 << 30, 4, 4, 1))):
        assert lib.moray_microbench_case(0, *args, ctypes.byref(r)) == 0, name
        rates[name] = r.value
    print(rates, flush=True)
    assert 1e8 < rates["scattered"] <= rates["runs64"] * 1.05 < 2e12
    for k in ("copy", "copy_nt", "read", "read_nt"):
        assert 100.0 < rates[k] < 8000.0, k
