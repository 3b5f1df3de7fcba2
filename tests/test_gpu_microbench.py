"""The device-peak microbenchmark on the GPU: its measured scattered and
coherent float64 atomic rates and its copy bandwidth are positive, ordered as
the memory system makes them (coherent lanes share lines, so they are at
least as fast as scattered ones) and below what the hardware can do (a copy
under the 8 TB/s HBM peak)."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_microbenchmark_rates_are_plausible():
    path = os.path.join(ROOT, "paper_1012_2865_amd", "libmoray_microbench.so")
    assert os.path.exists(path), "build libmoray_microbench.so first"
    lib = ctypes.CDLL(path)
    lib.moray_microbench.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.moray_microbench.restype = ctypes.c_int
    out = (ctypes.c_double * 3)()
    assert lib.moray_microbench(0, out) == 0
    scattered, coherent, copy_gbs = out[0], out[1], out[2]
    print(f"scattered {scattered:.3e}/s coherent {coherent:.3e}/s copy {copy_gbs:.0f} GB/s", flush=True)
    assert 1e8 < scattered <= coherent * 1.05
    assert coherent < 1e12
    assert 100.0 < copy_gbs < 8000.0
