"""A plain C caller of the ABI (tests/capi_host_demo.c: only moray.h and
libmoray.so, host fields and results, no Python or HIP calls) traces two
problems in one batch, in both precisions; its totals and k_ph/heating sums
equal the Python binding's for the same inputs (counts exactly, sums to
1e-12 relative)."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1012_2865_amd import moray as M
from paper_1012_2865_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _write_input(path, problems):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(problems)))
        for p in problems:
            g = p.grids[0]
            nz, ny, nx = g.n_h.shape
            sp, pr = p.spectrum, p.params
            f.write(struct.pack("<5i", nx, ny, nz, p.n_sources, len(sp.energy_ev)))
            f.write(struct.pack("<4d", g.dx_cm, sp.e_ion_ev, pr.phi_c, pr.p_min_frac))
            f.write(struct.pack("<2i", pr.level_init, pr.level_max))
            f.write(np.ascontiguousarray(g.n_h, np.float32).tobytes())
            f.write(np.ascontiguousarray(g.x_hi, np.float32).tobytes())
            f.write(np.ascontiguousarray(p.sources, np.float64).tobytes())
            for a in (sp.energy_ev, sp.sigma_cm2, sp.frac):
                f.write(np.ascontiguousarray(a, np.float64).tobytes())


def test_c_caller_matches_binding():
    problems = [W.lognormal_problem(91, 0, 20, 2), W.lognormal_problem(91, 1, 28, 3, params=W.Params(level_init=0))]
    with tempfile.TemporaryDirectory() as d:
        exe, inp = os.path.join(d, "demo"), os.path.join(d, "input.bin")
        libdir = os.path.dirname(M.LIB_PATH)
        subprocess.check_call(["gcc", "-std=c11", "-O1", "-I", os.path.join(ROOT, "include"),
                               os.path.join(HERE, "capi_host_demo.c"), "-L", libdir, "-lmoray",
                               "-Wl,-rpath," + libdir, "-o", exe])
        _write_input(inp, problems)
        out = subprocess.run([exe, inp], capture_output=True, text=True, timeout=120)
        print(out.stdout, out.stderr, flush=True)
        assert out.returncode == 0
    rows = {}
    for line in out.stdout.splitlines():
        t = line.split()
        if t[0] == "precision":
            rows[(int(t[1]), int(t[3]))] = {t[k]: float(t[k + 1]) for k in range(4, len(t), 2)}
    for prec in (M.MORAY_FP64, M.MORAY_FP32_ACC64):
        ctx = M.moray_init(device=0, precision=prec)
        try:
            ref = M.moray_trace(ctx, problems, out_on_device=False)
        finally:
            M.moray_free(ctx)
        for i, r in enumerate(ref):
            c = rows[(prec, i)]
            assert c["segments"] == r["segments"] and c["splits"] == r["splits"]
            for k in ("emitted", "absorbed", "escaped", "truncated"):
                assert c[k] == pytest.approx(r[k], rel=1e-12, abs=1e-12 * r["emitted"]), (prec, i, k)
            assert c["sum_kph"] == pytest.approx(float(np.sum(r["k_ph"][0])), rel=1e-12)
            assert c["sum_heat"] == pytest.approx(float(np.sum(r["heating"][0])), rel=1e-12)
