"""CPU sanitizer builds (no GPU needed).

* The oracle, compiled with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc), runs every entry point on small problems -- uniform and irregular
  media, general source positions, a refined child grid, the covering factor,
  radiation pressure, time-dependent steps and rejected inputs -- and must
  finish clean with photon conservation held (oracle/sanitize_driver.c).
* The library's host code (runtime, serving engine, time-dependent state),
  compiled for the host only with the same sanitizers, runs its entry points
  with NULL contexts and bad parameters, context creation without a device,
  and the problem validation and queue-sizing routines on valid and invalid
  problems (tests/sanitize_runtime.cpp).
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_2865_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1012_2865_amd", "_build")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    return r.returncode, r.stdout, err


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_san")
        rc, out, err = _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-I",
                             os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "sanitize_driver.c"),
                             os.path.join(ROOT, "oracle", "moray_oracle.c"), "-lm", "-o", exe])
        assert rc == 0, err
        rc, out, err = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1"), timeout=600)
        print(out)
        assert rc == 0 and "ALL OK" in out, err[-4000:]
        assert "runtime error" not in err and "AddressSanitizer" not in err, err[-4000:]


@pytest.mark.slow
def test_library_host_code_under_sanitizers():
    objs = [os.path.join(BUILD, f) for f in ("moray_kernels.o", "moray_equilibrium.o", "moray_td_kernels.o",
                                             "moray_noalloc.o")]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the library's objects are not built (run __graft_entry__.build())")
    san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", CSRC, "-I",
              os.path.join(ROOT, "include")] + san
    with tempfile.TemporaryDirectory() as d:
        built = []
        for src in (os.path.join(CSRC, "moray_runtime.cpp"), os.path.join(CSRC, "moray_serve.cpp"),
                    os.path.join(CSRC, "moray_td.cpp"), os.path.join(CSRC, "moray_tune_cache.cpp"),
                    os.path.join(ROOT, "tests", "sanitize_runtime.cpp")):
            o = os.path.join(d, os.path.basename(src) + ".o")
            rc, _, err = _run([HIPCC] + common + ["-c", src, "-o", o])
            assert rc == 0, err
            built.append(o)
        exe = os.path.join(d, "rt_san")
        rc, _, err = _run([HIPCC, "--offload-arch=gfx950"] + san + built + objs + ["-pthread", "-o", exe])
        assert rc == 0, err
        rc, out, err = _run([exe], env=ENV, timeout=300)
        print(out)
        assert rc == 0 and "ALL OK" in out, (out[-3000:], err[-3000:])
        assert "runtime error" not in err and "AddressSanitizer" not in err, err[-4000:]
