"""The FP64 oracle and the host side of the C ABI under the address and
undefined-behaviour sanitizers (CPU only): each is built with them into a
small driver program (tests/sanitize/) that runs it through its paths, and
the run must end cleanly with no sanitizer report.

* Oracle: gcc, every part of the step (mixed and inflow boundaries, the
  three fixed potentials, floors, both MUSCL forms and first order, the
  three solvers, passive scalars, the learned correction, self-gravity with
  particles, the single-face entry points); leak checking on.
* ABI: hipcc with the sanitizers on the host code only (the device code
  is built as usual); configuration checking and the workspace arithmetic
  for every boundary kind, solver, reconstruction and source, and the
  argument checks each entry point makes before touching a device.  Leak
  checking is off: the HIP runtime keeps allocations to the end of the
  process.
"""
import concurrent.futures
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1502_02935_amd", "csrc")
HIP_SOURCES = ("mhd_abi.hip", "mhd_kernels.hip", "mhd_flux.hip", "mhd_mlp.hip",
               "mhd_gravity.hip", "mhd_nbody.hip")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_driver")
        rc, out = _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(SAN, "orc_driver.c"), os.path.join(ROOT, "oracle", "orc.c"),
                        "-lm", "-o", exe])
        assert rc == 0, out
        env = dict(os.environ, OMP_NUM_THREADS="2",
                   ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "checksum" in out and "ERROR" not in out and "runtime error" not in out, out


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_under_sanitizers():
    # sanitizers on the host compilation only: each -fsanitize= follows -Xarch_host
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory() as d:
        srcs = [os.path.join(SAN, "abi_driver.cpp")] + [os.path.join(CSRC, s) for s in HIP_SOURCES]
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in srcs]
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            res = list(ex.map(lambda so: _run([HIPCC, *flags, "-c", so[0], "-o", so[1]]),
                              zip(srcs, objs)))
        for rc, out in res:
            assert rc == 0, out
        exe = os.path.join(d, "abi_driver")
        rocm_lib = os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "lib")
        rc, out = _run([HIPCC, *flags, *objs, "-L" + rocm_lib, "-Wl,-rpath," + rocm_lib,
                        "-lrocprofiler-sdk-roctx", "-o", exe])
        assert rc == 0, out
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
        rc, out = _run([exe], env=env)
    assert rc == 0, out
    assert "0 failures" in out and "ERROR" not in out and "runtime error" not in out, out
