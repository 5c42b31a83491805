"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU only).

Two programs are built in a temporary directory and run:
- the HIP library's sources, compiled with both sanitizers on the host pass
  (the device code is compiled as usual and never launched), linked with
  tests/sanitize/host_checks.cpp: the mesh and kinetic + Bloch matrix, the
  host Coulomb routine, the workspace arithmetic and the argument checks of
  every entry point, all without a device;
- the oracle's Gaussian elimination (oracle/ge.c), compiled with gcc and both
  sanitizers, linked with tests/sanitize/ge_checks.c.
A sanitizer report, a leak or a failed check fails the test."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_11590_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_SOURCES = ["assemble.hip", "lu.hip", "gemm.hip", "gemm_h3.hip", "solve.hip", "wsolve.hip", "coulomb.hip",
               "abi.hip", "trace.hip", "batch.hip", "woodbury.hip"]
# sanitizers on the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
RUN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, cwd, env=None):
    r = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:]
    return r.stdout


def _env():
    env = dict(os.environ)
    env.update(RUN_ENV)
    return env


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_library_under_sanitizers(tmp_path):
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, *HOST_SAN]
    jobs = [[HIPCC, "--offload-arch=gfx950", *flags, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-c", os.path.join(CSRC, s), "-o", s + ".o"] for s in HIP_SOURCES]
    jobs.append([HIPCC, *flags, "-x", "c++", "-c", os.path.join(CSRC, "mesh.cpp"), "-o", "mesh.o"])
    jobs.append([HIPCC, *flags, "-x", "c++", "-c", os.path.join(HERE, "host_checks.cpp"), "-o", "host_checks.o"])
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda c: _run(c, str(tmp_path)), jobs))
    objs = [s + ".o" for s in HIP_SOURCES] + ["mesh.o", "host_checks.o"]
    _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, *objs, "-o", "host_checks"], str(tmp_path))
    exe = tmp_path / "host_checks"
    assert b"__asan_report" in exe.read_bytes() and b"__ubsan_handle" in exe.read_bytes()
    out = _run([str(exe)], str(tmp_path), env=_env())
    assert "host checks ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_elimination_under_sanitizers(tmp_path):
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "ge.c"), os.path.join(HERE, "ge_checks.c"),
          "-o", "ge_checks", "-lm"], str(tmp_path))
    out = _run([str(tmp_path / "ge_checks")], str(tmp_path), env=_env())
    assert "oracle elimination checks ok" in out
