"""CPU builds of the host-side code under AddressSanitizer + UndefinedBehaviorSanitizer.

* The library's scheme construction (csrc/scheme_design.cpp: named schemes, the centred, biased and
  dissipation generators, the general Taylor solver, the checks) with tests/sanitize/scheme_selftest.cpp.
* The oracle's C line operator (oracle/lines.c) with tests/sanitize/oracle_selftest.c.

Built with g++/gcc on the host (no GPU code); the sanitizers abort the program on any error.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd, env=None):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitize"))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_scheme_construction_under_sanitizers(workdir):
    exe = os.path.join(workdir, "scheme_selftest")
    _run(["g++", "-std=gnu++17", "-fext-numeric-literals", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I" + os.path.join(ROOT, "paper_2302_14858_amd", "csrc"),
          os.path.join(ROOT, "tests", "sanitize", "scheme_selftest.cpp"),
          os.path.join(ROOT, "paper_2302_14858_amd", "csrc", "scheme_design.cpp"),
          "-lquadmath", "-o", exe], ROOT)
    out = _run([exe], ROOT, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "OK (0 failures)" in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_line_operator_under_sanitizers(workdir):
    exe = os.path.join(workdir, "oracle_selftest")
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_selftest.c"),
          os.path.join(ROOT, "oracle", "lines.c"), "-lm", "-o", exe], ROOT)
    out = _run([exe], ROOT, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "OK (0 failures)" in out, out
