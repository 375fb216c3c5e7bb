"""Sanitizer builds of the host code (CPU only): the library's constant solves
and description validation, and the oracle's C sources, compiled with
AddressSanitizer and UndefinedBehaviorSanitizer by the plain host compilers
and run on small, odd and malformed inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_05869_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitizers")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    subprocess.check_call(cmd, cwd=ROOT)
    # other preloaded libraries may precede the ASan runtime: do not insist on
    # being first in the link order
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_constants_and_validation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "host_driver.cpp"), os.path.join(CSRC, "constants.cpp"),
           os.path.join(CSRC, "validate.cpp"), "-o", exe]
    _run(cmd, exe, tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_c_sources_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11", *SAN, "-ffp-contract=off", os.path.join(HERE, "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "sweep.c"), os.path.join(ROOT, "oracle", "spectral.c"),
           "-lm", "-o", exe]
    _run(cmd, exe, tmp_path)
