"""CPU builds of the oracle and of the library's host-only C++ (lattice
builder, spline and setfl code, PTA arithmetic) with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc / g++, -fno-sanitize-recover: the first
report ends the run), each driven by a small program under
tests/sanitize/ that exercises their entry points, including short
capacities, truncated files and bad arguments.  The device code is not part
of these builds (no sanitizer runs on the GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, cwd, env=None, timeout=300):
    return subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    b = _run(["gcc", "-std=c11", "-ffp-contract=off", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
              os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
              "-o", exe, "-lm"], cwd=str(tmp_path))
    if b.returncode != 0 and "asan" in b.stderr.lower():
        pytest.skip("no sanitizer runtime: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4")
    r = _run([exe], cwd=str(tmp_path), env=env)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_2603_07321_amd", "csrc")
    b = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", csrc,
              os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
              *[os.path.join(csrc, f) for f in ("lattice.cpp", "eam_table.cpp", "pta.cpp")], "-o", exe],
             cwd=str(tmp_path))
    if b.returncode != 0 and "asan" in b.stderr.lower():
        pytest.skip("no sanitizer runtime: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    r = _run([exe, str(tmp_path)], cwd=str(tmp_path))
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
