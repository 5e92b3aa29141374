"""The oracle's C code and the host planner under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: tests/sanitize/oracle_drive.c runs
the codec at every rate on special blocks and arbitrary byte strings, the
stencils and gradients on tiny and ragged grids; tests/sanitize/plan_drive.cpp
plans and race-checks the forward and adjoint operation lists over a sweep of
configurations (the bench job's included).  Each is compiled with gcc / g++
and the sanitizers, then run; any report fails the test (no recovery)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2204_11315_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(cmd, exe, tmp_path):
    if shutil.which(cmd[0]) is None:
        pytest.skip("%s not found" % cmd[0])
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("compiler without sanitizer runtimes: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    return r.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    src = [os.path.join(HERE, "sanitize", "oracle_drive.c")] + [
        os.path.join(ORACLE, f) for f in ("codec_ref.c", "stencil_ref.c", "wave_ref.c")]
    out = _build_and_run(["gcc", "-std=c11", "-fopenmp", "-I" + ORACLE] + SAN + src + ["-lm"],
                         str(tmp_path / "oracle_drive"), tmp_path)
    assert "clean" in out


def test_host_planner_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    src = [os.path.join(HERE, "sanitize", "plan_drive.cpp"), os.path.join(CSRC, "oc_plan.cpp")]
    out = _build_and_run(["g++", "-std=c++17", "-I" + CSRC] + SAN + src,
                         str(tmp_path / "plan_drive"), tmp_path)
    assert "clean" in out
