"""Host builds under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the oracle's every entry point (gcc), and the library's exact predicates
(exact.hpp, host code only) against their own exact expansion.  A report
from either sanitizer fails the run (no recovery)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_oracle")
    subprocess.check_call([
        "gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
        "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "oracle.c"),
        os.path.join(NATIVE, "sanitize_oracle.c"), "-o", exe, "-lm"])
    assert "ok" in _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})


def test_exact_predicates_under_sanitizers(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "san_exact")
    # host code only; each sanitizer flag applies to the host pass
    subprocess.check_call([
        hipcc, "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all",
        "-I", os.path.join(ROOT, "paper_1508_05931_amd", "csrc"),
        os.path.join(NATIVE, "sanitize_exact.cpp"), "-o", exe],
        stderr=subprocess.DEVNULL)
    assert "ok" in _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
