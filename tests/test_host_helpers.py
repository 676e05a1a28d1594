"""CPU checks of the device helpers that are plain arithmetic (compiled with
hipcc as host code, no GPU needed): the table-driven log used for the
Equation 2 distance against the C library log, and the bit-sliced
carry-save counting + plane transpose against direct counting; the rank
launch's host logic (work lists, per-XCD queues, fixed-point scale)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_helpers_on_host(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "helpers_check")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_0905_1744_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "helpers_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_worklists_on_host(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "worklist_check")
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_0905_1744_amd", "csrc"),
                        os.path.join(ROOT, "tests", "host", "worklist_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    """The oracle's C built with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), driven through every entry point and edge case."""
    exe = str(tmp_path / "oracle_sanitize")
    r = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer",
                        os.path.join(ROOT, "oracle", "kd_oracle.c"),
                        os.path.join(ROOT, "tests", "host", "oracle_sanitize.c"), "-o", exe, "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
