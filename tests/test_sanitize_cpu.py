"""The library's host-only code (threshold table, greedy colouring, error
strings) and the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, built with the host compilers (no GPU code)."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
DRIVER = ROOT / "tests" / "helpers" / "sanitize_host.cpp"
HOST = ROOT / "paper_2510_23419_amd" / "csrc" / "host.cpp"
ORACLE = ROOT / "oracle" / "pbit_oracle.c"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
       "-ffp-contract=off"]


def test_host_code_and_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("host compilers not available")
    oracle_o = tmp_path / "oracle.o"
    subprocess.run(["gcc", "-std=c11", "-c", str(ORACLE), "-o", str(oracle_o)] + SAN, check=True)
    exe = tmp_path / "sanitize_host"
    subprocess.run(["g++", "-std=c++17", "-pthread", str(DRIVER), str(HOST), str(oracle_o), "-o", str(exe), "-lm"]
                   + SAN, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_serving_scheduler_policy_with_a_stub_device(tmp_path):
    """serve_sched.h, the admission and round policy of the serving loop, driven
    by a host stub of the device (under the sanitizers too)."""
    if not shutil.which("g++"):
        pytest.skip("host compiler not available")
    exe = tmp_path / "sched_stub"
    subprocess.run(["g++", "-std=c++17", "-I" + str(ROOT / "paper_2510_23419_amd" / "csrc"),
                    str(ROOT / "tests" / "helpers" / "sched_stub.cpp"), "-o", str(exe)] + SAN, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sched ok" in r.stdout
