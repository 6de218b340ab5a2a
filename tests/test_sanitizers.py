"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

* The oracle (plain C) built with gcc -fsanitize=address,undefined runs its own pins: every test in
  tests/test_oracle_*.py, in a child process with the sanitizer runtime preloaded.
* The library's host code (argument validation, coefficient set-up, planning) built with clang's
  sanitizers, linked with the kernel units, runs the ABI tests of tests/test_abi.py.

A sanitizer report or a non-zero exit fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_MARKERS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "UndefinedBehaviorSanitizer")


def _run_child(args, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args], cwd=ROOT,
                          env=env, capture_output=True, text=True, timeout=timeout)


def _assert_clean(proc):
    out = proc.stdout + proc.stderr
    for m in REPORT_MARKERS:
        assert m not in out, out[-4000:]
    assert proc.returncode == 0, out[-4000:]


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    src = os.path.join(ROOT, "oracle", "sc_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-o", lib, src, "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    proc = _run_child([*tests, "-m", "not gpu"], {"LD_PRELOAD": asan, "SC_ORACLE_LIBRARY_PATH": lib}, timeout=900)
    _assert_clean(proc)


def test_host_library_abi_under_sanitizers(tmp_path):
    from paper_2007_03041_amd import build as b

    rt = b.asan_runtime()
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    lib = b.build_sanitized(str(tmp_path))
    proc = _run_child([os.path.join("tests", "test_abi.py")], {"LD_PRELOAD": rt, "SC_LIBRARY_PATH": lib}, timeout=600)
    _assert_clean(proc)
