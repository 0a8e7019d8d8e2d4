"""The C reference (oracle/lb_oracle.c) built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven through every call, argument checks
included, on small single and binary lattices with one and two threads
(tests/c/oracle_sanitize_driver.c).  Host code only; no GPU involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_reference_under_address_and_ub_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_sanitized"
    cmd = [cc, "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-Wall", "-Werror",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "lb_oracle.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "ERROR" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
