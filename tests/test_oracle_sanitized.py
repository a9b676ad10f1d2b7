"""The oracle's memory handling under AddressSanitizer and UndefinedBehaviorSanitizer:
a plain-C driver (sanitize/oracle_driver.c) runs every oracle entry point (both
buffer schemes, both precision policies, staged events with admission, cell
scoring, instrumentation, a capacity overflow, a state hand-over, free-slot rings
that wrap around) in a build with both sanitizers, any report fatal."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-I", ORACLE, os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ORACLE, "oracle.c"), "-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle driver ok" in r.stdout
