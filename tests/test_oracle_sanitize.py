"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize_driver.c compiles the oracle's single C file together
with a driver that runs every solver path on small problems, with each
output array allocated at exactly its documented size.  Any out-of-bounds
access, use after free, leak or undefined behaviour (signed overflow,
misaligned or null access, out-of-range shift) ends the run with a report.
CPU only; skipped when gcc's sanitizer runtimes are not installed.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
           "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("gcc sanitizer runtimes not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_clean_under_sanitizers(driver):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    if r.returncode != 0 and "LeakSanitizer has encountered a fatal error" in r.stderr:
        # leak checking needs ptrace, which some containers refuse
        env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
        r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert "runtime error" not in report, report
    assert "AddressSanitizer" not in report, report
    assert r.returncode == 0, report
    assert "failures 0" in r.stdout
