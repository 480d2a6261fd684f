"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer,
on a GPU.

tests/_build/hk_host_san (built by tests/build_host_sanitize.py, which
__graft_entry__.build() runs) links the library's sources, sanitized on the
host side only, with tests/host_sanitize_driver.cpp.  The driver goes
through the C ABI: operators, solves and every getter, prefix solutions,
true residuals, several right-hand sides, the caller-owned workspace, the
allocation-free run, the serving loop and the argument checks.  Each host
output array has exactly its documented size.  Any heap or stack overrun,
use after free or undefined behaviour in the runtime ends the run with a
report.  Leak checking is off: the HIP runtime keeps allocations until
the process exits.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "hk_host_san")


def test_host_runtime_clean_under_sanitizers():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/_build/hk_host_san is missing: run __graft_entry__.build()"
    env = dict(os.environ)
    # the sanitizer runtime is linked in; other preloaded libraries may come first
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    print("running the host-sanitized driver", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=180)
    report = r.stdout + r.stderr
    print(r.stdout[-2000:], flush=True)
    assert "AddressSanitizer" not in report, report[-4000:]
    assert "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "failures 0" in r.stdout
