"""The C-ABI library loads and exports every function include/hk.h declares;
argument validation that needs no GPU (CPU-only: no device work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hk.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hk_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def hk():
    import paper_2502_02721_amd as hk
    if not os.path.exists(hk.LIB_PATH):
        from paper_2502_02721_amd import build
        build.build()
    return hk


def test_header_lists_the_binding_functions(hk):
    assert header_functions() == sorted(hk.ABI_FUNCTIONS)


def test_library_exports_every_header_function(hk):
    raw = C.CDLL(hk.LIB_PATH)
    for name in header_functions():
        assert hasattr(raw, name), name


def test_version_and_null_argument_errors(hk):
    L = hk.lib()
    assert hk.hk_abi_version() == 2
    assert L.hk_solve_wait(None) == hk.HK_EINVAL
    assert "null" in hk.hk_last_error()
    assert L.hk_op_destroy(None) == hk.HK_EINVAL
    assert L.hk_context_destroy(None) == hk.HK_EINVAL
    assert L.hk_context_create(0, None, None) == hk.HK_EINVAL
    assert L.hk_op_create_blur(None, 4, 4, None, None, 1, 0, 0, None) == hk.HK_EINVAL
    assert L.hk_solve_create(None, None, None) == hk.HK_EINVAL
    assert L.hk_solve_create_with_workspace(None, None, None, 0, None) == hk.HK_EINVAL
    assert L.hk_solve_get_true_residuals(None, None) == hk.HK_EINVAL
    assert L.hk_solve_get_prefix_solution(None, 1, None) == hk.HK_EINVAL
    assert L.hk_solve_grid(None, None) == hk.HK_EINVAL
    assert L.hk_solve_select_rhs(None, 0) == hk.HK_EINVAL
    assert L.hk_solve_run_noalloc(None, None, None, None, None) == hk.HK_EINVAL
    # the serving loop: null handles are refused before any device work
    assert L.hk_server_create(None, 4, 0, 0, None) == hk.HK_EINVAL
    assert L.hk_server_destroy(None) == hk.HK_EINVAL
    assert L.hk_server_submit(None, None, None, None, None, None) == hk.HK_EINVAL
    assert L.hk_server_poll(None, None) == hk.HK_EINVAL
    assert L.hk_server_wait(None, 0) == hk.HK_EINVAL
    assert L.hk_server_result(None, 0, None, None, None, None, None, None) == hk.HK_EINVAL


def test_unknown_handles_are_refused_without_use(hk):
    """A handle the library did not create (or has destroyed) is refused with
    HK_EINVAL before its memory is read: the address below is never mapped
    as a handle."""
    import ctypes as C
    L = hk.lib()
    bogus = C.c_void_p(0x10)
    assert L.hk_solve_wait(bogus) == hk.HK_EINVAL
    assert "unknown or destroyed" in hk.hk_last_error()
    assert L.hk_solve_destroy(bogus) == hk.HK_EINVAL
    assert L.hk_op_destroy(bogus) == hk.HK_EINVAL
    assert L.hk_context_destroy(bogus) == hk.HK_EINVAL
    assert L.hk_server_destroy(bogus) == hk.HK_EINVAL
    assert L.hk_server_poll(bogus, None) == hk.HK_EINVAL


def test_log_level_one_reports_refused_calls(hk):
    """HK_LOG=1: a refused call is also written to stderr (the level is read
    once per process, so this runs in a child)."""
    import subprocess
    import sys
    code = "import paper_2502_02721_amd as hk; hk.lib().hk_solve_wait(None)"
    env = dict(os.environ, HK_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "hk: status -1: null handle sv" in r.stderr
    env["HK_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert "hk:" not in r.stderr


def test_params_struct_layout(hk, tmp_path):
    """The ctypes mirror of hk_params matches the C header, as compiled by gcc."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"hk.h\"\n"
        "int main(void) { printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(hk_params),"
        " offsetof(hk_params, lambda), offsetof(hk_params, seed), offsetof(hk_params, basis_dtype),"
        " offsetof(hk_params, flags), offsetof(hk_params, pivot_sample)); return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    P = hk.hk_params
    assert got == [C.sizeof(P), P.lambda_.offset, P.seed.offset, P.basis_dtype.offset, P.flags.offset,
                   P.pivot_sample.offset]
