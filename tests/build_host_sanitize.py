"""Build tests/_build/hk_host_san: the library's sources and
tests/host_sanitize_driver.cpp linked into one executable, with
AddressSanitizer and UndefinedBehaviorSanitizer on the host side only (each
-fsanitize option behind -Xarch_host; the device code is built as for
libhk.so).  tests/test_gpu_host_sanitize.py runs it on a GPU.

Usage: python tests/build_host_sanitize.py   (or call build())
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2502_02721_amd import build as hkbuild  # noqa: E402

OUT_DIR = os.path.join(HERE, "_build")
EXE = os.path.join(OUT_DIR, "hk_host_san")
DRIVER = os.path.join(HERE, "host_sanitize_driver.cpp")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hkbuild.HIPCC, *hkbuild.FLAGS, *SAN, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip", "-g"]      # host code: line numbers in the reports
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = [os.path.join(hkbuild.CSRC, s) for s in hkbuild.SOURCES] + [DRIVER]
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = EXE + ".tmp"
    cmd = [hkbuild.HIPCC, f"--offload-arch={hkbuild.ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, EXE)
    if verbose:
        print(f"built {EXE}")
    return EXE


if __name__ == "__main__":
    build(verbose=True)
