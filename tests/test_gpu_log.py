"""HK_LOG=2 on a GPU: each solve's plan (kernel, grid, tiles, LDS,
workspace) and each server admission are written to stderr.  The level is
read once per process, so the solve runs in a child process."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import numpy as np, torch
import paper_2502_02721_amd as hk
ctx = hk.Context(0)
op = hk.Operator.gaussian_blur(ctx, 64, 64, 2.0, 6, 1, hk.HK_F64)
sv = hk.Solve(op, 10, 22, 0.0, 0, 4, 7)
x = sv.run(torch.tensor(np.random.default_rng(0).standard_normal(4096), device="cuda:0"))
print("status", sv.wait(), flush=True)
srv = hk.Server(ctx, slots=2)
b = torch.tensor(np.random.default_rng(1).standard_normal(4096), device="cuda:0")
xs = torch.empty(4096, dtype=torch.float64, device="cuda:0")
print("server", srv.wait(srv.submit(op, b, xs, 8, 20, 0.0, 0, 4, 7)), flush=True)
srv.close()
"""


def test_log_level_two_reports_plans_and_admissions():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, HK_LOG="2")
    print("running a logged solve in a child process", flush=True)
    r = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, env=env, capture_output=True, text=True, timeout=180)
    print(r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "status 0" in r.stdout and "server 0" in r.stdout
    assert "hk: solve: blur (single barrier) kernel" in r.stderr
    # 4096 pixels over at most one workgroup per compute unit: 64 tiles of 8 x 8
    assert "64 workgroups, tiles of 8x8 pixels" in r.stderr
    assert "hk: server: request 0 admitted on slot 0" in r.stderr
