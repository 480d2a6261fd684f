"""A solve on a workspace the caller owns (hk_solve_create_with_workspace):
the same results as on the library's own workspace, bit for bit, also when
the caller's memory starts out as garbage and when one workspace serves two
problems one after the other; misaligned and too-small workspaces are
refused before any device work."""
import numpy as np
import pytest

import workloads as W
from hk_gpu import make_operator, storage_np, tiny_blur

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_02721_amd as hk
    hk.lib()
    return hk


@pytest.fixture(scope="module")
def ctx(hk):
    return hk.Context(0)


def _solve(hk, ctx, P, workspace=None):
    import torch
    op = make_operator(hk, ctx, P)
    bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=bdt, workspace=workspace)
    try:
        b = torch.tensor(P.b.astype(storage_np(P.dtype)), device="cuda:0")
        x = sv.run(b)
        st = sv.wait()
        return {"st": st, "x": x.cpu().numpy().copy(), "H": sv.hessenberg()[0].copy(),
                "piv": np.asarray(sv.pivots()[0]).copy(), "res": np.asarray(sv.residuals()).copy()}
    finally:
        sv.close()
        op.close()


def _problems():
    return [tiny_blur(96, 130, 1.5, 5, W.BC_REFLECT, k=40, s=82, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN,
                      zeta=5, dtype="f32"),
            W.config("c1_tik")]


def test_caller_workspace_equals_library_workspace(hk, ctx):
    import torch
    probs = _problems()
    need = []
    for P in probs:
        op = make_operator(hk, ctx, P)
        bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
        prm = hk.make_params(P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, bdt, 0, P.pivot_sample, 0)
        need.append(hk.hk_solve_workspace_bytes(op.handle, prm))
        op.close()
    # one workspace for both problems, run one after the other, starting as garbage
    ws = torch.full((max(need),), 0xA5, dtype=torch.uint8, device="cuda:0")
    for P in probs:
        print(f"problem {P.name} n={P.n} k={P.k} workspace {max(need)} bytes", flush=True)
        ref = _solve(hk, ctx, P)
        got = _solve(hk, ctx, P, workspace=ws)
        assert got["st"] == ref["st"] == 0
        np.testing.assert_array_equal(got["x"], ref["x"])
        np.testing.assert_array_equal(got["H"], ref["H"])
        np.testing.assert_array_equal(got["piv"], ref["piv"])
        np.testing.assert_array_equal(got["res"], ref["res"])


def test_caller_workspace_refusals(hk, ctx):
    import torch
    P = _problems()[0]
    op = make_operator(hk, ctx, P)
    try:
        prm = hk.make_params(P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, hk.HK_F32, 0, 0, 0)
        need = hk.hk_solve_workspace_bytes(op.handle, prm)
        ws = torch.zeros(need + 512, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(hk.HKError) as e:
            hk.hk_solve_create_with_workspace(op.handle, prm, ws.data_ptr() + 8, need)
        assert e.value.args[0].startswith(f"hk status {hk.HK_EINVAL}")
        with pytest.raises(hk.HKError) as e:
            hk.hk_solve_create_with_workspace(op.handle, prm, ws.data_ptr(), need - 256)
        assert e.value.args[0].startswith(f"hk status {hk.HK_ENOMEM}")
    finally:
        op.close()
