"""The entry point that allocates nothing (hk_solve_run_noalloc), called
through the C ABI: its result equals that of hk_solve_create + hk_solve_run
on the same problem, bit for bit, on two calls in a row (the second with a
smaller input, so it runs on what the first left in the static workspace),
and a problem whose workspace exceeds the static array is refused."""
import numpy as np
import pytest

import workloads as W
from hk_gpu import gpu_solve, make_operator, storage_np, tiny_blur

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


def _noalloc(hk, ctx, P):
    import torch
    op = make_operator(hk, ctx, P)
    try:
        bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
        prm = hk.make_params(P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, bdt, 0, P.pivot_sample, 0)
        b = torch.tensor(P.b.astype(storage_np(P.dtype)), device="cuda:0")
        x = torch.full((P.n,), float("nan"), dtype=b.dtype, device="cuda:0")
        info = torch.full((2,), -99, dtype=torch.int32, device="cuda:0")
        hk.hk_solve_run_noalloc(op.handle, prm, b.data_ptr(), x.data_ptr(), info.data_ptr())
        torch.cuda.synchronize()
        return x.cpu().numpy().astype(np.float64), [int(v) for v in info.cpu().numpy()]
    finally:
        op.close()


@pytest.mark.parametrize("first,second", [
    # the 512 x 512 deblurring workload, then a smaller FP64 problem with a
    # Gaussian sketch (other kernels, other layout of the same array)
    ("c2", "c1_tik"),
    # a ragged FP32 image twice smaller than the first, sparse sign both times
    ("ragged96", "ragged50"),
])
def test_noalloc_equals_allocating_path(hk, ctx, first, second):
    probs = {"c2": lambda: W.config("c2"), "c1_tik": lambda: W.config("c1_tik"),
             "ragged96": lambda: tiny_blur(96, 130, 1.5, 5, W.BC_REFLECT, k=40, s=82, lam=1e-2,
                                           sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32"),
             "ragged50": lambda: tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=1e-2,
                                           sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32")}
    for name in (first, second):
        P = probs[name]()
        print(f"no-alloc {name}: n={P.n} k={P.k} s={P.s} {P.dtype}", flush=True)
        x, info = _noalloc(hk, ctx, P)
        g = gpu_solve(hk, ctx, P, keep_basis=False)
        print(f"  info {info}, status {g['status']} k_done {g['k_done']}, "
              f"max |x - x_alloc| {np.max(np.abs(x - g['x'])):.3e}", flush=True)
        assert info == [g["status"], g["k_done"]]
        assert np.array_equal(x, g["x"]), "no-alloc and allocating results differ"


def test_noalloc_refuses_beyond_the_static_workspace(hk, ctx):
    # 1024 x 512 with k = 100: the FP32 basis alone is 212 MB
    P = tiny_blur(1024, 512, 2.0, 7, W.BC_REFLECT, k=100, s=202, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN,
                  zeta=8, dtype="f32")
    with pytest.raises(hk.HKError) as e:
        _noalloc(hk, ctx, P)
    assert e.value.status == hk.HK_ENOMEM
    assert "static workspace" in str(e.value)
