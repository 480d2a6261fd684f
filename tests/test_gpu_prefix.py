"""Prefix solutions (hk_solve_get_prefix_solution): x after the first kp
basis vectors, from the run's own small-problem factors.
 - kp = k_done gives the run's x bit for bit;
 - every prefix agrees with the oracle's prefix solution (the k-step oracle
   solve's small problem restricted to kp columns, pinned in
   test_oracle_prefix.py) at the workload's class bar, elementwise;
 - with several right-hand sides, the prefix of the selected one equals the
   prefix of its own single solve bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from hk_gpu import X_TOL, make_operator, random_csr, rounded_problem, storage_np, tiny_blur

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


def _prefixes(hk, ctx, P, kps, nrhs=1, probs=None, sel=0):
    import torch
    op = make_operator(hk, ctx, P)
    bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=bdt, nrhs=nrhs)
    try:
        bs = [Q.b for Q in (probs or [P])]
        b = torch.tensor(np.stack(bs) if nrhs > 1 else bs[0], dtype=getattr(torch, "float64" if P.dtype == "f64"
                                                                            else "float32"), device="cuda:0")
        x = sv.run(b)
        st = sv.wait()
        sv.select(sel)
        kd = sv.k_done()
        xr = (x[sel] if nrhs > 1 else x).cpu().numpy().astype(np.float64)
        out = {"st": st, "k_done": kd, "x": xr}
        for kp in kps(kd):
            out[kp] = sv.prefix_solution(kp).cpu().numpy().astype(np.float64)
        return out
    finally:
        sv.close()
        op.close()


CASES = {
    "c1_tik_f64": lambda: W.config("c1_tik"),
    "ragged_f32_sparse": lambda: tiny_blur(96, 130, 1.5, 5, W.BC_REFLECT, k=40, s=82, lam=1e-2,
                                           sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32"),
    "csr_rect_f64": lambda: random_csr(300, 180, 0.05, k=30, s=70, lam=0.05),
}


@pytest.mark.parametrize("name", list(CASES))
def test_prefix_solutions_match_oracle(hk, ctx, orc, name):
    P = CASES[name]()
    print(f"case {name}: m={P.m} n={P.n} k={P.k} s={P.s}", flush=True)
    kps = lambda kd: sorted({1, 2, kd // 3, kd // 2, kd - 1, kd})
    g = _prefixes(hk, ctx, P, kps)
    assert g["st"] == 0
    kd = g["k_done"]
    np.testing.assert_array_equal(g[kd], g["x"])
    o = orc.solve(rounded_problem(P), keep_basis=True)
    assert o["k_done"] == kd
    bar = X_TOL[P.dtype]
    for kp in kps(kd):
        xo = orc.prefix_solution(o, kp, P.lam)
        e = np.max(np.abs(g[kp] - xo)) / np.max(np.abs(xo))
        print(f"  kp {kp}: elementwise error {e:.3e}", flush=True)
        assert e <= bar, (kp, e)


def test_prefix_of_selected_rhs_equals_single(hk, ctx):
    P = tiny_blur(96, 130, 1.5, 5, W.BC_REFLECT, k=40, s=82, lam=1e-2, sketch=W.SKETCH_GAUSSIAN, zeta=5,
                  dtype="f32")
    probs = W.blur_rhs_family(P, 3)
    kps = lambda kd: (1, 17, kd)
    for r in (1, 2):
        multi = _prefixes(hk, ctx, P, kps, nrhs=3, probs=probs, sel=r)
        single = _prefixes(hk, ctx, probs[r], kps)
        assert multi["k_done"] == single["k_done"]
        for kp in kps(single["k_done"]):
            np.testing.assert_array_equal(multi[kp], single[kp])


def _host_apply(P, x):
    """A x in FP64 on the host (scipy), on the operator as the GPU sees it."""
    import scipy.sparse as sp
    if P.kind == "blur":
        return W.blur_apply_scipy(x.reshape(P.ny, P.nx), P.taps_y, P.taps_x, P.bc, psf=P.psf).ravel()
    val = P.val.astype(storage_np(P.dtype)).astype(np.float64)
    return sp.csr_matrix((val, P.col, P.rowptr), shape=(P.m, P.n)) @ x


@pytest.mark.parametrize("name", list(CASES))
def test_true_residuals(hk, ctx, orc, name):
    """||b - A x_kp|| from the library against the same norm of its own prefix
    solutions evaluated on the host in FP64, and against the oracle's prefix
    solutions (the definition: Sec. 2, the residual the sketch stands in for)."""
    import torch
    P = CASES[name]()
    print(f"case {name}: m={P.m} n={P.n} k={P.k}", flush=True)
    op = make_operator(hk, ctx, P)
    bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=bdt)
    try:
        b = torch.tensor(P.b.astype(storage_np(P.dtype)), device="cuda:0")
        sv.run(b)
        assert sv.wait() == 0
        kd = sv.k_done()
        tr = sv.true_residuals()
        assert np.all(tr[kd:] == 0.0) and np.all(tr[:kd] > 0.0)
        bh = P.b.astype(storage_np(P.dtype)).astype(np.float64)
        own = np.array([np.linalg.norm(bh - _host_apply(P, sv.prefix_solution(kp).cpu().numpy().astype(np.float64)))
                        for kp in range(1, kd + 1)])
    finally:
        sv.close()
        op.close()
    e_own = np.max(np.abs(tr[:kd] - own) / own)
    o = orc.solve(rounded_problem(P), keep_basis=True)
    ref = np.array([np.linalg.norm(bh - _host_apply(P, orc.prefix_solution(o, kp, P.lam))) for kp in range(1, kd + 1)])
    e_or = np.max(np.abs(tr[:kd] - ref) / ref)
    print(f"  true residuals: vs host norm of own prefixes {e_own:.2e}, vs oracle {e_or:.2e} "
          f"(first {tr[0]:.4e}, last {tr[kd - 1]:.4e})", flush=True)
    # FP64 operators: products and norms in FP64; FP32 operators: A x is
    # rounded to FP32 by the product kernel
    assert e_own <= (1e-12 if P.dtype == "f64" else 1e-5), e_own
    assert e_or <= (1e-8 if P.dtype == "f64" else 1e-3), e_or
