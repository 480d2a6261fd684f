"""GPU tests of several right-hand sides solved together (hk_params.nrhs):
the right-hand sides share the basis kernel's grid barriers, and with a
Gaussian sketch the sketches of all their bases form one MFMA block
contraction.  Each right-hand side's results (x, H, pivots, residual
history, sketches, basis) equal the single-right-hand-side solve's bit for
bit, and agree with the oracle at the class bars."""
import numpy as np
import pytest

import workloads as W
from hk_gpu import compare_solve, gpu_solve, make_operator, rounded_problem, storage_np, tiny_blur

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


def _flush(msg):
    print(msg, flush=True)


def family(P, nr):
    """nr problems on P's operator (the first is P itself)."""
    return W.blur_rhs_family(P, nr)


def multi_solve(hk, ctx, probs):
    """Solve all right-hand sides of `probs` (one operator) together."""
    import torch
    P = probs[0]
    nr = len(probs)
    op = make_operator(hk, ctx, P)
    bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, basis_dtype=bdt, nrhs=nr)
    try:
        b = torch.tensor(np.stack([Q.b.astype(storage_np(P.dtype)) for Q in probs]), device="cuda:0")
        x = sv.run(b)
        status = None
        try:
            status = sv.wait()
        except hk.HKError as e:
            status = e.status
        outs = []
        xs = x.detach().cpu().numpy().astype(np.float64)
        for r in range(nr):
            sv.select(r)
            g = {"x": xs[r]}
            try:
                g["k_done"] = sv.k_done()
            except hk.HKError as e:
                g["error"] = e.status
                outs.append(g)
                continue
            g["H"], g["W"] = sv.hessenberg()
            g["t"], g["g"] = sv.pivots()
            g["res"] = sv.residuals()
            g["Z"], g["F"], g["c"] = sv.sketches()
            g["L"] = sv.basis(0).detach().cpu().numpy().astype(np.float64).T
            outs.append(g)
        return status, outs
    finally:
        sv.close()
        op.close()


KEYS = ("x", "H", "t", "res", "Z", "F", "c", "L")


def assert_same(g, s, label):
    for key in KEYS:
        a, b = np.asarray(g[key]), np.asarray(s[key])
        assert a.shape == b.shape and np.array_equal(a, b), f"{label}: {key} differs from the single solve"


@pytest.mark.parametrize("case,nr", [("ragged_f64_gauss", 2), ("ragged_f32_sparse", 3), ("ragged_f64_none", 2),
                                     ("b96_f32_gauss", 4)])
def test_multi_rhs_equals_single(hk, ctx, orc, case, nr):
    if case == "ragged_f64_gauss":
        P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=1e-2, sketch=W.SKETCH_GAUSSIAN, dtype="f64")
    elif case == "ragged_f32_sparse":
        P = tiny_blur(50, 70, 1.5, 5, W.BC_ZERO, k=25, s=60, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN, zeta=5,
                      dtype="f32")
    elif case == "ragged_f64_none":
        P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=1e-3, sketch=W.SKETCH_NONE, dtype="f64")
    else:
        P = tiny_blur(96, 96, 2.0, 7, W.BC_REFLECT, k=40, s=82, lam=1e-2, sketch=W.SKETCH_GAUSSIAN, dtype="f32")
    probs = family(P, nr)
    _flush(f"multi-rhs {case}: {nr} right-hand sides, n={P.n} k={P.k} {P.dtype}")
    status, outs = multi_solve(hk, ctx, probs)
    assert status in (0, 1), status
    for r, (Q, g) in enumerate(zip(probs, outs)):
        s1 = gpu_solve(hk, ctx, Q)
        _flush(f"  rhs {r}: k_done {g['k_done']} (alone {s1['k_done']})")
        assert g["k_done"] == s1["k_done"]
        assert_same(g, s1, f"rhs {r}")
        o = orc.solve(rounded_problem(Q), keep_basis=True)
        g.update(status=s1["status"], W=None, g=None)
        compare_solve(rounded_problem(Q), g, o)


def test_multi_rhs_deblur512(hk, ctx, orc):
    # the 512 x 512 deblurring operator with four right-hand sides, k = 100,
    # Gaussian sketch s = 400 (the multi-right-hand-side benchmark's setting)
    P = W.config("c2").replace(sketch=W.SKETCH_GAUSSIAN)
    probs = family(P, 4)
    _flush("multi-rhs 512x512: 4 right-hand sides, k=100")
    status, outs = multi_solve(hk, ctx, probs)
    assert status == 0
    for r in (0, 3):
        s1 = gpu_solve(hk, ctx, probs[r])
        assert_same(outs[r], s1, f"rhs {r}")
    o = orc.solve(rounded_problem(probs[3]), keep_basis=True)
    g = dict(outs[3], status=0, W=None, g=None)
    compare_solve(rounded_problem(probs[3]), g, o)


def test_multi_rhs_breakdown_and_error_are_per_rhs(hk, ctx):
    P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=20, s=50, lam=1e-2, sketch=W.SKETCH_GAUSSIAN, dtype="f64")
    probs = family(P, 3)
    # right-hand side 1 is zero: it breaks down at once, the others go on
    probs[1] = probs[1].replace(b=np.zeros_like(probs[1].b))
    status, outs = multi_solve(hk, ctx, probs)
    assert status == 1
    assert outs[1]["k_done"] == 0 and np.all(outs[1]["x"] == 0)
    for r in (0, 2):
        assert_same(outs[r], gpu_solve(hk, ctx, probs[r]), f"rhs {r}")
    # a NaN in right-hand side 2: the run reports HK_ENUMERIC, the others
    # are still solved
    probs[1] = family(P, 2)[1]
    b2 = probs[2].b.copy()
    b2[100] = np.nan
    probs[2] = probs[2].replace(b=b2)
    status, outs = multi_solve(hk, ctx, probs)
    assert status == hk.HK_ENUMERIC
    assert outs[2].get("error") == hk.HK_ENUMERIC
    assert_same(outs[0], gpu_solve(hk, ctx, probs[0]), "rhs 0")


def test_multi_rhs_refusals(hk, ctx):
    from hk_gpu import random_csr
    P = tiny_blur(32, 32, 1.0, 3, W.BC_ZERO, k=8, s=20)
    op = make_operator(hk, ctx, P)
    for kw, st in [(dict(nrhs=9), hk.HK_EINVAL), (dict(nrhs=2, pivot_sample=5), hk.HK_EUNSUPPORTED)]:
        with pytest.raises(hk.HKError) as e:
            hk.Solve(op, 8, 20, **kw)
        assert e.value.status == st
    op.close()
    C = random_csr(300, 200, 0.05, k=8, s=20)
    cop = make_operator(hk, ctx, C)
    with pytest.raises(hk.HKError) as e:
        hk.Solve(cop, 8, 20, nrhs=2)
    assert e.value.status == hk.HK_EUNSUPPORTED
    cop.close()
    # eight right-hand sides of k = 255 do not fit the kernel's LDS
    big = tiny_blur(128, 128, 1.0, 3, W.BC_ZERO, k=255, s=512, dtype="f32")
    bop = make_operator(hk, ctx, big)
    with pytest.raises(hk.HKError) as e:
        hk.Solve(bop, 255, 512, nrhs=8, basis_dtype=hk.HK_F32)
    assert e.value.status == hk.HK_EUNSUPPORTED
    bop.close()
