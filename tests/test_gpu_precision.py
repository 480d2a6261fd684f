"""GPU tests of the reduced-precision storage tier: Krylov bases stored in
bfloat16 or IEEE binary16 under an FP32 blur operator, FP64 arithmetic.

A 16-bit basis changes the subspace the method builds, so its solution is not
held to a fixed bar against the FP64 oracle.  What the arithmetic fixes is
checked exactly, on the GPU's own stored basis:
  1. structure of the Hessenberg process with partial pivoting (Sec. 3.1):
     each stored column is exactly zero at the earlier pivots and takes its
     largest magnitude at its own pivot;
  2. the Hessenberg relation A L_k = L_{k+1} H_k (eq. (Hessenberg_s)) holds
     up to the one rounding of each new column to the storage type,
     elementwise: |A l_j - sum_i H(i, j) l_i| <= 2 u |H(j+1, j) l_{j+1}| plus
     FP32 rounding of the pivot block, u the unit roundoff of the type;
  3. the sketches Z = S2 A L_k, F = S1 L_k, c = S2 b (Sec. 2), the residual
     history and x = L_k y of the sketched Tikhonov problem (Sec. 3.3) agree
     with the oracle's computation from the same stored basis at FP64-level
     bars.
The error against the FP64 oracle's own solution and against x_true is
printed for each type and bounded loosely: the reconstruction error may not
exceed the FP64 oracle's by more than MARGIN.
"""
import numpy as np
import pytest

import workloads as W
from hk_gpu import make_operator, rel, rounded_problem

pytestmark = pytest.mark.gpu

# unit roundoff of each storage type
UNIT = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
# Largest increase of the reconstruction error ||x - x_true|| / ||x_true||
# over the FP64 oracle's that is accepted (a statement of measured accuracy,
# not a derived bound: the 16-bit subspace differs from the FP64 one).
MARGIN = {"f32": 1e-3, "f16": 0.03, "bf16": 0.1}


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_02721_amd as hk
    hk.lib()   # raises if the library is not built: no fallback
    return hk


@pytest.fixture(scope="module")
def ctx(hk):
    return hk.Context(0)


def _flush(msg):
    print(msg, flush=True)


def _bdt(hk, name):
    return {"f32": hk.HK_F32, "bf16": hk.HK_BF16, "f16": hk.HK_F16}[name]


def run_stored(hk, ctx, P, basis):
    """Solve on the GPU with `basis` storage; return results and the stored
    (unnormalised) basis as FP64."""
    import torch
    op = make_operator(hk, ctx, P)
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, basis_dtype=_bdt(hk, basis))
    b = torch.tensor(P.b.astype(np.float32), device=f"cuda:{ctx.device}")
    x = sv.run(b)
    st = sv.wait()
    out = {"x": x.cpu().numpy().astype(np.float64), "status": st, "k_done": sv.k_done()}
    out["H"], _ = sv.hessenberg()
    out["t"], _ = sv.pivots()
    out["res"] = sv.residuals()
    out["Z"], out["F"], out["c"] = sv.sketches()
    out["V"] = sv.basis(2).float().cpu().numpy().astype(np.float64).T     # n x (k+1)
    out["iter_ms"], out["total_ms"] = sv.timing()
    sv.close()
    op.close()
    return out


def blur_fp64(P, X):
    """A X column by column in FP64 (SciPy's separable correlation)."""
    img = X.T.reshape(-1, P.ny, P.nx)
    return np.stack([W.blur_apply_scipy(im, P.taps_y, P.taps_x, P.bc).ravel() for im in img], axis=1)


def check_stored_basis(orc, P, g, basis):
    kd = g["k_done"]
    t = [int(v) for v in g["t"][: kd + 1]]
    V = g["V"][:, : kd + 1]
    u = UNIT[basis]
    # 1. structure: exact zeros at earlier pivots, the pivot entry is the max
    for j in range(kd + 1):
        assert V[t[j], j] != 0.0, f"column {j}: zero pivot entry"
        assert np.all(V[t[:j], j] == 0.0), f"column {j}: nonzero at an earlier pivot row"
        assert np.max(np.abs(V[:, j])) == abs(V[t[j], j]), f"column {j}: pivot entry is not the largest"
    assert len(set(t)) == len(t), "pivots repeat"
    Lt = V / V[t, np.arange(kd + 1)]                     # l_j = v_j / v_j(t_j)
    # 2. Hessenberg relation, elementwise, one rounding per column
    AL = blur_fp64(P, Lt[:, :kd])
    H = g["H"][: kd + 1, :kd]
    R = AL - Lt @ H
    worst = 0.0
    for j in range(kd):
        hsum = np.sum(np.abs(H[: j + 1, j]))
        bound = 2.0 * u * np.abs(H[j + 1, j] * Lt[:, j + 1]) + 1e-6 * (np.max(np.abs(AL[:, j])) + hsum)
        worst = max(worst, float(np.max(np.abs(R[:, j]) / bound)))
    # 3. sketches, residual history and x from the stored basis
    S2 = orc.sketch_dense(P.sketch, P.s, P.n, P.zeta, P.seed, 2)
    Z = S2 @ AL
    c = S2 @ P.b.astype(np.float32).astype(np.float64)
    del S2
    if P.lam > 0:
        S1 = orc.sketch_dense(P.sketch, P.s, P.n, P.zeta, P.seed, 1)
        F = S1 @ Lt[:, :kd]
        del S1
    else:
        F = np.zeros_like(Z)
    y, res = orc.small_ls(Z, F, P.lam, c)
    x = Lt[:, :kd] @ y
    ez = float(np.max(np.linalg.norm(g["Z"][:, :kd] - Z, axis=0) / np.linalg.norm(Z, axis=0)))
    ef = float(np.max(np.linalg.norm(g["F"][:, :kd] - F, axis=0) / np.linalg.norm(F, axis=0))) if P.lam > 0 else 0.0
    ec = rel(g["c"], c)
    er = float(np.max(np.abs(g["res"][:kd] - res) / res))
    ex = rel(g["x"], x)
    _flush(f"  {basis}: k_done {kd} relation/bound {worst:.3f} Z {ez:.2e} F {ef:.2e} c {ec:.2e} "
           f"res {er:.2e} x(stored basis) {ex:.2e}")
    assert worst <= 1.0, f"Hessenberg relation exceeds the rounding bound ({worst:.3f})"
    # Gaussian entries are evaluated in FP32 for FP32 data (about 1e-7)
    zt = 1e-10 if P.sketch == W.SKETCH_SPARSE_SIGN else 1e-6
    assert ez <= zt and ef <= zt and ec <= zt, (ez, ef, ec)
    assert er <= max(zt, 1e-8), er
    assert ex <= 1e-5, ex


def report_vs_fp64(P, g, o64, basis):
    e64 = rel(g["x"], o64["x"])
    et = rel(g["x"], P.x_true)
    e0 = rel(o64["x"], P.x_true)
    kd = min(g["k_done"], o64["k_done"])
    rr = np.abs(g["res"][:kd] - o64["res"][:kd]) / o64["res"][:kd]
    _flush(f"  {basis}: vs FP64 oracle x {e64:.3e}  error vs x_true {et:.4f} (FP64 oracle {e0:.4f})  "
           f"residual history max rel diff {np.max(rr):.2e} (last {rr[-1]:.2e})")
    assert et <= e0 + MARGIN[basis], f"reconstruction error {et:.4f} vs FP64 {e0:.4f}"
    return e64


def small_c4(sketch):
    if sketch == "sparse":
        # the deblurring recipe at 128 x 128 (sigma 4, 31 x 31, reflective, 2% noise)
        return W.blur_problem("c4s", 128, 128, 4.0, 15, W.BC_REFLECT, "piecewise", 0.02, k=60, s=240,
                              lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN, zeta=8, dtype="f32", cfg_id=4)
    # ragged tiles, zero boundary, Gaussian sketch
    return W.blur_problem("c4g", 100, 90, 2.0, 7, W.BC_ZERO, "blobs", 0.01, k=30, s=62, lam=1e-2,
                          sketch=W.SKETCH_GAUSSIAN, dtype="f32", cfg_id=4)


@pytest.mark.parametrize("sketch", ["sparse", "gauss"])
@pytest.mark.parametrize("basis", ["f32", "bf16", "f16"])
def test_precision_tier_small(hk, ctx, orc, basis, sketch):
    P = small_c4(sketch)
    _flush(f"precision tier {P.name} {P.ny}x{P.nx} k={P.k} basis {basis}")
    g = run_stored(hk, ctx, P, basis)
    assert g["status"] == 0 and g["k_done"] == P.k
    check_stored_basis(orc, P, g, basis)
    o64 = orc.solve(rounded_problem(P))
    report_vs_fp64(P, g, o64, basis)


@pytest.fixture(scope="module")
def c2_fp64(orc):
    P = W.config("c2")
    _flush("FP64 oracle on the 512x512 deblurring workload")
    return P, orc.solve(rounded_problem(P), keep_basis=True)


@pytest.mark.parametrize("basis", ["f32", "bf16", "f16"])
def test_precision_tier_deblur512(hk, ctx, orc, c2_fp64, basis):
    P, o64 = c2_fp64
    _flush(f"precision tier deblur 512x512 k={P.k} basis {basis}")
    g = run_stored(hk, ctx, P, basis)
    assert g["status"] == 0 and g["k_done"] == P.k
    check_stored_basis(orc, P, g, basis)
    report_vs_fp64(P, g, o64, basis)
    _flush(f"  {basis}: basis kernel {g['iter_ms']:.3f} ms, solve {g['total_ms']:.3f} ms")


def test_precision_tier_per_iteration_deblur512(hk, ctx, orc, c2_fp64):
    """The error of each storage type against the FP64 oracle after every
    tenth step: relative error of x_k' against the oracle's x_k' (both the
    minimiser over the first k' basis vectors), against x_true, the sketched
    objective res[k'-1] and the true relative residual ||b - A x_k'|| / ||b||
    (FP64 on the host).  Written as JSON lines to $HK_PRECISION_REPORT when
    set.  Bounded loosely, as the final solution: the reconstruction error of
    every x_k' may exceed the FP64 oracle's by at most MARGIN."""
    import json
    import os
    import torch
    P, o64 = c2_fp64
    kps = list(range(10, P.k + 1, 10))
    b64 = P.b.astype(np.float32).astype(np.float64)
    nb = np.linalg.norm(b64)

    def true_res(x):
        return np.linalg.norm(b64 - W.blur_apply_scipy(x.reshape(P.ny, P.nx), P.taps_y, P.taps_x, P.bc).ravel()) / nb

    x64 = {kp: orc.prefix_solution(o64, kp, P.lam) for kp in kps}
    rows = []
    for basis in ("f32", "bf16", "f16"):
        op = make_operator(hk, ctx, P)
        sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, 0, basis_dtype=_bdt(hk, basis))
        try:
            b = torch.tensor(P.b.astype(np.float32), device=f"cuda:{ctx.device}")
            sv.run(b)
            assert sv.wait() == 0 and sv.k_done() == P.k
            res = sv.residuals()
            for kp in kps:
                x = sv.prefix_solution(kp).cpu().numpy().astype(np.float64)
                row = {"basis": basis, "k": kp, "err_vs_fp64": rel(x, x64[kp]),
                       "err_vs_true": rel(x, P.x_true), "fp64_err_vs_true": rel(x64[kp], P.x_true),
                       "sketched_res": float(res[kp - 1]), "fp64_sketched_res": float(o64["res"][kp - 1]),
                       "true_res": true_res(x), "fp64_true_res": true_res(x64[kp])}
                rows.append(row)
                _flush(f"  {basis} k'={kp:3d}: vs FP64 {row['err_vs_fp64']:.3e}  vs x_true {row['err_vs_true']:.4f} "
                       f"(FP64 {row['fp64_err_vs_true']:.4f})  sketched res {row['sketched_res']:.4e} "
                       f"(FP64 {row['fp64_sketched_res']:.4e})  true res {row['true_res']:.4e} "
                       f"(FP64 {row['fp64_true_res']:.4e})")
        finally:
            sv.close()
            op.close()
    path = os.environ.get("HK_PRECISION_REPORT")
    if path:
        with open(path, "w") as f:
            for row in rows:
                f.write(json.dumps(row) + "\n")
    for row in rows:
        assert row["err_vs_true"] <= row["fp64_err_vs_true"] + MARGIN[row["basis"]], row
        if row["basis"] == "f32":
            assert row["err_vs_fp64"] <= 1e-4, row


def test_precision_tier_rejects(hk, ctx):
    """16-bit bases are refused where they are not implemented."""
    from hk_gpu import random_csr
    P = random_csr(300, 300, 0.05, k=5, s=12, dtype="f32")
    op = make_operator(hk, ctx, P)
    with pytest.raises(Exception):
        hk.Solve(op, 5, 12, 0.0, W.SKETCH_GAUSSIAN, 2, 1, 0, basis_dtype=hk.HK_BF16)
    op.close()
    P = small_c4("gauss").replace(dtype="f64")
    op = make_operator(hk, ctx, P)
    with pytest.raises(Exception):
        hk.Solve(op, 5, 12, 0.0, W.SKETCH_GAUSSIAN, 2, 1, 0, basis_dtype=hk.HK_F16)
    op.close()
