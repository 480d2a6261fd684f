"""Helpers shared by the GPU parity tests: run a solve through the C ABI and
compare it with the oracle on the same inputs (not collected by pytest)."""
from __future__ import annotations

import json
import os

import numpy as np

import workloads as W

# Bars by the workload's precision class (the storage type of its operator
# and data): relative solution error <= 1e-10 for FP64 workloads and <= 1e-4
# for FP32 workloads (FP64 arithmetic in both cases).
X_TOL = {"f64": 1e-10, "f32": 1e-4}
# A pivot mismatch is excused only at a near-tie: the oracle's normalised
# vector has |l(p_gpu)| within TAU of 1 at the GPU's pivot.
TAU = {"f64": 1e-12, "f32": 1e-4}
# H, the sketches and the residual history are intermediate results: with FP32
# storage (or an FP32-class workload) each later basis vector carries the
# rounding of the earlier ones, so they are compared column-relatively at 1e-3.
MID_TOL = {"f64": 1e-8, "f32": 1e-3}


def storage_np(dtype):
    return np.float64 if dtype == "f64" else np.float32


def rounded_problem(P):
    """The problem exactly as the GPU sees it: b (and CSR values) rounded to
    the storage type, widened back to FP64 for the oracle."""
    t = storage_np(P.dtype)
    kw = {"b": P.b.astype(t).astype(np.float64)}
    if P.kind == "csr":
        kw["val"] = P.val.astype(t)
    return P.replace(**kw)


def make_operator(hk, ctx, P):
    dt = hk.HK_F64 if P.dtype == "f64" else hk.HK_F32
    if P.kind == "blur":
        if P.psf is not None:
            return hk.Operator.blur_psf(ctx, P.ny, P.nx, P.psf, P.radius, P.bc, dt)
        return hk.Operator.blur(ctx, P.ny, P.nx, P.taps_y, P.taps_x, P.radius, P.bc, dt)
    return hk.Operator.csr(ctx, P.m, P.n, P.rowptr, P.col, P.val.astype(storage_np(P.dtype)), dt)


def gpu_solve(hk, ctx, P, method=0, keep_basis=True, runs=1, max_workgroups=0):
    import torch
    op = make_operator(hk, ctx, P)
    bdt = hk.HK_F64 if P.basis_dtype == "f64" else hk.HK_F32
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, method, basis_dtype=bdt,
                  pivot_sample=P.pivot_sample, max_workgroups=max_workgroups)
    try:
        b = torch.tensor(P.b.astype(storage_np(P.dtype)), device=f"cuda:{ctx.device}")
        xs = []
        for _ in range(runs):
            x = sv.run(b)
            st = sv.wait()
            xs.append(x.detach().cpu().numpy().astype(np.float64))
        out = {"x": xs[-1], "xs": xs, "status": st, "k_done": sv.k_done()}
        out["H"], out["W"] = sv.hessenberg()
        out["t"], out["g"] = sv.pivots()
        out["res"] = sv.residuals()
        out["Z"], out["F"], out["c"] = sv.sketches()
        if keep_basis:
            out["L"] = sv.basis(0).detach().cpu().numpy().astype(np.float64).T
            if sv.rect:
                out["D"] = sv.basis(1).detach().cpu().numpy().astype(np.float64).T
        out["timing"] = sv.timing()
        out["grid"] = sv.grid()
    finally:
        sv.close()
        op.close()
    return out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def first_mismatch(p_gpu, p_or):
    n = min(len(p_gpu), len(p_or))
    for i in range(n):
        if p_gpu[i] != p_or[i]:
            return i
    return None if len(p_gpu) == len(p_or) else n


def check_pivots(gpu_piv, or_piv, or_basis, dtype):
    """Pivots must agree exactly up to the first excused near-tie.  Returns the
    number of leading pivots that agree (compared part of H/W)."""
    gpu_piv = [int(v) for v in gpu_piv if v >= 0]
    or_piv = [int(v) for v in or_piv]
    i = first_mismatch(gpu_piv, or_piv)
    if i is None:
        return len(or_piv)
    assert i < len(gpu_piv) and i < len(or_piv), f"pivot count differs: {len(gpu_piv)} vs {len(or_piv)}"
    col = or_basis[:, i]
    near = 1.0 - abs(col[gpu_piv[i]])
    assert near <= TAU[dtype], (f"pivot {i}: gpu {gpu_piv[i]} vs oracle {or_piv[i]} is not a near-tie "
                                f"(1 - |l(p_gpu)| = {near:.3e})")
    return i


def col_rel(A, B):
    """Largest column-wise relative difference."""
    nb = np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    return float(np.max(np.linalg.norm(A - B, axis=0) / nb)) if A.size else 0.0


def sensitivity_bars(name):
    """Bars for a workload whose FP64 result is itself rounding-sensitive,
    from its fixture (tests/golden/<name>_sensitivity.json, written by
    tests/golden/make_sensitivity.py from the oracle alone): one-ulp changes of
    b move the oracle's own bases by up to `drift` column-relatively before the
    pivots split, so a pivot tie closer than that and an intermediate
    difference of that size are not decided by the arithmetic.  Twice the
    largest drift seen is allowed."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_sensitivity.json")
    with open(path) as f:
        runs = json.load(f)["runs"]
    basis = max(max(r["D_drift"], r["L_drift"]) for r in runs)
    mid = max(max(r["H_drift"], r["Z_drift"]) for r in runs)
    return {"tau": 2.0 * basis, "mid": 2.0 * mid}


def col_maxrel(A, B):
    """Largest column-wise elementwise difference, relative to the column's
    largest magnitude: max_j max_r |A(r, j) - B(r, j)| / max_r |B(r, j)|."""
    if not A.size:
        return 0.0
    nb = np.maximum(np.max(np.abs(B), axis=0), 1e-300)
    return float(np.max(np.max(np.abs(A - B), axis=0) / nb))


def basis_agree(g_piv, o_piv):
    """Basis columns whose pivot agrees: column j is v_j normalised at its
    pivot, so the leading columns up to the first mismatch are comparable."""
    i = first_mismatch([int(v) for v in g_piv if v >= 0], [int(v) for v in o_piv])
    return len(o_piv) if i is None else i


# measured deviations of the last compare_solve (for reports)
LAST = {}


def compare_solve(P, g, o, bars=None):
    """Element-by-element comparison of a GPU solve with the oracle.  All
    diagnostics are printed before any assertion.  `bars` may widen the
    near-tie and intermediate bars of a rounding-sensitive workload (see
    sensitivity_bars); the bar on x is always the class bar, both as a
    relative 2-norm and elementwise relative to max |x|."""
    cls = P.dtype                      # precision class of the workload
    tau = max(TAU[cls], (bars or {}).get("tau", 0.0))
    mid = max(MID_TOL[cls], (bars or {}).get("mid", 0.0))
    kd = o["k_done"]
    err = rel(g["x"], o["x"])
    xmax = float(np.max(np.abs(o["x"]))) if o["x"].size else 0.0
    emax = float(np.max(np.abs(g["x"] - o["x"]))) / (xmax if xmax > 0 else 1.0)
    nL = o["Lmat"] if o["method"] == 0 else o["Dmat"]
    gp = [int(v) for v in g["t"] if v >= 0]
    i = first_mismatch(gp, [int(v) for v in o["t"]])
    near = None
    if i is not None and i < len(gp) and i < nL.shape[1]:
        near = 1.0 - abs(nL[gp[i], i])
    agree = len(o["t"]) if i is None else i
    hk_ = min(agree - 1, kd)
    eH = col_rel(g["H"][: hk_ + 1, :hk_], o["H"][: hk_ + 1, :hk_]) if hk_ > 0 else 0.0
    m = min(agree, kd)
    ez = col_rel(g["Z"][:, :m], o["Z"][:, :m])
    ef = col_rel(g["F"][:, :m], o["F"][:, :m]) if P.lam > 0 else 0.0
    er = float(np.max(np.abs(g["res"][:m] - o["res"][:m]) / np.maximum(o["res"][:m], 1e-300))) if m else 0.0
    ec = rel(g["c"], o["c"])
    # bases, column by column, elementwise, on the agreed pivot prefix: L for
    # sCMRH, D (data space) and L for sLSLU
    eb = 0.0
    nb_cols = 0
    if "L" in g:
        if o["method"] == 0:
            nc = min(agree, o["Lmat"].shape[1], g["L"].shape[1])
            eb = col_maxrel(g["L"][:, :nc], o["Lmat"][:, :nc])
            nb_cols = nc
        else:
            nd = min(agree, o["Dmat"].shape[1], g["D"].shape[1])
            ag = basis_agree(g["g"], o["g"])
            nl = min(ag, len(o["g"]), o["Lmat"].shape[1], g["L"].shape[1])
            eb = max(col_maxrel(g["D"][:, :nd], o["Dmat"][:, :nd]),
                     col_maxrel(g["L"][:, :nl], o["Lmat"][:, :nl]))
            nb_cols = nd + nl
    LAST.clear()
    LAST.update(x=err, xmax=emax, H=eH, Z=ez, F=ef, res=er, c=ec, basis=eb, basis_cols=nb_cols,
                agree=agree, k_done=kd)
    log = os.environ.get("HK_PARITY_LOG")
    if log:   # measured deviations, one JSON line per comparison
        with open(log, "a") as f:
            f.write(json.dumps({"name": P.name, "dtype": P.dtype, "basis_dtype": P.basis_dtype, "m": P.m, "n": P.n,
                                "k": P.k, "s": P.s, "lam": P.lam, "sketch": P.sketch, **LAST}) + "\n")
    print(f"  k_done {g['k_done']}/{kd} status {g['status']}/{o['status']} x_err {err:.3e} x_max {emax:.3e} "
          f"first_pivot_mismatch {i} near {near} H {eH:.2e} Z {ez:.2e} F {ef:.2e} res {er:.2e} "
          f"c {ec:.2e} basis {eb:.2e} ({nb_cols} cols)", flush=True)
    assert g["k_done"] == kd, (g["k_done"], kd)
    assert (g["status"] == 1) == (o["status"] == 1)
    assert err <= X_TOL[cls], f"relative solution error {err:.3e} > {X_TOL[cls]:.0e}"
    assert emax <= X_TOL[cls], f"elementwise solution error {emax:.3e} > {X_TOL[cls]:.0e} max|x|"
    if i is not None:
        assert near is not None and near <= tau, f"pivot {i} mismatch is not a near-tie ({near})"
    if o["method"] == 1:
        gg = [int(v) for v in g["g"] if v >= 0]
        j = first_mismatch(gg, [int(v) for v in o["g"]])
        if j is not None:
            assert j < len(gg) and j < o["Lmat"].shape[1]
            nearg = 1.0 - abs(o["Lmat"][gg[j], j])
            assert nearg <= tau, f"pivot g{j} mismatch is not a near-tie ({nearg})"
    assert eH <= mid, f"H differs: {eH:.3e}"
    assert ez <= mid, f"Z differs: {ez:.3e}"
    assert ef <= mid, f"F differs: {ef:.3e}"
    assert er <= mid, f"residual history differs: {er:.3e}"
    assert eb <= mid, f"basis differs: {eb:.3e}"
    # S2 b depends on b only; FP32-class workloads evaluate the Gaussian
    # entries in FP32 (about 1e-7 relative), FP64 workloads in FP64
    assert ec <= (1e-13 if P.dtype == "f64" else 1e-6), f"S2 b differs: {ec:.3e}"
    return err


def tiny_blur(ny, nx, sigma, r, bc, k, s, lam=0.0, sketch=W.SKETCH_GAUSSIAN, zeta=4, dtype="f64",
              phantom="blobs"):
    return W.blur_problem(f"b{ny}x{nx}", ny, nx, sigma, r, bc, phantom, 0.01, k=k, s=s, lam=lam,
                          sketch=sketch, zeta=zeta, dtype=dtype, cfg_id=7)


def random_csr(m, n, density, k, s, lam=0.0, sketch=W.SKETCH_GAUSSIAN, zeta=4, dtype="f64", seed=5):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=seed, format="csr",
                  data_rvs=lambda size: rng.uniform(0.1, 1.0, size))
    A.sort_indices()
    b = A @ rng.uniform(0, 1, n) + 0.01 * rng.standard_normal(m)
    t = storage_np(dtype)
    return W.Problem(name=f"csr{m}x{n}", kind="csr", m=m, n=n, b=b, x_true=np.zeros(n), k=k, s=s,
                     lam=lam, sketch=sketch, zeta=zeta, seed=W.SKETCH_SEED_BASE + 11, dtype=dtype,
                     rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                     val=A.data.astype(t))
