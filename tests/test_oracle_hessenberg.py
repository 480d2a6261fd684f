"""Pins for the oracle's basis construction and solve.

 - the Hessenberg relations, eq. (Hessenberg_s) and eq. (Hessenberg_r);
 - unit pivot entries and exact zeros at earlier pivot rows (unit lower
   triangular after row permutation, Sec. 3.1);
 - the LU-with-partial-pivoting connection (Sec. 1): L_k is the L factor of
   LU with partial pivoting of the Krylov matrix, checked with SciPy's LU;
 - with S = I, sCMRH is the minimum-residual (GMRES) iterate over K_k(A, b)
   (eq. (original_LS_proj)) and sLSLU with Tikhonov lambda is LSQR with
   damping lambda, checked with NumPy least squares and SciPy's LSQR;
 - k = n reaches the exact solution of a nonsingular square system;
 - breakdown on an invariant subspace;
 - the sketch-and-solve laws of Sec. 3.2: the lower residual bound of
   eq. (eqthm2) for every seed, the expected residual factor 1 + k/(l-k-1),
   and unbiasedness of the Gaussian sketch-and-solve solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.sparse.linalg import lsqr

import workloads as W


def dense_of(orc, P):
    op = orc.Operator(P)
    return np.column_stack([op.apply(e) for e in np.eye(P.n)])


def small_blur(ny=12, nx=11, sigma=1.2, r=3, bc=W.BC_ZERO, k=8, s=None, lam=0.0,
               sketch=W.SKETCH_GAUSSIAN, seed_phantom=5):
    P = W.blur_problem("t", ny, nx, sigma, r, bc, "random", 0.01, k=k, s=s or 2 * (k + 1),
                       lam=lam, sketch=sketch, zeta=4, dtype="f64", phantom_seed=seed_phantom)
    return P


def rect_problem(m=40, n=25, k=6, s=None, lam=0.0, sketch=W.SKETCH_GAUSSIAN, seed=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * (rng.uniform(size=(m, n)) < 0.6)
    b = rng.standard_normal(m)
    return W.dense_problem("r", A, b, k=k, s=s or 2 * (k + 1), lam=lam, sketch=sketch, zeta=3), A


# ------------------------------------------------------------------ structure
@pytest.mark.parametrize("bc", [W.BC_ZERO, W.BC_REFLECT])
def test_scmrh_hessenberg_relation_and_pivot_structure(orc, bc):
    P = small_blur(bc=bc, k=10)
    A = dense_of(orc, P)
    out = orc.solve(P, keep_basis=True)
    k = out["k_done"]
    assert k == 10 and out["status"] == 0
    L = out["Lmat"][:, :k + 1]
    H = out["H"]
    # A L_k = L_{k+1} H_{k+1,k}
    lhs, rhs = A @ L[:, :k], L @ H
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(A) * np.linalg.norm(L)
    # H is upper Hessenberg
    assert np.all(np.tril(H, -2) == 0)
    t = out["t"]
    assert len(set(t.tolist())) == k + 1
    for i in range(k + 1):
        assert L[t[i], i] == 1.0                 # unit pivot entry, exactly
        assert np.all(L[t[:i], i] == 0.0)        # zeros at earlier pivot rows, exactly
    assert np.max(np.abs(L)) <= 1.0              # partial pivoting bounds the entries


def test_slslu_generalized_hessenberg_relations(orc):
    P, A = rect_problem(k=7)
    out = orc.solve(P, keep_basis=True)
    k = out["k_done"]
    assert k == 7 and out["method"] == 1
    L, D = out["Lmat"][:, :k], out["Dmat"][:, :k + 1]
    H, Wm = out["H"], out["W"]
    nA = np.linalg.norm(A)
    # A L_k = D_{k+1} H_{k+1,k}   and   A^T D_k = L_k W_k
    assert np.linalg.norm(A @ L - D @ H) <= 1e-13 * nA * np.linalg.norm(L)
    assert np.linalg.norm(A.T @ D[:, :k] - L @ Wm) <= 1e-13 * nA * np.linalg.norm(D)
    assert np.all(np.tril(H, -2) == 0)
    assert np.all(np.tril(Wm, -1) == 0)          # W upper triangular
    t, g = out["t"], out["g"]
    for i in range(k + 1):
        assert D[t[i], i] == 1.0 and np.all(D[t[:i], i] == 0.0)
    for i in range(k):
        assert L[g[i], i] == 1.0 and np.all(L[g[:i], i] == 0.0)
    assert np.max(np.abs(L)) <= 1.0 and np.max(np.abs(D)) <= 1.0


# ------------------------------------------------------------------ LUPP
def _lupp_L(K):
    Pm, Lf, U = sla.lu(K)
    return Pm @ Lf            # L factor in original row order


def test_scmrh_basis_is_lupp_of_krylov_matrix(orc):
    P = small_blur(k=5, ny=9, nx=9, r=2, sigma=0.9)
    A = dense_of(orc, P)
    out = orc.solve(P, keep_basis=True)
    k = 5
    K = [P.b / np.linalg.norm(P.b)]
    for _ in range(k):
        v = A @ K[-1]
        K.append(v / np.linalg.norm(v))
    K = np.column_stack(K)                   # columns b, Ab, ..., A^k b (normalised)
    Lk = _lupp_L(K)
    assert np.allclose(out["Lmat"][:, :k + 1], Lk, atol=1e-9)
    # pivot order = LU row pivot order
    piv = [int(np.argmax(Lk[:, i] == 1.0)) for i in range(k + 1)]
    assert out["t"].tolist() == piv


def test_slslu_bases_are_lupp_of_krylov_matrices(orc):
    P, A = rect_problem(m=30, n=20, k=4)
    out = orc.solve(P, keep_basis=True)
    k = 4
    b = P.b
    KL = [A.T @ b]
    for _ in range(k - 1):
        KL.append(A.T @ (A @ KL[-1]))
    KD = [b]
    for _ in range(k):
        KD.append(A @ (A.T @ KD[-1]))
    KL = np.column_stack([v / np.linalg.norm(v) for v in KL])
    KD = np.column_stack([v / np.linalg.norm(v) for v in KD])
    assert np.allclose(out["Lmat"][:, :k], _lupp_L(KL), atol=1e-9)
    assert np.allclose(out["Dmat"][:, :k + 1], _lupp_L(KD), atol=1e-9)


# ------------------------------------------------------------------ S = I
def _orth_krylov(A, b, k):
    K = [b / np.linalg.norm(b)]
    for _ in range(k - 1):
        v = A @ K[-1]
        K.append(v / np.linalg.norm(v))
    Q, _ = np.linalg.qr(np.column_stack(K))
    return Q


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_scmrh_identity_sketch_is_minimum_residual(orc, lam):
    k = 6
    P = small_blur(k=k, lam=lam)
    P = P.replace(sketch=2, s=P.m)
    A = dense_of(orc, P)
    out = orc.solve(P)
    Q = _orth_krylov(A, P.b, k)
    M = np.vstack([A @ Q, lam * Q]) if lam > 0 else A @ Q
    rhs = np.concatenate([P.b, np.zeros(P.n)]) if lam > 0 else P.b
    z = np.linalg.lstsq(M, rhs, rcond=None)[0]
    x_ref = Q @ z
    assert np.linalg.norm(out["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    # the reported objective is the minimum over K_k
    assert np.isclose(out["res"][-1], np.linalg.norm(M @ z - rhs), rtol=1e-9)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_slslu_identity_sketch_is_damped_lsqr(orc, lam):
    k = 6
    P, A = rect_problem(m=40, n=25, k=k, lam=lam)
    P = P.replace(sketch=2, s=max(P.m, P.n))
    out = orc.solve(P)
    x_lsqr = lsqr(A, P.b, damp=lam, atol=0, btol=0, conlim=0, iter_lim=k)[0]
    assert np.linalg.norm(out["x"] - x_lsqr) <= 1e-8 * np.linalg.norm(x_lsqr)


def test_k_equals_n_gives_exact_solution(orc):
    n = 8
    rng = np.random.default_rng(11)
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    P = W.dense_problem("sq", A, b, k=n, s=n + 1)
    out = orc.solve(P, method=0)
    assert out["k_done"] == n
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(out["x"] - x) <= 1e-10 * np.linalg.norm(x)


# ------------------------------------------------------------------ breakdown
def test_breakdown_on_invariant_subspace(orc):
    n = 10
    A = np.diag(np.arange(1.0, n + 1))
    b = np.zeros(n); b[3] = 2.0
    P = W.dense_problem("d", A, b, k=5, s=12)
    out = orc.solve(P, method=0)
    assert out["status"] == orc.ORC_BREAKDOWN and out["k_done"] == 1
    assert out["H"][1, 0] == 0.0 and out["H"][0, 0] == 4.0
    x = np.zeros(n); x[3] = 0.5
    assert np.allclose(out["x"], x, rtol=1e-13, atol=1e-15)


def test_zero_rhs(orc):
    A = np.eye(6) * 2.0
    P = W.dense_problem("z", A, np.zeros(6), k=3, s=8)
    out = orc.solve(P, method=0)
    assert out["k_done"] == 0 and np.all(out["x"] == 0)


# ------------------------------------------------------------------ sketching laws
def test_residual_lower_bound_every_seed(orc):
    # eq. (eqthm2), left side: the sketched solution never beats the
    # minimum residual over the same subspace.
    k = 5
    P = small_blur(k=k, s=12)
    A = dense_of(orc, P)
    L = orc.solve(P, keep_basis=True)["Lmat"][:, :k]
    AL = A @ L
    rmin = np.linalg.norm(AL @ np.linalg.lstsq(AL, P.b, rcond=None)[0] - P.b)
    for seed in range(40):
        x = orc.solve(P, seed=seed)["x"]
        assert np.linalg.norm(A @ x - P.b) >= rmin * (1 - 1e-12)


def test_expected_residual_factor_and_unbiasedness(orc):
    # Sec. 3.2: E||A L y^S - b||^2 = (1 + k/(l-k-1)) min||A L y - b||^2 and
    # E[x^S] = x^LS for a Gaussian sketch (the basis L_k does not depend on S).
    k, s = 4, 14
    P = small_blur(k=k, s=s, ny=8, nx=8, r=2)
    A = dense_of(orc, P)
    L = orc.solve(P, keep_basis=True)["Lmat"][:, :k]
    AL = A @ L
    y_ls = np.linalg.lstsq(AL, P.b, rcond=None)[0]
    x_ls = L @ y_ls
    r2min = np.linalg.norm(AL @ y_ls - P.b) ** 2
    ratios, xs = [], []
    for seed in range(3000):
        x = orc.solve(P, seed=1000 + seed)["x"]
        ratios.append(np.linalg.norm(A @ x - P.b) ** 2 / r2min)
        xs.append(x)
    ratios = np.array(ratios)
    expect = 1 + k / (s - k - 1)
    se = ratios.std() / np.sqrt(len(ratios))
    assert abs(ratios.mean() - expect) < 4 * se
    xs = np.array(xs)
    se_x = xs.std(axis=0) / np.sqrt(len(xs))
    z = np.abs(xs.mean(axis=0) - x_ls) / np.maximum(se_x, 1e-300)
    assert np.mean(z < 4) > 0.97


# ------------------------------------------------------------------ small LS
@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_small_ls_matches_lstsq_and_prefix_residuals(orc, lam):
    rng = np.random.default_rng(2)
    s, k = 20, 7
    Z = rng.standard_normal((s, k)); F = rng.standard_normal((s, k)); c = rng.standard_normal(s)
    y, res = orc.small_ls(Z, F, lam, c)
    for j in range(1, k + 1):
        M = np.vstack([Z[:, :j], lam * F[:, :j]]) if lam > 0 else Z[:, :j]
        rhs = np.concatenate([c, np.zeros(s)]) if lam > 0 else c
        yj = np.linalg.lstsq(M, rhs, rcond=None)[0]
        assert np.isclose(res[j - 1], np.linalg.norm(M @ yj - rhs), rtol=1e-12)
        if j == k:
            assert np.allclose(y, yj, rtol=1e-12, atol=1e-13)
