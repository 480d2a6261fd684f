"""Pins for the oracle's unsketched variants, CMRH and LSLU (Sec. 3.1).

With sketch kind 3 the oracle solves eq. (TSP),
    min ||beta e_1 - H_{k+1,k} y||^2 + lambda^2 ||y||^2,
on the Hessenberg matrix of the basis it built.  It is checked against the
definitions it stands for, evaluated by brute force with pseudoinverses:
 - eq. (Hessenber_LS): x_k = argmin over x in R(L_k) of ||M_{k+1}^+ (A x - b)||,
   M = L for CMRH and M = D for LSLU;
 - eq. (TP): the same with the Tikhonov term lambda^2 ||L_k^+ x||^2;
 - the bound of eq. (eqthm): the minimum residual over R(L_k) is a lower
   bound for ||A x_k - b||, and kappa(M_{k+1}) times it an upper bound;
 - k = n on a nonsingular square system reaches the exact solution.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_hessenberg import dense_of, rect_problem, small_blur


def _brute(A, L, M, b, k, lam):
    """argmin_y ||M^+ (A L_k y - b)||^2 + lam^2 ||L_k^+ L_k y||^2 by dense lstsq."""
    Mp = np.linalg.pinv(M)
    Lk = L[:, :k]
    G = Mp @ A @ Lk
    rhs = Mp @ b
    if lam > 0:
        G = np.vstack([G, lam * (np.linalg.pinv(Lk) @ Lk)])
        rhs = np.concatenate([rhs, np.zeros(k)])
    y = np.linalg.lstsq(G, rhs, rcond=None)[0]
    return Lk @ y, np.linalg.norm(G @ y - rhs)


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_cmrh_is_oblique_projection(orc, lam):
    k = 6
    P = small_blur(k=k, lam=lam).replace(sketch=W.SKETCH_NONE)
    A = dense_of(orc, P)
    out = orc.solve(P, keep_basis=True)
    L = out["Lmat"]
    x_ref, obj = _brute(A, L, L[:, : k + 1], P.b, k, lam)
    assert np.linalg.norm(out["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert np.isclose(out["res"][-1], obj, rtol=1e-9)
    # prefix property: res[j] is the objective with j + 1 columns
    for j in range(1, k):
        _, oj = _brute(A, L, L[:, : j + 2], P.b, j + 1, lam)
        assert np.isclose(out["res"][j], oj, rtol=1e-8), j


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_lslu_is_oblique_projection(orc, lam):
    k = 6
    P, A = rect_problem(m=40, n=25, k=k, lam=lam)
    P = P.replace(sketch=W.SKETCH_NONE)
    out = orc.solve(P, keep_basis=True)
    L, D = out["Lmat"], out["Dmat"]
    x_ref, obj = _brute(A, L, D[:, : k + 1], P.b, k, lam)
    assert np.linalg.norm(out["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert np.isclose(out["res"][-1], obj, rtol=1e-9)


def test_cmrh_residual_within_kappa_of_minimum(orc):
    k = 7
    P = small_blur(k=k).replace(sketch=W.SKETCH_NONE)
    A = dense_of(orc, P)
    out = orc.solve(P, keep_basis=True)
    L = out["Lmat"]
    Lk, M = L[:, :k], L[:, : k + 1]
    y = np.linalg.lstsq(A @ Lk, P.b, rcond=None)[0]
    rmin = np.linalg.norm(A @ Lk @ y - P.b)
    r = np.linalg.norm(A @ out["x"] - P.b)
    assert rmin * (1 - 1e-12) <= r <= np.linalg.cond(M) * rmin * (1 + 1e-12)


def test_cmrh_k_equals_n_is_exact(orc):
    n = 8
    rng = np.random.default_rng(11)
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    P = W.dense_problem("sq", A, b, k=n, s=n + 1, sketch=W.SKETCH_NONE)
    out = orc.solve(P, method=0)
    assert out["k_done"] == n
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(out["x"] - x) <= 1e-10 * np.linalg.norm(x)


def test_unsketched_outputs_are_the_projected_problem(orc):
    """Z, F, c returned for the unsketched solve are H, [I; 0] and beta e_1."""
    k = 5
    P = small_blur(k=k, lam=0.1).replace(sketch=W.SKETCH_NONE)
    out = orc.solve(P, keep_basis=True)
    H = out["H"]
    assert out["Z"].shape == (k + 1, k)
    assert np.array_equal(out["Z"], H)
    assert np.array_equal(out["F"], np.eye(k + 1, k))
    t0 = int(out["t"][0])
    assert out["c"][0] == P.b[t0] and np.all(out["c"][1:] == 0.0)
