"""Pins for the oracle's sampled partial pivoting (Sec. 3.2: the pivot is the
largest magnitude in a small random sample of entries; the experiments use 5
entries for sCMRH and 25 for sLSLU).

The sample changes the pivots and the basis but not the Krylov subspace, so
what is fixed by the mathematics is checked:
 - the basis still satisfies the Hessenberg relations with exact zeros at
   earlier pivot rows and unit pivot entries, and its entries can now exceed
   1 in magnitude (the sample is active);
 - with S = I the solution is the same minimum-residual iterate as with full
   pivoting: GMRES over K_k(A, b) for sCMRH and damped LSQR for sLSLU, since
   x_k depends only on the subspace and on S;
 - the unsketched solution is the oblique projection of eq. (Hessenber_LS)
   for the sampled basis, by brute force with pseudoinverses;
 - the candidate rows floor(w len / 2^32) of the oracle's own (separately
   pinned) Philox words are uniform over the rows (chi-square).
"""
import numpy as np
import pytest
from scipy.sparse.linalg import lsqr

import workloads as W
from test_oracle_hessenberg import _orth_krylov, dense_of, rect_problem, small_blur
from test_oracle_unsketched import _brute


def test_sampled_basis_structure_and_relation(orc):
    k = 10
    P = small_blur(ny=16, nx=15, k=k).replace(pivot_sample=5)
    A = dense_of(orc, P)
    o = orc.solve(P, keep_basis=True)
    f = orc.solve(P.replace(pivot_sample=0), keep_basis=True)
    L, H, t = o["Lmat"], o["H"], [int(v) for v in o["t"]]
    assert len(set(t)) == len(t) == k + 1
    for j in range(k + 1):
        assert L[t[j], j] == 1.0
        assert np.all(L[t[:j], j] == 0.0)
    R = A @ L[:, :k] - L @ H
    assert np.max(np.abs(R)) <= 1e-12 * np.abs(A).sum(axis=1).max() * np.max(np.abs(L))
    assert np.max(np.abs(L)) > 1.0                      # sampling is active ...
    assert np.max(np.abs(f["Lmat"])) <= 1.0             # ... full pivoting keeps |l| <= 1
    assert [int(v) for v in f["t"]] != t


@pytest.mark.parametrize("ms", [1, 5, 25])
def test_sampled_cmrh_identity_sketch_is_gmres(orc, ms):
    k = 6
    P = small_blur(k=k).replace(sketch=2, pivot_sample=ms)
    P = P.replace(s=P.m)
    A = dense_of(orc, P)
    out = orc.solve(P)
    Q = _orth_krylov(A, P.b, k)
    z = np.linalg.lstsq(A @ Q, P.b, rcond=None)[0]
    assert np.linalg.norm(out["x"] - Q @ z) <= 1e-9 * np.linalg.norm(Q @ z)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_sampled_slslu_identity_sketch_is_damped_lsqr(orc, lam):
    k = 6
    P, A = rect_problem(m=40, n=25, k=k, lam=lam)
    P = P.replace(sketch=2, s=max(P.m, P.n), pivot_sample=25)
    out = orc.solve(P)
    x_lsqr = lsqr(A, P.b, damp=lam, atol=0, btol=0, conlim=0, iter_lim=k)[0]
    assert np.linalg.norm(out["x"] - x_lsqr) <= 1e-8 * np.linalg.norm(x_lsqr)


def test_sampled_unsketched_is_oblique_projection(orc):
    k = 6
    P = small_blur(k=k, lam=0.05).replace(sketch=W.SKETCH_NONE, pivot_sample=5)
    A = dense_of(orc, P)
    out = orc.solve(P, keep_basis=True)
    L = out["Lmat"]
    x_ref, obj = _brute(A, L, L[:, : k + 1], P.b, k, 0.05)
    assert np.linalg.norm(out["x"] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert np.isclose(out["res"][-1], obj, rtol=1e-9)


def test_sample_candidates_uniform(orc):
    n, draws = 37, 0
    counts = np.zeros(n)
    key = [0x02721, 0x2502]
    for i in range(400):
        for c in range(8):
            w = orc.philox4x32_10([c, i, 3, 0], key)
            r = (w.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)
            np.add.at(counts, r.astype(np.int64), 1)
            draws += 4
    e = draws / n
    chi2 = float(np.sum((counts - e) ** 2 / e))
    # 36 degrees of freedom: the 99.99% quantile is about 75
    assert chi2 < 75.0, chi2
