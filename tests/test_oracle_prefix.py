"""Pins for the oracle's prefix solutions (x after the first kp basis
vectors, eq. (sketched_LSLU) / eq. (sketched_LSLU_hybrid) on the first kp
columns), used for the per-iteration error report of the storage tier:
 - a prefix of a k-step solve equals a separate oracle solve stopped after
   kp steps with the same sketch (the Hessenberg process, the sketches and
   the pivots of the first kp steps do not depend on k);
 - its sketched objective, evaluated directly, equals res[kp-1] of the full
   run, which the Householder factorisation of all k columns reports by its
   own formula (norm of the discarded rotated right-hand side);
 - it equals an independent dense least-squares solve (numpy lstsq) of the
   stacked problem;
 - kp = k gives the run's own x.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_hessenberg import rect_problem, small_blur


def _objective(o, kp, lam, x_coef):
    Z, F, c = o["Z"][:, :kp], o["F"][:, :kp], o["c"]
    r = c - Z @ x_coef
    return np.sqrt(r @ r + lam * lam * np.sum((F @ x_coef) ** 2))


@pytest.mark.parametrize("case", ["blur_gauss", "blur_sparse_tik", "rect_gauss_tik", "blur_none"])
def test_prefix_solution_equals_the_shorter_solve(orc, case):
    if case == "blur_gauss":
        P, lam = small_blur(k=12, s=40), 0.0
    elif case == "blur_sparse_tik":
        P, lam = small_blur(k=12, s=40, lam=0.05, sketch=W.SKETCH_SPARSE_SIGN), 0.05
    elif case == "rect_gauss_tik":
        P, lam = rect_problem(k=10, s=36, lam=0.1)[0], 0.1
    else:
        P, lam = small_blur(k=12, lam=0.0).replace(sketch=W.SKETCH_NONE), 0.0
    full = orc.solve(P, keep_basis=True)
    k = full["k_done"]
    assert k == P.k
    for kp in (1, 3, 7, k - 1, k):
        xp = orc.prefix_solution(full, kp, lam)
        if P.sketch == W.SKETCH_NONE:
            short = orc.solve(P.replace(k=kp))        # s = kp + 1 rows: H_{kp+1,kp}
        else:
            short = orc.solve(P.replace(k=kp), s=P.s)
        scale = np.max(np.abs(short["x"]))
        assert np.max(np.abs(xp - short["x"])) <= 1e-10 * scale, kp
        # the objective at the prefix minimiser is the full run's res[kp-1]
        Lk = full["Lmat"][:, :kp]
        yk = np.linalg.lstsq(Lk, xp, rcond=None)[0]
        assert abs(_objective(full, kp, lam, yk) - full["res"][kp - 1]) <= 1e-10 * max(1.0, full["res"][0])
    np.testing.assert_allclose(orc.prefix_solution(full, k, lam), full["x"], rtol=0, atol=1e-12 * scale)


def test_prefix_solution_matches_dense_lstsq(orc):
    P = small_blur(k=10, s=30, lam=0.2)
    lam = 0.2
    full = orc.solve(P, keep_basis=True)
    for kp in (2, 5, 9):
        M = np.vstack([full["Z"][:, :kp], lam * full["F"][:, :kp]])
        rhs = np.concatenate([full["c"], np.zeros(P.s)])
        y = np.linalg.lstsq(M, rhs, rcond=None)[0]
        x_ref = full["Lmat"][:, :kp] @ y
        xp = orc.prefix_solution(full, kp, lam)
        assert np.max(np.abs(xp - x_ref)) <= 1e-11 * np.max(np.abs(x_ref))


def test_prefix_solution_rejects_bad_lengths(orc):
    P = small_blur(k=5)
    full = orc.solve(P, keep_basis=True)
    for kp in (0, 6):
        with pytest.raises(ValueError):
            orc.prefix_solution(full, kp, 0.0)
