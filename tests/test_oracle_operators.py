"""Pins for the oracle's operators (A and A^T reached only through products,
Sec. 1 eq. (1); blur model of Sec. 4.1, tomography of Sec. 4.2).

Pinned against SciPy's library routines (2-D correlation, sparse products),
the Kronecker form of a separable blur, and the adjoint identity."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy import ndimage

import workloads as W


def _blur_problem(ny, nx, r, bc, seed=0):
    rng = np.random.default_rng(seed)
    ty = rng.uniform(0.1, 1.0, 2 * r + 1)
    tx = rng.uniform(0.1, 1.0, 2 * r + 1)
    return W.Problem(name="t", kind="blur", m=ny * nx, n=ny * nx, b=np.zeros(ny * nx),
                     x_true=np.zeros(ny * nx), k=1, s=2, lam=0.0, sketch=0, zeta=1, seed=0,
                     dtype="f64", ny=ny, nx=nx, taps_y=ty, taps_x=tx, radius=r, bc=bc)


@pytest.mark.parametrize("bc,mode", [(W.BC_ZERO, "constant"), (W.BC_REFLECT, "reflect")])
@pytest.mark.parametrize("ny,nx,r", [(9, 13, 2), (16, 16, 7), (5, 40, 3), (31, 31, 15)])
def test_blur_matches_scipy_correlate(orc, bc, mode, ny, nx, r):
    P = _blur_problem(ny, nx, r, bc)
    op = orc.Operator(P)
    img = np.random.default_rng(1).standard_normal((ny, nx))
    got = op.apply(img.ravel()).reshape(ny, nx)
    ref = ndimage.correlate(img, np.outer(P.taps_y, P.taps_x), mode=mode, cval=0.0)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("bc,mode", [(W.BC_ZERO, "constant"), (W.BC_REFLECT, "reflect")])
@pytest.mark.parametrize("kind,ny,nx,r", [("motion", 20, 23, 6), ("random", 9, 13, 2), ("random", 31, 31, 15)])
def test_general_psf_matches_scipy_correlate(orc, bc, mode, kind, ny, nx, r):
    # a PSF of full rank (random) or a motion blur at 30 degrees (rank > 1):
    # the oracle's definitional correlation against SciPy's
    if kind == "motion":
        psf = W.motion_psf(2 * r - 1, 30.0, r)
        assert np.linalg.matrix_rank(psf) > 1
    else:
        psf = np.random.default_rng(7).uniform(-0.5, 1.0, (2 * r + 1, 2 * r + 1))
    P = _blur_problem(ny, nx, r, bc).replace(psf=psf, taps_y=None, taps_x=None)
    op = orc.Operator(P)
    img = np.random.default_rng(2).standard_normal((ny, nx))
    got = op.apply(img.ravel()).reshape(ny, nx)
    ref = ndimage.correlate(img, psf, mode=mode, cval=0.0)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    # an asymmetric PSF: its operator's transpose is the correlation with the
    # flipped PSF under the zero boundary (A^T y = sum_a,b p(a, b) y(. - a, . - b))
    if bc == W.BC_ZERO:
        y = np.random.default_rng(3).standard_normal((ny, nx))
        at_y = ndimage.correlate(y, psf[::-1, ::-1], mode="constant", cval=0.0)
        assert np.isclose(np.dot(got.ravel(), y.ravel()), np.dot(img.ravel(), at_y.ravel()), rtol=1e-12)


def test_motion_psf_geometry():
    # sums to one, lies on the segment, symmetric under a half turn, and is
    # rank one (a row) only when the motion is horizontal
    r = 7
    p0 = W.motion_psf(9.0, 0.0, r)
    p30 = W.motion_psf(9.0, 30.0, r)
    assert np.isclose(p0.sum(), 1.0) and np.isclose(p30.sum(), 1.0)
    assert np.linalg.matrix_rank(p0) == 1 and np.count_nonzero(p0.sum(axis=1)) == 1
    assert np.linalg.matrix_rank(p30) > 1
    assert np.allclose(p30, p30[::-1, ::-1])
    yy, xx = np.nonzero(p30)
    # every weight sits within one grid step (in each axis) of the segment:
    # its distance from the line is below |cos| + |sin|
    d = np.abs((yy - r) * np.cos(np.pi / 6) + (xx - r) * np.sin(np.pi / 6))
    assert np.all(d < np.cos(np.pi / 6) + np.sin(np.pi / 6))
    assert np.max(np.hypot(yy - r, xx - r)) <= 4.5 + np.sqrt(2)


def test_blur_is_kronecker_of_1d_operators(orc):
    # separable PSF: A = A_y (x) A_x, with A_y, A_x the 1-D correlation matrices
    ny, nx, r = 7, 6, 2
    P = _blur_problem(ny, nx, r, W.BC_ZERO)

    def corr1d(N, t):
        M = np.zeros((N, N))
        for i in range(N):
            for a in range(-r, r + 1):
                if 0 <= i + a < N:
                    M[i, i + a] += t[a + r]
        return M

    A = np.kron(corr1d(ny, P.taps_y), corr1d(nx, P.taps_x))
    op = orc.Operator(P)
    dense = np.column_stack([op.apply(e) for e in np.eye(ny * nx)])
    assert np.allclose(dense, A, rtol=1e-14, atol=1e-15)


def test_symmetric_psf_zero_bc_gives_symmetric_operator(orc):
    ny, nx, r = 8, 9, 3
    t = W.gaussian_taps(1.5, r)
    P = _blur_problem(ny, nx, r, W.BC_ZERO).replace(taps_y=t, taps_x=t.copy())
    op = orc.Operator(P)
    dense = np.column_stack([op.apply(e) for e in np.eye(ny * nx)])
    assert np.allclose(dense, dense.T, atol=1e-15)


def test_blur_pixel_matches_full_apply(orc):
    P = _blur_problem(12, 10, 4, W.BC_REFLECT)
    op = orc.Operator(P)
    img = np.random.default_rng(3).standard_normal(120)
    full = op.apply(img).reshape(12, 10)
    for (y, x) in [(0, 0), (11, 9), (5, 3), (0, 9)]:
        assert op.blur_pixel(img, y, x) == full[y, x]


def _csr(m, n, density, seed):
    A = sp.random(m, n, density=density, random_state=seed, format="csr")
    A.sort_indices()
    return A


def test_csr_products_match_scipy(orc):
    A = _csr(37, 23, 0.2, 4)
    P = W.dense_problem("t", A.toarray(), np.zeros(37), k=1, s=2)
    op = orc.Operator(P)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(23), rng.standard_normal(37)
    assert np.allclose(op.apply(x), A @ x, rtol=1e-14, atol=1e-14)
    assert np.allclose(op.apply_t(y), A.T @ y, rtol=1e-14, atol=1e-14)
    # adjoint identity <A x, y> = <x, A^T y>
    assert np.isclose(op.apply(x) @ y, x @ op.apply_t(y), rtol=1e-13)


def test_joseph_projector_rows():
    # Interior rays at 0 and 90 degrees cross the full N-pixel image: the
    # weights along them sum to the chord length N (unit pixels).
    N = 32
    rowptr, col, val, m, n = W.joseph_parallel_csr(N, 12, 46, dtype=np.float64)
    A = sp.csr_matrix((val, col, rowptr), shape=(m, n))
    sums = np.asarray(A.sum(axis=1)).ravel().reshape(12, 46)
    centre = 46 // 2
    for a in (0, 6):    # theta = 0 and 90 degrees
        assert np.allclose(sums[a, centre - 5:centre + 5], N, rtol=1e-12)
    # a diagonal ray (45 degrees) through the centre has chord length ~ N*sqrt(2)
    assert abs(sums[3, centre] - N * np.sqrt(2)) / (N * np.sqrt(2)) < 0.03
    assert val.min() > 0
    # the projection of a constant image: every ray's sum equals its weight sum
    assert np.allclose(A @ np.ones(n), sums.ravel())
