"""GPU parity: the HIP path, called through the C ABI, against the FP64
oracle on identical seeded inputs.

Bars: pivot sequences bit-exact except at excused near-ties; relative
solution error <= 1e-10 with FP64 storage and <= 1e-4 with FP32 storage;
H, the sketches and the residual history agree on the common pivot prefix;
operator products agree to rounding.
"""
import numpy as np
import pytest

import workloads as W
from hk_gpu import sensitivity_bars, compare_solve, gpu_solve, random_csr, rel, rounded_problem, storage_np, tiny_blur

pytestmark = pytest.mark.gpu


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


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ny,nx,r,bc", [(64, 64, 7, W.BC_ZERO), (50, 70, 3, W.BC_REFLECT),
                                        (37, 129, 15, W.BC_ZERO), (512, 512, 15, W.BC_REFLECT)])
def test_blur_apply(hk, ctx, orc, dtype, ny, nx, r, bc):
    import torch
    _flush(f"blur apply {ny}x{nx} r={r} bc={bc} {dtype}")
    P = tiny_blur(ny, nx, r / 3.5, r, bc, k=1, s=2, dtype=dtype)
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    x = np.random.default_rng(3).standard_normal(P.n).astype(storage_np(dtype))
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    ref = orc.Operator(P).apply(x.astype(np.float64))
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert np.max(np.abs(y - ref)) <= tol * np.max(np.abs(ref))


def motion_blur(ny, nx, length, angle, r, bc, k, s, lam=0.0, sketch=W.SKETCH_SPARSE_SIGN, zeta=4, dtype="f32"):
    """A deblurring problem under linear motion blur (a PSF of rank > 1)."""
    return W.blur_problem(f"motion{ny}x{nx}", ny, nx, None, r, bc, "piecewise", 0.01, k=k, s=s, lam=lam,
                          sketch=sketch, zeta=zeta, dtype=dtype, cfg_id=8, psf=W.motion_psf(length, angle, r))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ny,nx,r,bc,kind", [(64, 64, 7, W.BC_ZERO, "motion"), (50, 70, 3, W.BC_REFLECT, "random"),
                                             (512, 512, 15, W.BC_REFLECT, "motion"),
                                             (37, 129, 15, W.BC_ZERO, "random")])
def test_general_psf_apply(hk, ctx, orc, dtype, ny, nx, r, bc, kind):
    import torch
    _flush(f"general PSF apply {ny}x{nx} r={r} bc={bc} {kind} {dtype}")
    if kind == "motion":
        psf = W.motion_psf(2 * r - 1, 30.0, r)
    else:
        psf = np.random.default_rng(9).uniform(-0.2, 1.0, (2 * r + 1, 2 * r + 1))
    P = tiny_blur(ny, nx, 1.0, r, bc, k=1, s=2, dtype=dtype).replace(psf=psf)
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    x = np.random.default_rng(3).standard_normal(P.n).astype(storage_np(dtype))
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    ref = orc.Operator(P).apply(x.astype(np.float64))
    tol = 1e-14 if dtype == "f64" else 1e-6
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    _flush(f"  max rel {err:.2e}")
    assert err <= tol


def test_general_psf_limits(hk, ctx):
    from hk_gpu import make_operator
    P = tiny_blur(64, 64, 1.0, 25, W.BC_ZERO, k=1, s=2)
    dense = np.full((51, 51), 1.0 / 51 ** 2)
    dense[0, 0] *= 2.0          # not of rank one: 2601 nonzero taps
    with pytest.raises(hk.HKError) as e:
        make_operator(hk, ctx, P.replace(psf=dense))
    assert e.value.status == hk.HK_EUNSUPPORTED
    bad = np.zeros((5, 5)); bad[2, 2] = np.nan
    with pytest.raises(hk.HKError) as e:
        make_operator(hk, ctx, tiny_blur(16, 16, 1.0, 2, W.BC_ZERO, k=1, s=2).replace(psf=bad))
    assert e.value.status == hk.HK_ENUMERIC


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_csr_apply_and_transpose(hk, ctx, orc, dtype):
    import torch
    _flush(f"csr apply {dtype}")
    P = random_csr(700, 333, 0.05, k=1, s=2, dtype=dtype)
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(P.n).astype(storage_np(dtype))
    z = rng.standard_normal(P.m).astype(storage_np(dtype))
    O = orc.Operator(rounded_problem(P))
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    yt = op.apply(torch.tensor(z, device="cuda"), transpose=True).cpu().numpy().astype(np.float64)
    tol = 1e-13 if dtype == "f64" else 1e-6
    assert rel(y, O.apply(x.astype(np.float64))) <= tol
    assert rel(yt, O.apply_t(z.astype(np.float64))) <= tol


# ---------------------------------------------------------------- sCMRH
def _parity(hk, ctx, orc, P, method=0, bars=None, max_workgroups=0):
    _flush(f"solve {P.name} m={P.m} n={P.n} k={P.k} s={P.s} lam={P.lam} sketch={P.sketch} {P.dtype} "
           f"max_workgroups={max_workgroups}")
    Pr = rounded_problem(P)
    o = orc.solve(Pr, keep_basis=True, method=None if method == 0 else (0 if method == 1 else 1))
    g = gpu_solve(hk, ctx, P, method=method, max_workgroups=max_workgroups)
    err = compare_solve(Pr, g, o, bars)
    _flush(f"  rel x err {err:.3e}, k_done {g['k_done']}")
    return g, o


@pytest.mark.parametrize("name", ["c1", "c1_tik"])
def test_scmrh_64x64_fp64(hk, ctx, orc, name):
    _parity(hk, ctx, orc, W.config(name))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("sketch,lam", [(W.SKETCH_GAUSSIAN, 0.0), (W.SKETCH_SPARSE_SIGN, 0.0),
                                        (W.SKETCH_GAUSSIAN, 1e-2), (W.SKETCH_SPARSE_SIGN, 1e-2)])
def test_scmrh_ragged_image(hk, ctx, orc, dtype, sketch, lam):
    # 50 x 70 image: several tiles with a ragged right and bottom edge
    P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=lam, sketch=sketch, zeta=5, dtype=dtype)
    _parity(hk, ctx, orc, P)


# ---------------------------------------------------------------- sLSLU
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("sketch,lam", [(W.SKETCH_GAUSSIAN, 0.0), (W.SKETCH_SPARSE_SIGN, 0.5)])
@pytest.mark.parametrize("m,n", [(900, 613), (613, 900)])
def test_slslu_random_csr(hk, ctx, orc, dtype, sketch, lam, m, n):
    P = random_csr(m, n, 0.02, k=20, s=44, lam=lam, sketch=sketch, zeta=3, dtype=dtype)
    _parity(hk, ctx, orc, P)


def test_scmrh_on_square_csr(hk, ctx, orc):
    P = random_csr(500, 500, 0.03, k=30, s=62, dtype="f64")
    _parity(hk, ctx, orc, P, method=hk.HK_METHOD_HESSENBERG)


# ---------------------------------------------------------------- unsketched CMRH / LSLU
# eq. (TSP) on the H the kernels build: no sketch partials, F = [I; 0],
# c = beta e_1, the same small least-squares kernel
@pytest.mark.parametrize("name,dtype,lam", [("blur64", "f64", 0.0), ("blur64", "f64", 1e-3),
                                            ("ragged", "f32", 1e-2), ("deblur512", "f32", 1e-2)])
def test_cmrh_unsketched(hk, ctx, orc, name, dtype, lam):
    if name == "blur64":
        P = W.config("c1").replace(lam=lam)
    elif name == "ragged":
        P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=lam, dtype=dtype)
    else:
        P = W.config("c2")
    _parity(hk, ctx, orc, P.replace(sketch=W.SKETCH_NONE))


@pytest.mark.parametrize("dtype,lam", [("f64", 0.0), ("f64", 0.5), ("f32", 0.0)])
def test_lslu_unsketched_random_csr(hk, ctx, orc, dtype, lam):
    P = random_csr(900, 613, 0.02, k=20, s=44, lam=lam, dtype=dtype)
    _parity(hk, ctx, orc, P.replace(sketch=W.SKETCH_NONE))


def test_cmrh_unsketched_square_csr(hk, ctx, orc):
    P = random_csr(500, 500, 0.03, k=30, s=62, dtype="f64")
    _parity(hk, ctx, orc, P.replace(sketch=W.SKETCH_NONE), method=hk.HK_METHOD_HESSENBERG)


# ---------------------------------------------------------------- sampled pivoting
# the pivot is the largest |v| in a Philox-drawn sample of non-pivot rows
# (5 rows for sCMRH and 25 for sLSLU in the paper's experiments)
@pytest.mark.parametrize("name,sketch,lam,ms", [("blur64", W.SKETCH_GAUSSIAN, 0.0, 5),
                                                ("blur64", W.SKETCH_NONE, 1e-3, 5),
                                                ("ragged_f32", W.SKETCH_SPARSE_SIGN, 1e-2, 5),
                                                ("ragged_f64", W.SKETCH_GAUSSIAN, 0.0, 1),
                                                ("deblur512", W.SKETCH_SPARSE_SIGN, 1e-2, 5)])
def test_cmrh_sampled_pivots(hk, ctx, orc, name, sketch, lam, ms):
    if name == "blur64":
        P = W.config("c1").replace(lam=lam)
    elif name.startswith("ragged"):
        P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=lam, sketch=sketch, zeta=5,
                      dtype=name[-3:])
    else:
        # FP64 basis storage: with 5-row samples the basis entries grow past 1
        # and FP32 storage rounding, compounded over 100 columns, moves H by
        # about 3e-3 (x still agrees to 5e-5); the sampled pivot path is
        # checked here with the basis rounding taken out
        P = W.config("c2").replace(basis="f64")
    _parity(hk, ctx, orc, P.replace(sketch=sketch, lam=lam, pivot_sample=ms))


@pytest.mark.parametrize("dtype,sketch,lam", [("f64", W.SKETCH_GAUSSIAN, 0.0), ("f64", W.SKETCH_NONE, 0.5),
                                              ("f32", W.SKETCH_SPARSE_SIGN, 0.5)])
def test_lslu_sampled_pivots_random_csr(hk, ctx, orc, dtype, sketch, lam):
    P = random_csr(900, 613, 0.02, k=20, s=44, lam=lam, sketch=sketch, zeta=3, dtype=dtype)
    _parity(hk, ctx, orc, P.replace(pivot_sample=25))


def long_row_csr(m, n, step, k, s, dtype, seed=17):
    """CSR with row i holding (i * step) % n entries (empty rows included;
    most rows longer than the 512 entries a wave loads in one batch), at
    random sorted columns, values in [0.1, 1)."""
    rng = np.random.default_rng(seed)
    lens = (np.arange(m) * step) % n
    rowptr = np.zeros(m + 1, np.int64)
    rowptr[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, L, replace=False)) for L in lens]).astype(np.int32)
    val = rng.uniform(0.1, 1.0, int(rowptr[-1]))
    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, rowptr), shape=(m, n))
    b = A @ rng.uniform(0, 1, n) + 0.01 * rng.standard_normal(m)
    return W.Problem(name=f"longrows{m}x{n}", kind="csr", m=m, n=n, b=b, x_true=np.zeros(n), k=k, s=s,
                     lam=0.0, sketch=W.SKETCH_GAUSSIAN, zeta=4, seed=W.SKETCH_SEED_BASE + 13, dtype=dtype,
                     rowptr=rowptr, col=col, val=val.astype(storage_np(dtype)))


@pytest.mark.parametrize("shape", ["square", "rect"])
def test_csr_rows_longer_than_one_batch(hk, ctx, orc, shape):
    # rows of 0 to about 1400 entries: a wave takes rows of more than 512
    # entries in several batches, and empty rows as a whole
    if shape == "square":
        P = long_row_csr(1200, 1200, 37, k=20, s=42, dtype="f64")
        assert np.diff(P.rowptr).max() > 1024 and (np.diff(P.rowptr) == 0).any()
        _parity(hk, ctx, orc, P, method=hk.HK_METHOD_HESSENBERG)
    else:
        P = long_row_csr(700, 1500, 53, k=20, s=42, dtype="f64")
        assert np.diff(P.rowptr).max() > 1024
        _parity(hk, ctx, orc, P)


def test_cmrh_sampled_pivots_square_csr(hk, ctx, orc):
    P = random_csr(500, 500, 0.03, k=30, s=62, dtype="f64").replace(pivot_sample=5)
    _parity(hk, ctx, orc, P, method=hk.HK_METHOD_HESSENBERG)


# ---------------------------------------------------------------- edge cases
def test_breakdown_invariant_subspace(hk, ctx, orc):
    n = 300
    A = np.diag(np.arange(1.0, n + 1))
    b = np.zeros(n); b[123] = 2.0
    P = W.dense_problem("diag", A, b, k=5, s=12)
    g = gpu_solve(hk, ctx, P, method=hk.HK_METHOD_HESSENBERG)
    assert g["status"] == hk.HK_BREAKDOWN and g["k_done"] == 1
    x = np.zeros(n); x[123] = 2.0 / 124.0
    assert rel(g["x"], x) <= 1e-14
    assert g["t"][0] == 123 and np.all(g["t"][1:] == -1)


def test_zero_rhs(hk, ctx):
    P = tiny_blur(32, 32, 1.0, 3, W.BC_ZERO, k=4, s=10).replace(b=np.zeros(1024))
    g = gpu_solve(hk, ctx, P)
    assert g["k_done"] == 0 and np.all(g["x"] == 0) and g["status"] == hk.HK_BREAKDOWN


def test_k_equals_n_exact_solve(hk, ctx):
    n = 12
    rng = np.random.default_rng(11)
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    P = W.dense_problem("sq", A, b, k=n, s=n + 1)
    g = gpu_solve(hk, ctx, P, method=hk.HK_METHOD_HESSENBERG)
    assert g["k_done"] == n
    assert rel(g["x"], np.linalg.solve(A, b)) <= 1e-10


@pytest.mark.parametrize("dtype,k", [("f32", 255), ("f64", 180)])
def test_largest_k(hk, ctx, orc, dtype, k):
    # k = 255, the largest basis the kernels hold (k + 1 pivot slots); the
    # pivot block (k (k + 1) / 2 entries) lives in LDS, which bounds k at
    # about 180 for FP64 bases.  A random sparse matrix keeps the long basis
    # well conditioned: on a 64 x 64 blur the FP64 oracle's own pivots split
    # at step 77 under one-ulp changes of b, so no bar would hold there.
    P = random_csr(1200, 1200, 0.02, k=k, s=2 * (k + 1), lam=1e-3, dtype=dtype)
    _parity(hk, ctx, orc, P, method=hk.HK_METHOD_HESSENBERG)


def test_k_beyond_lds_refused(hk, ctx):
    P = tiny_blur(64, 64, 2.0, 7, W.BC_ZERO, k=255, s=512, dtype="f64")
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    with pytest.raises(hk.HKError) as e:
        hk.Solve(op, k=255, s=512)
    assert e.value.status == hk.HK_EUNSUPPORTED


def test_largest_image(hk, ctx, orc):
    # n = 524288 = 256 tiles of 2048 pixels, the largest single-kernel plan
    P = tiny_blur(1024, 512, 2.0, 7, W.BC_REFLECT, k=12, s=48, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN,
                  zeta=8, dtype="f32")
    _parity(hk, ctx, orc, P)


@pytest.mark.parametrize("r,bc,dtype,sketch", [(16, W.BC_ZERO, "f64", W.SKETCH_SPARSE_SIGN),
                                               (20, W.BC_REFLECT, "f32", W.SKETCH_SPARSE_SIGN),
                                               (23, W.BC_ZERO, "f32", W.SKETCH_GAUSSIAN)])
def test_wide_stencil_windows(hk, ctx, orc, r, bc, dtype, sketch):
    # a grid capped at 128 workgroups tiles the 512 x 512 image in 32 x 64
    # tiles, so a (2r+1)-wide window with r >= 16 meets a tile in more than
    # 32 columns: the window sums of u at the pivots take several column
    # passes per lane (the single-barrier kernel's LDS plan fits these
    # cases: zeta = 4 keeps the sparse-sign row lists at 32 KiB)
    P = tiny_blur(512, 512, (r + 1) / 4.0, r, bc, k=12, s=48, lam=1e-2, sketch=sketch,
                  zeta=4, dtype=dtype)
    g, _ = _parity(hk, ctx, orc, P, max_workgroups=128)
    assert g["grid"] == 128


@pytest.mark.parametrize("kind,bad", [("blur", np.nan), ("blur", np.inf), ("csr", np.nan), ("csr", -np.inf)])
def test_nonfinite_rhs_is_numeric_error(hk, ctx, kind, bad):
    if kind == "blur":
        P = tiny_blur(64, 64, 2.0, 7, W.BC_REFLECT, k=10, s=40, sketch=W.SKETCH_SPARSE_SIGN, dtype="f32")
    else:
        P = random_csr(900, 613, 0.02, k=10, s=30, dtype="f64")
    b = P.b.copy()
    b[len(b) // 3] = bad
    with pytest.raises(hk.HKError) as e:
        gpu_solve(hk, ctx, P.replace(b=b), keep_basis=False)
    _flush(f"  {kind} with {bad} in b: status {e.value.status}")
    assert e.value.status == hk.HK_ENUMERIC


def test_rank_deficient_small_problem(hk, ctx, orc):
    # b lies in the null space of A: A l_1 = 0 ends the basis after one
    # column and the sketched problem's only column S2 A l_1 is zero
    n = 300
    d = np.arange(1.0, n + 1)
    d[123] = 0.0
    b = np.zeros(n); b[123] = 2.0
    P = W.dense_problem("nullspace", np.diag(d), b, k=5, s=12)
    with pytest.raises(RuntimeError):
        orc.solve(P, method=0)            # the oracle reports it too (R_11 = 0)
    with pytest.raises(hk.HKError) as e:
        gpu_solve(hk, ctx, P, method=hk.HK_METHOD_HESSENBERG, keep_basis=False)
    assert e.value.status == hk.HK_ENUMERIC


# ---------------------------------------------------------------- general PSF (motion blur)
@pytest.mark.parametrize("case", ["512_f32_sparse", "ragged_f64_gauss", "ragged_f32_none", "rank1_as_2d"])
def test_scmrh_general_psf(hk, ctx, orc, case):
    # the deblurring experiment's motion blur (Sec. 4.1): a PSF of rank > 1
    # through the stencil's tap list; a rank-one PSF given as a 2-D array
    # takes the separable path
    if case == "512_f32_sparse":
        P = motion_blur(512, 512, 21.0, 30.0, 15, W.BC_REFLECT, k=40, s=160, lam=1e-2)
    elif case == "ragged_f64_gauss":
        P = motion_blur(50, 70, 9.0, 60.0, 6, W.BC_ZERO, k=25, s=60, sketch=W.SKETCH_GAUSSIAN, dtype="f64")
    elif case == "ragged_f32_none":
        P = motion_blur(50, 70, 9.0, 120.0, 6, W.BC_REFLECT, k=25, s=60, lam=1e-2, sketch=W.SKETCH_NONE)
    else:
        t = W.gaussian_taps(1.5, 5)
        P = tiny_blur(50, 70, 1.5, 5, W.BC_REFLECT, k=25, s=60, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN, zeta=5,
                      dtype="f64").replace(psf=np.outer(t, t))
    _parity(hk, ctx, orc, P)


def test_large_sketch_column_ls(hk, ctx, orc):
    # s = 8192: the blocked least-squares panel does not fit in LDS, so the
    # column-by-column kernel solves the small problem
    P = tiny_blur(64, 64, 2.0, 7, W.BC_ZERO, k=12, s=8192, lam=0.0, sketch=W.SKETCH_GAUSSIAN, dtype="f64")
    _parity(hk, ctx, orc, P)


def test_image_too_large_refused(hk, ctx):
    P = tiny_blur(1024, 1024, 2.0, 7, W.BC_ZERO, k=4, s=10, dtype="f32")
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    with pytest.raises(hk.HKError) as e:
        hk.Solve(op, k=4, s=10)
    assert e.value.status == hk.HK_EUNSUPPORTED


def test_repeat_runs_are_bitwise_identical(hk, ctx):
    P = tiny_blur(64, 96, 2.0, 7, W.BC_REFLECT, k=30, s=62, lam=1e-3, sketch=W.SKETCH_SPARSE_SIGN,
                  dtype="f32")
    g = gpu_solve(hk, ctx, P, runs=3, keep_basis=False)
    assert all(np.array_equal(g["xs"][0], x) for x in g["xs"][1:])


def test_invalid_parameters_rejected(hk, ctx):
    P = tiny_blur(16, 16, 1.0, 2, W.BC_ZERO, k=4, s=10)
    from hk_gpu import make_operator
    op = make_operator(hk, ctx, P)
    for kw in [dict(k=0, s=10), dict(k=4, s=4), dict(k=4, s=10, lam=-1.0), dict(k=300, s=400),
               dict(k=4, s=10, sketch=hk.HK_SKETCH_SPARSE_SIGN, zeta=11)]:
        with pytest.raises(hk.HKError):
            hk.Solve(op, **kw)
    with pytest.raises(hk.HKError) as e:
        hk.Solve(op, k=4, s=10, method=hk.HK_METHOD_CHANGING_HESSENBERG)
    assert e.value.status == hk.HK_EUNSUPPORTED


# ---------------------------------------------------------------- full-size workloads
def test_scmrh_512_fp32_sparse_sign(hk, ctx, orc):
    # the full 512 x 512 deblurring workload (k = 100, s = 400, zeta = 8, lambda = 1e-2)
    _parity(hk, ctx, orc, W.config("c2"))


def test_slslu_tomography_fp32(hk, ctx, orc):
    # the full 256 x 256 parallel-beam workload (180 x 362 rays, k = 150, s = 302);
    # its FP64 result is rounding-sensitive, so the near-tie and intermediate
    # bars come from the oracle's own one-ulp spread (x keeps the FP32 bar)
    _parity(hk, ctx, orc, W.config("c3"), bars=sensitivity_bars("c3"))
