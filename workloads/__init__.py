"""Seeded synthetic inputs for the sketched inner-product-free Krylov solvers.

This module only *makes inputs*: phantoms, point-spread-function taps, a
parallel-beam projection matrix in CSR form, and noisy data b.  It holds none
of the solver's arithmetic (no Hessenberg step, no sketch, no least squares);
the forward model used to synthesise b is applied with SciPy library routines
(``scipy.ndimage.correlate`` / ``scipy.sparse``), which neither the CPU oracle
nor the HIP library uses.  Both the oracle and the GPU path consume the arrays
built here, so they are fed identical inputs.

The paper's data (Sec. 4: a 256x256 test image under motion blur, a simulated
neutron tomography image, two X-ray datasets) is not available; the recipes
below are synthetic stand-ins with the same structure: a linear inverse problem
b = A x_true + e (Sec. 1, eq. (1)) with a blur or a tomography operator and
Gaussian noise at a fixed relative level.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

PHANTOM_SEED = 2502
NOISE_SEED = 2721
SKETCH_SEED_BASE = 0x250202721

BC_ZERO = 0
BC_REFLECT = 1

SKETCH_GAUSSIAN = 0
SKETCH_SPARSE_SIGN = 1
SKETCH_NONE = 3          # no sketch: the CMRH / LSLU projected problem


# --------------------------------------------------------------------------
# point-spread functions
# --------------------------------------------------------------------------
def gaussian_taps(sigma: float, radius: int) -> np.ndarray:
    """1-D taps g(a) ~ exp(-a^2 / (2 sigma^2)), a = -radius..radius, sum 1.

    The 2-D Gaussian PSF is the outer product g(a) g(b); with both factors
    normalised it sums to one, so the blur preserves the mean intensity.
    """
    a = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(a * a) / (2.0 * sigma * sigma))
    return g / g.sum()


def motion_psf(length: float, angle_deg: float, radius: int) -> np.ndarray:
    """Linear motion blur on a (2r+1) x (2r+1) grid: a segment of `length`
    pixels through the centre at `angle_deg` (counter-clockwise from the x
    axis, image rows pointing down), sampled at 8 points per pixel of length,
    each sample spread bilinearly over its four nearest grid points; the
    array sums to one.  A PSF of rank > 1 unless the segment is axis-aligned.
    Indexing: psf[a + r, b + r] weighs the pixel at offset (a, b) (row,
    column) in the correlation (A u)(y, x) = sum psf[a+r, b+r] u(y+a, x+b)."""
    w = 2 * radius + 1
    psf = np.zeros((w, w))
    th = np.deg2rad(angle_deg)
    ns = max(2, int(np.ceil(8 * length)) + 1)
    for t in np.linspace(-length / 2.0, length / 2.0, ns):
        py, px = -t * np.sin(th) + radius, t * np.cos(th) + radius
        y0, x0 = int(np.floor(py)), int(np.floor(px))
        fy, fx = py - y0, px - x0
        for dy, wy in ((0, 1.0 - fy), (1, fy)):
            for dx, wx in ((0, 1.0 - fx), (1, fx)):
                yy, xx = y0 + dy, x0 + dx
                if 0 <= yy < w and 0 <= xx < w:
                    psf[yy, xx] += wy * wx
    return psf / psf.sum()


def radius_for_sigma(sigma: float) -> int:
    """Stencil half-width r = round(4 sigma) - 1 (sigma 2 -> 15x15, 4 -> 31x31)."""
    return max(1, int(round(4.0 * sigma)) - 1)


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
def _grid(ny: int, nx: int):
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64),
                         np.arange(nx, dtype=np.float64), indexing="ij")
    return yy, xx


def phantom_blobs(ny: int, nx: int, rng: np.random.Generator) -> np.ndarray:
    """Sum of 10 Gaussian blobs and 5 axis-aligned rectangles, clipped to [0, 1]."""
    yy, xx = _grid(ny, nx)
    img = np.zeros((ny, nx))
    for _ in range(10):
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        sb = rng.uniform(2, 8) * ny / 64.0
        amp = rng.uniform(0.3, 1.0)
        img += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sb * sb))
    for _ in range(5):
        h, w = rng.uniform(4, 16, size=2) * ny / 64.0
        y0, x0 = rng.uniform(0, ny - h), rng.uniform(0, nx - w)
        val = rng.uniform(0.3, 1.0)
        img[(yy >= y0) & (yy < y0 + h) & (xx >= x0) & (xx < x0 + w)] += val
    return np.clip(img, 0.0, 1.0)


def _ellipse_mask(yy, xx, cy, cx, ay, ax, theta):
    c, s = np.cos(theta), np.sin(theta)
    dy, dx = yy - cy, xx - cx
    u = (dx * c + dy * s) / ax
    v = (-dx * s + dy * c) / ay
    return u * u + v * v <= 1.0


def phantom_piecewise(ny: int, nx: int, rng: np.random.Generator) -> np.ndarray:
    """Smooth background (3 broad Gaussians) + 8 ellipses + 4 rectangles, in [0, 1]."""
    yy, xx = _grid(ny, nx)
    img = np.zeros((ny, nx))
    for _ in range(3):
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        sb = rng.uniform(0.2, 0.4) * ny
        img += rng.uniform(0.1, 0.3) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sb * sb))
    for _ in range(8):
        cy, cx = rng.uniform(0.15, 0.85) * ny, rng.uniform(0.15, 0.85) * nx
        ay, ax = rng.uniform(0.03, 0.15, size=2) * ny
        img[_ellipse_mask(yy, xx, cy, cx, ay, ax, rng.uniform(0, np.pi))] = rng.uniform(0.3, 1.0)
    for _ in range(4):
        h, w = rng.uniform(0.03, 0.12, size=2) * ny
        y0, x0 = rng.uniform(0, ny - h), rng.uniform(0, nx - w)
        img[(yy >= y0) & (yy < y0 + h) & (xx >= x0) & (xx < x0 + w)] = rng.uniform(0.3, 1.0)
    return np.clip(img, 0.0, 1.0)


def phantom_ellipses(n: int, rng: np.random.Generator) -> np.ndarray:
    """Generated head-like phantom: outer ellipse 1, inner ellipse 0.8, 8 small
    ellipses of value +-U[0.1, 0.3]; clipped at 0.  (Seeded, not a classical table.)"""
    yy, xx = _grid(n, n)
    c = (n - 1) / 2.0
    img = np.zeros((n, n))
    img[_ellipse_mask(yy, xx, c, c, 0.46 * n, 0.36 * n, 0.0)] = 1.0
    img[_ellipse_mask(yy, xx, c + 0.01 * n, c, 0.43 * n, 0.33 * n, 0.0)] = 0.8
    for _ in range(8):
        cy = c + rng.uniform(-0.3, 0.3) * n
        cx = c + rng.uniform(-0.22, 0.22) * n
        ay, ax = rng.uniform(0.02, 0.09, size=2) * n
        val = rng.choice([-1.0, 1.0]) * rng.uniform(0.1, 0.3)
        img[_ellipse_mask(yy, xx, cy, cx, ay, ax, rng.uniform(0, np.pi))] += val
    return np.clip(img, 0.0, None)


# --------------------------------------------------------------------------
# tomography: parallel-beam Joseph projector
# --------------------------------------------------------------------------
def joseph_parallel_csr(N: int, n_angles: int, n_bins: int, dtype=np.float32):
    """Parallel-beam projection matrix of an N x N image (unit pixels, image
    centred at the origin) as CSR (rowptr int64, col int32, val dtype).

    Angles theta_a = a * 180 / n_angles degrees; detector bins centred at
    t_b = b - (n_bins - 1) / 2; row index = a * n_bins + b; column index =
    row-major pixel index.  Joseph's method: march along the axis the ray is
    most aligned with, interpolate linearly between the two nearest pixel
    centres on the other axis, and weight by the path length per step
    1 / max(|cos|, |sin|).
    """
    import scipy.sparse as sp

    c = (N - 1) / 2.0
    rows, cols, vals = [], [], []
    t = np.arange(n_bins, dtype=np.float64) - (n_bins - 1) / 2.0
    for a in range(n_angles):
        th = np.deg2rad(a * 180.0 / n_angles)
        ct, st = np.cos(th), np.sin(th)
        # ray: points p with p . (ct, st) = t, direction (-st, ct)
        row0 = a * n_bins
        if abs(st) >= abs(ct):
            # march over pixel columns x_j; y from x*ct + y*st = t
            xs = np.arange(N, dtype=np.float64) - c
            y = (t[:, None] - xs[None, :] * ct) / st          # (bins, N)
            w = 1.0 / abs(st)
            fy = y + c
            i0 = np.floor(fy).astype(np.int64)
            frac = fy - i0
            for off, wt in ((0, 1.0 - frac), (1, frac)):
                ii = i0 + off
                jj = np.broadcast_to(np.arange(N), ii.shape)
                ok = (ii >= 0) & (ii < N) & (wt > 0)
                rr = np.broadcast_to(row0 + np.arange(n_bins)[:, None], ii.shape)
                rows.append(rr[ok]); cols.append(ii[ok] * N + jj[ok]); vals.append(wt[ok] * w)
        else:
            ys = np.arange(N, dtype=np.float64) - c
            x = (t[:, None] - ys[None, :] * st) / ct
            w = 1.0 / abs(ct)
            fx = x + c
            j0 = np.floor(fx).astype(np.int64)
            frac = fx - j0
            for off, wt in ((0, 1.0 - frac), (1, frac)):
                jj = j0 + off
                ii = np.broadcast_to(np.arange(N), jj.shape)
                ok = (jj >= 0) & (jj < N) & (wt > 0)
                rr = np.broadcast_to(row0 + np.arange(n_bins)[:, None], jj.shape)
                rows.append(rr[ok]); cols.append(ii[ok] * N + jj[ok]); vals.append(wt[ok] * w)
    r = np.concatenate(rows); cidx = np.concatenate(cols); v = np.concatenate(vals)
    m = n_angles * n_bins
    A = sp.csr_matrix((v, (r, cidx)), shape=(m, N * N))
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(dtype), m, N * N)


# --------------------------------------------------------------------------
# forward model for synthesising b (library routines only)
# --------------------------------------------------------------------------
def blur_apply_scipy(img: np.ndarray, taps_y: np.ndarray, taps_x: np.ndarray, bc: int, psf=None) -> np.ndarray:
    from scipy import ndimage
    if psf is None:
        psf = np.outer(taps_y, taps_x)
    mode = "constant" if bc == BC_ZERO else "reflect"
    return ndimage.correlate(img, psf, mode=mode, cval=0.0)


def add_noise(clean: np.ndarray, eta: float, rng: np.random.Generator) -> np.ndarray:
    """b = clean + e, e = eta * ||clean|| * eps / ||eps||, eps ~ N(0, I)."""
    eps = rng.standard_normal(clean.shape)
    return clean + eta * np.linalg.norm(clean) * eps / np.linalg.norm(eps)


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    name: str
    kind: str                     # "blur" or "csr"
    m: int
    n: int
    b: np.ndarray                 # float64, length m
    x_true: np.ndarray            # float64, length n
    k: int
    s: int
    lam: float
    sketch: int
    zeta: int
    seed: int
    dtype: str                    # storage of the operator, b and x: "f64" or "f32"
    # blur operator
    ny: int = 0
    nx: int = 0
    taps_y: Optional[np.ndarray] = None
    taps_x: Optional[np.ndarray] = None
    radius: int = 0
    bc: int = BC_ZERO
    # csr operator
    rowptr: Optional[np.ndarray] = None
    col: Optional[np.ndarray] = None
    val: Optional[np.ndarray] = None
    psf: Optional[np.ndarray] = None   # general (2r+1) x (2r+1) PSF (None: taps_y x taps_x)
    basis: str = ""               # storage of the Krylov bases ("" = same as dtype)
    pivot_sample: int = 0         # 0: full partial pivoting; m > 0: pivot from a sample of m rows

    @property
    def basis_dtype(self) -> str:
        return self.basis or self.dtype

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def blur_problem(name, ny, nx, sigma, radius, bc, phantom, eta, k, s, lam, sketch,
                 zeta=8, dtype="f64", cfg_id=0, phantom_seed=PHANTOM_SEED,
                 noise_seed=NOISE_SEED, psf=None) -> Problem:
    """A deblurring problem: a seeded phantom blurred by the Gaussian PSF of
    `sigma` (or by the general `psf`, a (2r+1) x (2r+1) array) plus noise."""
    rng = np.random.default_rng(phantom_seed)
    if phantom == "blobs":
        x = phantom_blobs(ny, nx, rng)
    elif phantom == "piecewise":
        x = phantom_piecewise(ny, nx, rng)
    elif phantom == "random":
        x = rng.uniform(0.0, 1.0, size=(ny, nx))
    else:
        raise ValueError(phantom)
    taps = gaussian_taps(sigma, radius) if sigma else None
    if psf is not None:
        psf = np.ascontiguousarray(psf, dtype=np.float64)
        assert psf.shape == (2 * radius + 1, 2 * radius + 1)
    clean = blur_apply_scipy(x, taps, taps, bc, psf=psf)
    b = add_noise(clean, eta, np.random.default_rng(noise_seed))
    return Problem(name=name, kind="blur", m=ny * nx, n=ny * nx, b=b.ravel().copy(),
                   x_true=x.ravel().copy(), k=k, s=s, lam=lam, sketch=sketch, zeta=zeta,
                   seed=SKETCH_SEED_BASE + cfg_id, dtype=dtype, ny=ny, nx=nx,
                   taps_y=taps, taps_x=None if taps is None else taps.copy(), radius=radius, bc=bc,
                   psf=psf)


def blur_rhs_family(P: Problem, nr: int, eta: float = 0.02) -> list:
    """nr deblurring problems on P's (separable) blur operator: P itself,
    then piecewise-smooth phantoms and noise drawn from seeds 17 r past P's,
    blurred by the same operator (several right-hand sides of one operator)."""
    out = [P]
    for r in range(1, nr):
        rng = np.random.default_rng(PHANTOM_SEED + 17 * r)
        x = phantom_piecewise(P.ny, P.nx, rng)
        clean = blur_apply_scipy(x, P.taps_y, P.taps_x, P.bc, psf=P.psf)
        b = add_noise(clean, eta, np.random.default_rng(NOISE_SEED + 17 * r)).ravel()
        out.append(P.replace(b=b, x_true=x.ravel().copy()))
    return out


def csr_problem(name, N, n_angles, n_bins, eta, k, s, lam, sketch, zeta=8, dtype="f32",
                cfg_id=0, phantom_seed=PHANTOM_SEED, noise_seed=NOISE_SEED) -> Problem:
    import scipy.sparse as sp
    rowptr, col, val, m, n = joseph_parallel_csr(N, n_angles, n_bins,
                                                 dtype=np.float32 if dtype == "f32" else np.float64)
    x = phantom_ellipses(N, np.random.default_rng(phantom_seed)).ravel()
    A = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(m, n))
    clean = A @ x
    b = add_noise(clean, eta, np.random.default_rng(noise_seed))
    return Problem(name=name, kind="csr", m=m, n=n, b=b, x_true=x, k=k, s=s, lam=lam,
                   sketch=sketch, zeta=zeta, seed=SKETCH_SEED_BASE + cfg_id, dtype=dtype,
                   rowptr=rowptr, col=col, val=val)


def dense_problem(name, A: np.ndarray, b: np.ndarray, k, s, lam=0.0, sketch=SKETCH_GAUSSIAN,
                  zeta=2, dtype="f64", seed=SKETCH_SEED_BASE) -> Problem:
    """Wrap a small dense matrix as a CSR problem (test helper)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(m):
        nz = np.nonzero(A[i])[0]
        cols.append(nz.astype(np.int32)); vals.append(A[i, nz])
        rowptr[i + 1] = rowptr[i] + len(nz)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return Problem(name=name, kind="csr", m=m, n=n, b=np.asarray(b, np.float64).copy(),
                   x_true=np.zeros(n), k=k, s=s, lam=lam, sketch=sketch, zeta=zeta, seed=seed,
                   dtype=dtype, rowptr=rowptr, col=col.astype(np.int32),
                   val=val.astype(np.float64 if dtype == "f64" else np.float32))


# The workloads.  c1 / c1_tik: 64x64 deblurring in FP64 (lambda 0 and 1e-3).
# c2: 512x512 deblurring with FP32 operator and bases and a sparse-sign
# sketch (the throughput workload).  c3: 256x256 parallel-beam tomography,
# rectangular, FP32 matrix; its bases are kept in FP64 because with lambda = 0
# and k = 150 the solution is too sensitive to FP32 rounding of the basis.
# c4_bf16 / c4_f16: c2 with bfloat16 / binary16 bases.
def config(name: str) -> Problem:
    if name in ("c1", "c1_tik"):
        lam = 0.0 if name == "c1" else 1e-3
        return blur_problem(name, 64, 64, 2.0, 7, BC_ZERO, "blobs", 0.01, k=50, s=102, lam=lam,
                            sketch=SKETCH_GAUSSIAN, dtype="f64", cfg_id=1)
    if name == "c2":
        return blur_problem(name, 512, 512, 4.0, 15, BC_REFLECT, "piecewise", 0.02, k=100, s=400,
                            lam=1e-2, sketch=SKETCH_SPARSE_SIGN, zeta=8, dtype="f32", cfg_id=2)
    if name in ("c4_bf16", "c4_f16"):
        # the reduced-precision storage tier on the 512x512 deblurring
        # workload: same operator and data, 16-bit Krylov bases
        return config("c2").replace(name=name, basis=name[3:])
    if name == "c3":
        return csr_problem(name, 256, 180, 362, 0.01, k=150, s=302, lam=0.0,
                           sketch=SKETCH_GAUSSIAN, dtype="f32", cfg_id=3).replace(basis="f64")
    if name == "c3_f32basis":
        return csr_problem("c3", 256, 180, 362, 0.01, k=150, s=302, lam=0.0,
                           sketch=SKETCH_GAUSSIAN, dtype="f32", cfg_id=3)
    raise KeyError(name)


CONFIG_NAMES = ("c1", "c1_tik", "c2", "c3")


# --------------------------------------------------------------------------
# serving mix
# --------------------------------------------------------------------------
SERVE_SEED = 0x5E7E
# deblurring sizes the single-kernel tile plan accepts (n <= 256 tiles x 2048
# pixels); the 1024 x 1024 images of the original mix exceed it
SERVE_BLUR_SIZES = (128, 256, 384, 512)
SERVE_TOMO_SIZES = (64, 128, 256)
SERVE_TOMO_ANGLES = (60, 90, 120, 180)


def serving_requests(n: int = 512, rate: float = 200.0, seed: int = SERVE_SEED):
    """The serving mix: n requests with Poisson arrivals (exponential gaps of
    mean 1/rate seconds), half deblurring (sizes SERVE_BLUR_SIZES, sigma
    U[1, 6], r = round(4 sigma) - 1, boundary zero or reflective, sparse-sign
    sketch with 8 nonzeros) and half tomography (SERVE_TOMO_SIZES x
    SERVE_TOMO_ANGLES parallel-beam operators, Gaussian sketch); k uniform in
    20..200, s = 2(k + 1), lambda in {0, 1e-3, 1e-2}.  Returns a list of
    dicts with the arrival time (seconds from the first) and the request."""
    rng = np.random.default_rng(seed)
    t = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0 / rate, size=n - 1))])
    out = []
    for i in range(n):
        k = int(rng.integers(20, 201))
        lam = float(rng.choice([0.0, 1e-3, 1e-2]))
        req = {"arrival": float(t[i]), "k": k, "s": 2 * (k + 1), "lam": lam, "id": i}
        if rng.random() < 0.5:
            N = int(rng.choice(SERVE_BLUR_SIZES))
            sigma = float(rng.uniform(1.0, 6.0))
            req.update(kind="blur", N=N, sigma=sigma, r=radius_for_sigma(sigma),
                       bc=int(rng.integers(0, 2)), sketch=SKETCH_SPARSE_SIGN, zeta=8)
        else:
            req.update(kind="csr", N=int(rng.choice(SERVE_TOMO_SIZES)),
                       angles=int(rng.choice(SERVE_TOMO_ANGLES)), sketch=SKETCH_GAUSSIAN, zeta=8)
        req["seed"] = SKETCH_SEED_BASE + 5000 + i
        out.append(req)
    return out


def serving_data(req, phantom_seed: int = PHANTOM_SEED, noise_seed: int = NOISE_SEED):
    """b (float64) of a serving request: a seeded phantom through the request's
    operator plus 1% noise, applied with SciPy (blur) or a sparse product."""
    rng = np.random.default_rng(phantom_seed + req["id"])
    if req["kind"] == "blur":
        N = req["N"]
        x = phantom_piecewise(N, N, rng)
        taps = gaussian_taps(req["sigma"], req["r"])
        clean = blur_apply_scipy(x, taps, taps, req["bc"]).ravel()
    else:
        raise ValueError("tomography data needs its operator: use serving_tomo_data")
    return add_noise(clean, 0.01, np.random.default_rng(noise_seed + req["id"]))


def serving_tomo_data(req, A, phantom_seed: int = PHANTOM_SEED, noise_seed: int = NOISE_SEED):
    x = phantom_ellipses(req["N"], np.random.default_rng(phantom_seed + req["id"])).ravel()
    return add_noise(A @ x, 0.01, np.random.default_rng(noise_seed + req["id"]))
