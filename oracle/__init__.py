"""Python access to the FP64 CPU oracle (``oracle.c``) through ctypes.

TEST INFRASTRUCTURE ONLY: the oracle is the reference the GPU library is
checked against.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU library's binding never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK, ORC_BREAKDOWN, ORC_EINVAL, ORC_ENOMEM, ORC_ENUMERIC = 0, 1, -1, -2, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP on the operator loops)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Op(C.Structure):
    _fields_ = [("kind", C.c_int), ("m", C.c_int64), ("n", C.c_int64),
                ("ny", C.c_int64), ("nx", C.c_int64), ("radius", C.c_int32), ("bc", C.c_int32),
                ("taps_y", C.c_void_p), ("taps_x", C.c_void_p), ("psf", C.c_void_p),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("s", C.c_int32), ("lam", C.c_double), ("sketch", C.c_int32),
                ("zeta", C.c_int32), ("seed", C.c_uint64), ("method", C.c_int32),
                ("pivot_sample", C.c_int32)]


class _Out(C.Structure):
    _fields_ = [("x", C.c_void_p), ("H", C.c_void_p), ("W", C.c_void_p), ("t", C.c_void_p),
                ("g", C.c_void_p), ("res", C.c_void_p), ("Lb", C.c_void_p), ("Db", C.c_void_p),
                ("Z", C.c_void_p), ("F", C.c_void_p), ("c", C.c_void_p),
                ("k_done", C.c_int32), ("n_t", C.c_int32), ("n_g", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_gaussian_entry.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_int64]
        L.orc_gaussian_entry.restype = C.c_double
        L.orc_sparse_sign_column.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int, C.c_int64,
                                             C.c_void_p, C.c_void_p]
        L.orc_sketch_dense.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_uint64,
                                       C.c_uint32, C.c_void_p]
        L.orc_blur_pixel.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64]
        L.orc_blur_pixel.restype = C.c_double
        L.orc_op_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_op_apply_t.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_small_ls.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_double,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# --------------------------------------------------------------------------
# generator and sketch
# --------------------------------------------------------------------------
def philox4x32_10(counter, key) -> np.ndarray:
    ctr = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w))


def sketch_dense(kind: int, s: int, m: int, zeta: int, seed: int, stream: int) -> np.ndarray:
    """The embedding S in R^{s x m} as a dense array (stream 2 = S2, stream 1 = S1)."""
    out = np.zeros((s, m), dtype=np.float64)
    st = lib().orc_sketch_dense(kind, s, m, zeta, seed, stream, _ptr(out))
    if st != ORC_OK:
        raise RuntimeError(f"orc_sketch_dense failed: {st}")
    return out


def sparse_sign_column(seed: int, stream: int, s: int, zeta: int, i: int):
    rows = np.zeros(zeta, dtype=np.int64)
    vals = np.zeros(zeta, dtype=np.float64)
    lib().orc_sparse_sign_column(seed, stream, s, zeta, i, _ptr(rows), _ptr(vals))
    return rows, vals


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------
class Operator:
    """Keeps the arrays alive that the C struct points to."""

    def __init__(self, problem):
        P = problem
        self.problem = P
        self._keep = []
        op = _Op()
        op.m, op.n = P.m, P.n
        if P.kind == "blur":
            op.kind = 0
            op.ny, op.nx, op.radius, op.bc = P.ny, P.nx, P.radius, P.bc
            if getattr(P, "psf", None) is not None:
                pf = np.ascontiguousarray(P.psf, dtype=np.float64)
                assert pf.shape == (2 * P.radius + 1, 2 * P.radius + 1)
                self._keep.append(pf)
                op.psf = _ptr(pf)
            else:
                ty = np.ascontiguousarray(P.taps_y, dtype=np.float64)
                tx = np.ascontiguousarray(P.taps_x, dtype=np.float64)
                self._keep += [ty, tx]
                op.taps_y, op.taps_x = _ptr(ty), _ptr(tx)
        else:
            op.kind = 1
            rp = np.ascontiguousarray(P.rowptr, dtype=np.int64)
            cl = np.ascontiguousarray(P.col, dtype=np.int32)
            vl = np.ascontiguousarray(P.val, dtype=np.float64)
            self._keep += [rp, cl, vl]
            op.rowptr, op.col, op.val = _ptr(rp), _ptr(cl), _ptr(vl)
        self.op = op

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.op.m)
        lib().orc_op_apply(C.byref(self.op), _ptr(x), _ptr(y))
        return y

    def apply_t(self, y):
        if self.op.kind != 1:
            raise ValueError("adjoint apply is defined for CSR operators only")
        y = np.ascontiguousarray(y, dtype=np.float64)
        x = np.zeros(self.op.n)
        lib().orc_op_apply_t(C.byref(self.op), _ptr(y), _ptr(x))
        return x

    def blur_pixel(self, img, y, x):
        img = np.ascontiguousarray(img, dtype=np.float64)
        return lib().orc_blur_pixel(C.byref(self.op), _ptr(img), y, x)


# --------------------------------------------------------------------------
# small least squares and solve
# --------------------------------------------------------------------------
def small_ls(Z: np.ndarray, F, lam: float, c: np.ndarray):
    """argmin_y ||c - Z y||^2 + lam^2 ||F y||^2 (Householder QR); returns (y, res)."""
    Z = np.asfortranarray(Z, dtype=np.float64)
    s, k = Z.shape
    Fa = np.asfortranarray(F if F is not None else np.zeros((s, k)), dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    y = np.zeros(k); res = np.zeros(k)
    st = lib().orc_small_ls(s, k, _ptr(Z), _ptr(Fa), float(lam), _ptr(c), _ptr(y), _ptr(res))
    if st != ORC_OK:
        raise RuntimeError(f"orc_small_ls failed: {st}")
    return y, res


def prefix_solution(o: dict, kp: int, lam: float) -> np.ndarray:
    """x after the first kp basis vectors of a finished oracle solve (run with
    keep_basis): the small problem of eq. (sketched_LSLU) /
    eq. (sketched_LSLU_hybrid) restricted to the first kp columns of Z and F,
    solved afresh by the Householder routine above, then x = L_kp y.  The
    Hessenberg process for kp steps is the prefix of the one for k steps, so
    this is the solve that stops after kp steps."""
    if not 1 <= kp <= o["k_done"]:
        raise ValueError(f"prefix length {kp} outside [1, {o['k_done']}]")
    y, _ = small_ls(o["Z"][:, :kp], o["F"][:, :kp], lam, o["c"])
    return o["Lmat"][:, :kp] @ y


def solve(problem, k=None, s=None, lam=None, method=None, keep_basis=False, seed=None):
    """Run sCMRH (square) or sLSLU (rectangular) on a ``workloads.Problem``.

    Returns a dict with x, H, W, t, g, res, k_done, status (and L, D, Z, F, c
    when ``keep_basis``)."""
    P = problem
    k = P.k if k is None else k
    s = P.s if s is None else s
    if P.sketch == 3:                     # no sketch: the small problem has k+1 rows (eq. (TSP))
        s = k + 1
    lam = P.lam if lam is None else lam
    if method is None:                    # square -> sCMRH, rectangular -> sLSLU
        method = 0 if P.m == P.n else 1
    op = Operator(P)
    prm = _Params(k=k, s=s, lam=lam, sketch=P.sketch, zeta=P.zeta,
                  seed=P.seed if seed is None else seed, method=method,
                  pivot_sample=P.pivot_sample)
    m, n = P.m, P.n
    out = {
        "x": np.zeros(n), "H": np.zeros((k + 1, k), order="F"),
        "W": np.zeros((k, k), order="F") if method == 1 else None,
        "t": np.full(k + 1, -1, dtype=np.int64),
        "g": np.full(k, -1, dtype=np.int64) if method == 1 else None,
        "res": np.zeros(k),
    }
    if keep_basis:
        out["L"] = np.zeros((k + 1, n))          # row i = basis vector i (C order = column-major n x (k+1))
        out["D"] = np.zeros((k + 1, m)) if method == 1 else None
        out["Z"] = np.zeros((k, s)); out["F"] = np.zeros((k, s)); out["c"] = np.zeros(s)
    o = _Out()
    o.x, o.H, o.W = _ptr(out["x"]), _ptr(out["H"]), _ptr(out["W"])
    o.t, o.g, o.res = _ptr(out["t"]), _ptr(out["g"]), _ptr(out["res"])
    if keep_basis:
        o.Lb, o.Db = _ptr(out["L"]), _ptr(out["D"])
        o.Z, o.F, o.c = _ptr(out["Z"]), _ptr(out["F"]), _ptr(out["c"])
    st = lib().orc_solve(C.byref(op.op), C.byref(prm), _ptr(np.ascontiguousarray(P.b, np.float64)),
                         C.byref(o))
    if st < 0:
        raise RuntimeError(f"orc_solve failed: {st}")
    out["status"] = st
    out["k_done"] = o.k_done
    out["t"] = out["t"][: o.n_t]
    if out["g"] is not None:
        out["g"] = out["g"][: o.n_g]
    out["res"] = out["res"][: o.k_done]
    out["method"] = method
    if keep_basis:
        out["Z"] = out["Z"].T.copy()      # s x k
        out["F"] = out["F"].T.copy()
        out["Lmat"] = out["L"].T          # n x (k+1)
        if out["D"] is not None:
            out["Dmat"] = out["D"].T
    return out
