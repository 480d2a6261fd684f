"""Write the rounding-sensitivity fixture of the 256 x 256 tomography
workload (180 angles x 362 bins, k = 150, s = 302, lambda = 0) from the
oracle alone.

The oracle is solved on b and on copies of b with random one-ulp
perturbations.  The spread between those FP64 solves is how much of the
result the FP64 arithmetic itself does not determine for this workload: the
generalized Hessenberg process with partial pivoting (Sec. 3.1; the sLSLU
iteration of Algorithm 1) is stable in practice but not backward stable, and on this
operator small differences in the basis grow from step to step.  Recorded per
perturbation: the first step where the pivot sequences t / g differ, the
near-tie gap 1 - |d(t')| (resp. |l(g')|) of the unperturbed vector at the
perturbed pivot, the largest column-relative drift of H, Z, D and L before
that step, and the relative change of x.

Run:  python tests/golden/make_sensitivity.py   (about a minute on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

ULP = 2.0 ** -52


def colrel(A, B):
    if A.size == 0:
        return 0.0
    nb = np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    return float(np.max(np.linalg.norm(A - B, axis=0) / nb))


def first_mismatch(a, b):
    for i in range(min(len(a), len(b))):
        if a[i] != b[i]:
            return i
    return None


def main(name="c3", seeds=4):
    P = W.config(name)
    t = np.float32 if P.dtype == "f32" else np.float64
    Pr = P.replace(b=P.b.astype(t).astype(np.float64), val=P.val.astype(t))
    o = oracle.solve(Pr, keep_basis=True)
    runs = []
    for seed in range(seeds):
        rng = np.random.default_rng(1000 + seed)
        flip = rng.random(Pr.b.size) < 0.5
        sgn = rng.choice([-1.0, 1.0], size=Pr.b.size)
        q = oracle.solve(Pr.replace(b=Pr.b * (1.0 + ULP * sgn * flip)), keep_basis=True)
        it = first_mismatch(list(q["t"]), list(o["t"]))
        ig = first_mismatch(list(q["g"]), list(o["g"]))
        near_t = None if it is None else float(1.0 - abs(o["Dmat"][q["t"][it], it]))
        near_g = None if ig is None else float(1.0 - abs(o["Lmat"][q["g"][ig], ig]))
        a = min([v for v in (it, ig) if v is not None] or [o["k_done"]])
        runs.append({
            "seed": 1000 + seed,
            "first_t_mismatch": it, "near_t": near_t,
            "first_g_mismatch": ig, "near_g": near_g,
            "H_drift": colrel(q["H"][: a, : a - 1], o["H"][: a, : a - 1]),
            "Z_drift": colrel(q["Z"][:, :a], o["Z"][:, :a]),
            "D_drift": colrel(q["Dmat"][:, :a], o["Dmat"][:, :a]),
            "L_drift": colrel(q["Lmat"][:, :a], o["Lmat"][:, :a]),
            "x_drift": float(np.linalg.norm(q["x"] - o["x"]) / np.linalg.norm(o["x"])),
        })
        print(runs[-1], flush=True)
    out = {"workload": P.name, "perturbation": "b * (1 + u), u = +-2^-52 on a random half of the entries",
           "runs": runs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_sensitivity.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(*sys.argv[1:2])
