"""Benchmark: Hessenberg iterations per second of the sketched inner-product
free Krylov solver on the 512 x 512 deblurring workload, on one MI355X.

Workload (one "step" = one whole solve): 512 x 512 image (n = m = 262144),
separable Gaussian blur sigma = 4 px, 31 x 31 stencil, reflective boundary,
seeded piecewise-smooth phantom with 2% noise, k = 100 Hessenberg steps,
sparse-sign sketch s = 400 with 8 nonzeros per column, Tikhonov lambda = 1e-2.
FP32 storage of the operator input, b, x and the Krylov basis; FP64
arithmetic.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `roofline` is for the dominant kernel (the persistent
basis-iteration kernel): algorithmic bytes per launch (sum over steps j of
(j + 1) basis vectors of n FP32 values: read L_j, write l_{j+1}) over its
average launch duration from HIP events recorded on its stream during the
timed region.  `cpu_baseline` times the CPU oracle on the same workload.
"""
from __future__ import annotations

import argparse
import json
import subprocess
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2502_02721_amd", "csrc")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "blur_iterate_kernel_deblur512_pmc.md")


# the sources that define, plan and launch the basis kernel of the bench line
KERNEL_SOURCES = ("hk_blur.hpp", "hk_device.hpp", "hk_internal.hpp", "hk_iter_f32.hip", "hk_kernels.hip",
                  "hk_runtime.cpp")


def csrc_digest() -> str:
    """SHA-256 over the basis kernel's sources (names and contents, in order)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the iteration kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the
    copy-kernel calibration), or None when the summary was taken on other
    kernel sources than the ones here."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            kv = dict(line.split(":", 1) for line in f if line.startswith(("csrc_sha256:", "traffic_bytes_per_launch:")))
    except OSError:
        return None
    if kv.get("csrc_sha256", "").strip() != csrc_digest():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def calibrate_copy(nbytes: int, reps: int):
    """A plain device copy of known size (read nbytes, write nbytes) for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").uniform_()
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy": {"bytes_read": nbytes, "bytes_written": nbytes, "launches": reps,
                                         "kernel": "torch elementwise mul by 1.0 (float32)"}}), flush=True)


def algorithmic_bytes(n: int, k: int, w: int) -> int:
    # step j (1..k) reads the j basis vectors l_1..l_j (l_j is also the operator
    # input) and writes l_{j+1}: (j + 1) n w bytes.
    return sum((j + 1) * n * w for j in range(1, k + 1))


def algorithmic_bytes_csr(P, k: int, w: int) -> int:
    # rectangular process, step j (1..k): u = A l_j and q = A^T d_{j+1} each
    # stream the operator's column indices (int32) and values once; the two
    # eliminations read d_1..d_j and l_1..l_j (l_j is also the input of A) and
    # write d_{j+1} and l_{j+1}: (j + 1)(m + n) w bytes.  Row pointers are
    # staged in LDS once per solve and not counted.
    vb = 4 if P.dtype == "f32" else 8
    nnz = int(P.rowptr[-1])
    return sum(2 * nnz * (4 + vb) + (j + 1) * (P.m + P.n) * w for j in range(1, k + 1))


def csr_line(hk, ctx, steps: int, warmup: int):
    """The CSR tomography workload (256x256 image, 180 angles x 362 bins,
    k = 150, Gaussian s = 302, FP32 operator and data, FP64 bases): its solve
    time and the generic kernel's algorithmic bandwidth."""
    import torch
    import workloads as W
    P = W.config("c3")
    op = hk.Operator.csr(ctx, P.m, P.n, P.rowptr, P.col, P.val.astype(np.float32), hk.HK_F32)
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=hk.HK_F64)
    b = torch.tensor(P.b.astype(np.float32), device="cuda:0")
    x = torch.empty(P.n, dtype=torch.float32, device="cuda:0")
    for _ in range(warmup):
        sv.run(b, x)
    sv.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sv.run(b, x)
    st = sv.wait()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kd = sv.k_done()
    it_ms, tot_ms = sv.timing_history(steps)
    alg = algorithmic_bytes_csr(P, kd, 8)
    iter_avg = float(np.mean(it_ms))
    achieved = alg / (iter_avg * 1e-3) / 1e9
    sv.close()
    op.close()
    print(f"# csr tomography: {wall * 1e3 / steps:.3f} ms per solve", file=sys.stderr, flush=True)
    return {"workload": f"tomography 256x256, 180 angles x 362 bins (m={P.m}, n={P.n}, nnz={int(P.rowptr[-1])}), "
                        "k=150, Gaussian s=302, lambda=0, FP32 operator, FP64 bases",
            "status": st, "k": kd, "ms_per_solve": round(wall * 1e3 / steps, 4),
            "hessenberg_iters_per_s": round(kd * steps / wall, 1),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(achieved / PEAK_HBM_GBS, 4), "kernel": "iterate_kernel (generic, CSR)",
                         "alg_bytes_per_launch": alg, "avg_launch_ms": round(iter_avg, 4)}}


def cpu_baseline(P, max_seconds: float = 30.0):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    Pr = P.replace(b=P.b.astype(np.float32).astype(np.float64))
    t0 = time.perf_counter()
    o = oracle.solve(Pr)
    dt = time.perf_counter() - t0
    return {"value": o["k_done"] / dt, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": f"one full solve of the same workload (k={o['k_done']}) in {dt:.2f} s, "
                      "FP64, OpenMP over the operator loops"}


def serving(hk, ctx, n: int, rate: float, slots: int):
    """The serving mix (workloads.serving_requests): n requests with Poisson
    arrivals at `rate` per second, submitted to an hk Server as they arrive;
    latency is the library's submit-to-observed-completion time."""
    import torch
    import scipy.sparse as sp
    import workloads as W

    reqs = W.serving_requests(n, rate)
    tomo = {}
    ops, bs, xs = [], [], []
    for q in reqs:
        if q["kind"] == "csr":
            key = (q["N"], q["angles"])
            if key not in tomo:
                N, na = key
                rp, ci, cv, m, nn = W.joseph_parallel_csr(N, na, int(np.ceil(N * np.sqrt(2.0))) + 2)
                A = sp.csr_matrix((cv.astype(np.float64), ci, rp), shape=(m, nn))
                tomo[key] = (hk.Operator.csr(ctx, m, nn, rp, ci, cv, hk.HK_F32), A)
            op, A = tomo[key]
            b = W.serving_tomo_data(q, A)
        else:
            op = hk.Operator.gaussian_blur(ctx, q["N"], q["N"], q["sigma"], q["r"], q["bc"], hk.HK_F32)
            b = W.serving_data(q)
        ops.append(op)
        bs.append(torch.tensor(b.astype(np.float32), device="cuda:0"))
        xs.append(torch.empty(op.n, dtype=torch.float32, device="cuda:0"))
    torch.cuda.synchronize()
    srv = hk.Server(ctx, slots=slots)
    # load every kernel variant once, outside the measured run
    for q in (next(r for r in reqs if r["kind"] == "blur"), next(r for r in reqs if r["kind"] == "csr")):
        i = q["id"]
        srv.wait(srv.submit(ops[i], bs[i], xs[i], 20, 42, q["lam"], q["sketch"], q["zeta"], q["seed"]))
    print(f"# serving: {n} requests set up, running", file=sys.stderr, flush=True)
    base = srv.poll()
    tickets = []
    t0 = time.perf_counter()
    i = 0
    while i < n or srv.poll() < base + n:
        now = time.perf_counter() - t0
        while i < n and reqs[i]["arrival"] <= now:
            q = reqs[i]
            tickets.append(srv.submit(ops[i], bs[i], xs[i], q["k"], q["s"], q["lam"], q["sketch"], q["zeta"],
                                      q["seed"]))
            i += 1
        time.sleep(2e-5)
    res = [srv.result(t) for t in tickets]
    srv.close()
    # the mix's results: the first request of every (kind, size) bucket,
    # solved alone with the grid it had in the mix, gives the same x bit for bit
    checked, differ, seen = 0, 0, set()
    for q, r in zip(reqs, res):
        key = (q["kind"], q["N"])
        if key in seen or r["status"] < 0:
            continue
        seen.add(key)
        i = q["id"]
        sv = hk.Solve(ops[i], q["k"], q["s"], q["lam"], q["sketch"], q["zeta"], q["seed"],
                      max_workgroups=r["workgroups"])
        xa = sv.run(bs[i])
        sv.wait()
        checked += 1
        differ += 0 if torch.equal(xa, xs[i]) else 1
        sv.close()
    bad = [r["status"] for r in res if r["status"] < 0]
    lat = np.array([r["t_finish"] - r["t_submit"] for r in res]) * 1e3
    span = max(r["t_finish"] for r in res) - min(r["t_submit"] for r in res)
    iters = sum(r["k_done"] for r in res)
    # requests running at once, sampled at each admission
    starts = sorted(r["t_start"] for r in res)
    conc = max(sum(1 for r in res if r["t_start"] <= t < r["t_finish"]) for t in starts)
    return {"requests": n, "arrival_rate_req_s": rate, "slots": slots, "solves_per_s": round(n / span, 2),
            "hessenberg_iters_per_s": round(iters / span, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "mean": round(float(lat.mean()), 3)},
            "max_concurrent": int(conc), "errors": len(bad),
            "checked_against_alone": {"requests": checked, "differ": differ,
                                      "rule": "first request of each (kind, size) bucket, same grid, x bit for bit"},
            "mix": "deblur 128-512 px (sigma 1-6, zero/reflective, sparse sign), tomography 64-256 px "
                   "(60-180 angles, Gaussian), k 20-200, s = 2(k+1), lambda in {0, 1e-3, 1e-2}, FP32; "
                   "1024 px deblurring exceeds the single-kernel tile plan and is left out"}


def serving_child(args):
    """The serving mix in a child process whose HIP runtime uses
    args.serve_hw_queues hardware queues (read once, when HIP starts): with
    HIP's default of 4, the server's slot streams share few queues and
    their solves serialise.  Progress lines go to this process's stderr."""
    env = dict(os.environ)
    env["GPU_MAX_HW_QUEUES"] = str(args.serve_hw_queues)
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only",
           "--serve-requests", str(args.serve_requests), "--serve-rate", str(args.serve_rate),
           "--serve-slots", str(args.serve_slots), "--serve-hw-queues", str(args.serve_hw_queues)]
    r = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"serving run failed with exit status {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def multi_rhs(hk, ctx, nrhs: int, steps: int, warmup: int, only: bool = False, sparse: bool = False):
    """Several right-hand sides on the 512 x 512 deblurring operator solved
    together (hk_params.nrhs): the workload's operator and settings, with
    its own sparse-sign sketch (sparse) or a Gaussian sketch of s = 400
    (whose block contraction covers all the bases); right-hand sides from
    workloads.blur_rhs_family.  Reports Hessenberg iterations per second
    summed over the right-hand sides and the basis kernel's algorithmic
    bandwidth (nrhs times one solve's bytes)."""
    import torch
    import workloads as W
    P = W.config("c2")
    if not sparse:
        P = P.replace(sketch=W.SKETCH_GAUSSIAN)
    out = {}
    for nr in ([nrhs] if only else sorted({1, nrhs})):
        probs = W.blur_rhs_family(P, nr)
        op = hk.Operator.blur(ctx, P.ny, P.nx, P.taps_y, P.taps_x, P.radius, P.bc, hk.HK_F32)
        sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=hk.HK_F32, nrhs=nr)
        b = torch.tensor(np.stack([Q.b.astype(np.float32) for Q in probs]), device="cuda:0")
        x = torch.empty((nr, P.n), dtype=torch.float32, device="cuda:0")
        for _ in range(warmup):
            sv.run(b, x)
        sv.wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.run(b, x)
        st = sv.wait()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        it_ms, tot_ms = sv.timing_history(steps)
        kd = 0
        for r in range(nr):
            sv.select(r)
            kd += sv.k_done()
        alg = nr * algorithmic_bytes(P.n, P.k, 4)
        iter_avg = float(np.mean(it_ms))
        achieved = alg / (iter_avg * 1e-3) / 1e9
        out[str(nr)] = {"status": st, "ms_per_solve": round(wall * 1e3 / steps, 4),
                        "hessenberg_iters_per_s": round(kd * steps / wall, 1),
                        "basis_kernel_ms": round(iter_avg, 4), "total_ms": round(float(np.mean(tot_ms)), 4),
                        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                                     "alg_bytes_per_launch": alg, "basis_bytes": nr * P.n * (P.k + 1) * 4}}
        sv.close()
        op.close()
        print(f"# multi-rhs {nr}: {out[str(nr)]['ms_per_solve']} ms per solve", file=sys.stderr, flush=True)
    sk = "sparse-sign s=400 zeta=8" if sparse else "Gaussian s=400"
    return {"workload": f"deblur-512x512 operator, k=100, {sk}, lambda=1e-2, FP32 bases; "
                        f"{nrhs} right-hand sides solved together vs one",
            "runs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512, help="serving mix size (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-hw-queues", type=int, default=12,
                    help="hardware queues (GPU_MAX_HW_QUEUES) of the process that runs the serving mix; "
                         "it runs in a child process when this differs from the current setting (0: this process)")
    ap.add_argument("--serving-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--workload", default="c2", help=argparse.SUPPRESS)
    ap.add_argument("--no-csr", dest="csr", action="store_false", help="skip the CSR tomography line")
    ap.add_argument("--rhs", type=int, default=4, help="right-hand sides of the multi-right-hand-side line (0: skip)")
    ap.add_argument("--rhs-only", action="store_true",
                    help="run only the multi-right-hand-side line (--rhs right-hand sides, no single-solve line)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="run only a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, 3)
        return

    import torch
    import workloads as W
    import paper_2502_02721_amd as hk

    if args.serving_only:
        ctx = hk.Context(0)
        res = serving(hk, ctx, args.serve_requests, args.serve_rate, args.serve_slots)
        res["hw_queues"] = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        print(json.dumps(res), flush=True)
        return
    if args.rhs_only:
        ctx = hk.Context(0)
        print(json.dumps({"multi_rhs": multi_rhs(hk, ctx, max(1, args.rhs), args.steps, args.warmup, only=True)}),
              flush=True)
        return
    P = W.config(args.workload)
    tdt = np.float32 if P.dtype == "f32" else np.float64
    bdt = {"f64": hk.HK_F64, "f32": hk.HK_F32, "bf16": hk.HK_BF16, "f16": hk.HK_F16}[P.basis_dtype]
    ctx = hk.Context(0)
    dt = hk.HK_F32 if P.dtype == "f32" else hk.HK_F64
    if P.kind == "blur":
        op = hk.Operator.blur(ctx, P.ny, P.nx, P.taps_y, P.taps_x, P.radius, P.bc, dt)
    else:
        op = hk.Operator.csr(ctx, P.m, P.n, P.rowptr, P.col, P.val.astype(tdt), dt)
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, basis_dtype=bdt)
    b = torch.tensor(P.b.astype(tdt), device="cuda:0")
    x = torch.empty(P.n, dtype=b.dtype, device="cuda:0")

    for _ in range(args.warmup):
        sv.run(b, x)
    sv.wait()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} solves)", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    for _ in range(args.steps):
        sv.run(b, x)
    st = sv.wait()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_done = sv.k_done()
    it_ms, tot_ms = sv.timing_history(args.steps)
    print(f"# timed {args.steps} solves in {wall:.4f} s, status {st}", file=sys.stderr, flush=True)

    w = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[P.basis_dtype]
    ms_per_step = wall * 1e3 / args.steps
    iters = k_done * args.steps
    value = iters / wall
    alg = algorithmic_bytes(P.n, k_done, w) if P.kind == "blur" else algorithmic_bytes_csr(P, k_done, w)
    iter_avg = float(np.mean(it_ms))
    roof = None
    if alg is not None:
        achieved = alg / (iter_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic() if args.workload == "c2" else None,
                "kernel": ("blur_iterate_kernel (persistent basis iteration)" if P.kind == "blur"
                           else "iterate_kernel (generic, CSR)"),
                "alg_bytes_per_launch": alg, "avg_launch_ms": round(iter_avg, 4)}
    out = {
        "metric": "Hessenberg iters/s + HBM GB/s at 512² deblur; solves/s with p50/p99 latency",
        "value": round(value, 1),
        "unit": "Hessenberg iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "deblur-512x512 (n=262144), Gaussian blur sigma=4 31x31 reflective, "
                               "k=100, sparse-sign s=400 zeta=8, lambda=1e-2",
                   "storage": P.basis_dtype, "arithmetic": "f64", "k": k_done, "s": P.s,
                   "parallelism": "single GPU, one persistent workgroup per tile"},
        "solves_per_s": round(args.steps / wall, 2),
        "hbm_gbs": round(alg / (ms_per_step * 1e-3) / 1e9, 1) if alg else None,
        "latency_ms": {"p50": round(float(np.percentile(tot_ms, 50)), 4),
                       "p99": round(float(np.percentile(tot_ms, 99)), 4)},
        "roofline": roof,
    }
    if args.csr and args.workload == "c2":
        out["csr_tomography"] = csr_line(hk, ctx, 5, 2)
    if args.rhs > 0:
        out["multi_rhs"] = multi_rhs(hk, ctx, args.rhs, max(3, args.steps // 2), 2)
        # the workload's own sketch: three right-hand sides fit its LDS plan
        out["multi_rhs_sparse"] = multi_rhs(hk, ctx, 3, max(3, args.steps // 2), 2, sparse=True)
    if args.serve_requests > 0:
        if args.serve_hw_queues > 0 and os.environ.get("GPU_MAX_HW_QUEUES") != str(args.serve_hw_queues):
            out["serving"] = serving_child(args)
        else:
            out["serving"] = serving(hk, ctx, args.serve_requests, args.serve_rate, args.serve_slots)
            out["serving"]["hw_queues"] = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
