"""GPU tests of the serving loop (hk_server_*): continuous batching of solves
of different operators, sizes and iteration counts on one device.

 - every result in a mix of requests that run side by side is bit-identical
   to the same request solved alone with the same grid (the kernels are
   deterministic: fixed tile order, no floating-point atomics);
 - requests really overlap (more than one basis kernel in flight);
 - admission by device-memory footprint: with a budget for one workspace
   the requests run one at a time and all finish; a request larger than the
   budget fails with HK_ENOMEM without blocking the others;
 - the mix's results agree with the oracle at the class bars.
"""
import numpy as np
import pytest

import workloads as W
from hk_gpu import make_operator, random_csr, rel, rounded_problem, storage_np, tiny_blur

pytestmark = pytest.mark.gpu

CAP = 40     # workgroups per request: a share that lets several run at once


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_02721_amd as hk
    hk.lib()
    return hk


@pytest.fixture(scope="module")
def ctx(hk):
    return hk.Context(0)


def _flush(msg):
    print(msg, flush=True)


def mix_problems():
    """Blur and CSR problems of different sizes, precisions, sketches and k."""
    P = []
    for i, (N, dt, sk, k, lam) in enumerate([(64, "f64", W.SKETCH_GAUSSIAN, 30, 0.0),
                                            (96, "f32", W.SKETCH_SPARSE_SIGN, 45, 1e-2),
                                            (128, "f32", W.SKETCH_SPARSE_SIGN, 60, 1e-3),
                                            (80, "f64", W.SKETCH_NONE, 25, 1e-3),
                                            (128, "f64", W.SKETCH_SPARSE_SIGN, 70, 0.0)]):
        P.append(tiny_blur(N, N, 1.5 + 0.5 * i, 5 + i, i % 2, k=k, s=2 * (k + 1), lam=lam, sketch=sk,
                           zeta=5, dtype=dt))
    P.append(random_csr(900, 613, 0.02, k=20, s=44, lam=0.5, sketch=W.SKETCH_SPARSE_SIGN, zeta=3, dtype="f64"))
    P.append(random_csr(700, 700, 0.03, k=35, s=72, dtype="f32"))
    P.append(random_csr(613, 900, 0.02, k=25, s=52, dtype="f64").replace(pivot_sample=25))
    return P * 2          # every problem twice, so that equal requests also overlap


def _tensors(P):
    import torch
    b = torch.tensor(P.b.astype(storage_np(P.dtype)), device="cuda:0")
    x = torch.zeros(P.n, dtype=b.dtype, device="cuda:0")
    return b, x


def _submit(srv, op, P, b, x, cap=CAP):
    return srv.submit(op, b, x, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, pivot_sample=P.pivot_sample,
                      max_workgroups=cap)


def _alone(hk, op, P, b, cap=CAP):
    sv = hk.Solve(op, P.k, P.s, P.lam, P.sketch, P.zeta, P.seed, pivot_sample=P.pivot_sample, max_workgroups=cap)
    x = sv.run(b)
    sv.wait()
    out = x.clone()
    sv.close()
    return out


def _max_concurrent(res):
    return max(sum(1 for r in res if r["t_start"] <= s["t_start"] < r["t_finish"]) for s in res)


def test_mix_equals_alone_and_overlaps(hk, ctx, orc):
    import torch
    probs = mix_problems()
    ops = [make_operator(hk, ctx, P) for P in probs]
    bufs = [_tensors(P) for P in probs]
    srv = hk.Server(ctx, slots=4)
    _flush(f"serving mix of {len(probs)} requests")
    tickets = [_submit(srv, op, P, b, x) for op, P, (b, x) in zip(ops, probs, bufs)]
    for t in tickets:
        srv.wait(t)
    res = [srv.result(t) for t in tickets]
    srv.close()
    conc = _max_concurrent(res)
    _flush(f"  statuses {[r['status'] for r in res]} grids {[r['workgroups'] for r in res]} max concurrent {conc}")
    assert all(r["status"] >= 0 for r in res)
    assert conc >= 2, "no two requests ran side by side"
    for i, (op, P, (b, x)) in enumerate(zip(ops, probs, bufs)):
        xa = _alone(hk, op, P, b)
        assert torch.equal(x, xa), f"request {i} ({P.name}): mix and alone differ by {rel(x.cpu().numpy(), xa.cpu().numpy()):.3e}"
    # every request of the mix agrees with the oracle at its class bar, as a
    # relative 2-norm and elementwise relative to max |x|
    cache = {}
    for i, P in enumerate(probs):
        key = id(P)
        if key not in cache:
            cache[key] = orc.solve(rounded_problem(P), method=None)
        o = cache[key]
        xg = bufs[i][1].cpu().numpy().astype(np.float64)
        err = rel(xg, o["x"])
        emax = float(np.max(np.abs(xg - o["x"])) / max(np.max(np.abs(o["x"])), 1e-300))
        bar = 1e-10 if P.dtype == "f64" else 1e-4
        _flush(f"  request {i} ({P.name}, {P.dtype}) vs oracle {err:.3e} elementwise {emax:.3e}")
        assert err <= bar and emax <= bar
    for op in ops:
        op.close()


def test_request_follows_the_context_stream(hk, ctx):
    # b is produced on the context stream behind a long matrix product; the
    # request is submitted at once, so its solve must wait for that copy
    import torch
    P = tiny_blur(128, 128, 2.0, 7, 1, k=40, s=82, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32")
    op = make_operator(hk, ctx, P)
    src = torch.tensor(P.b.astype(np.float32), device="cuda:0")
    ref = _alone(hk, op, P, src)
    torch.cuda.synchronize()
    srv = hk.Server(ctx, slots=2)
    big = torch.randn(6144, 6144, device="cuda:0")
    b = torch.zeros_like(src)
    x = torch.full((P.n,), float("nan"), device="cuda:0")
    for _ in range(4):
        big = big @ big
        big = big / big.abs().max()
    b.copy_(src)
    t = _submit(srv, op, P, b, x)
    srv.wait(t)
    r = srv.result(t)
    srv.close()
    _flush(f"  status {r['status']}, equal to the solve alone: {bool(torch.equal(x, ref))}")
    assert r["status"] == 0 and torch.equal(x, ref)
    op.close()


def test_admission_by_memory_budget(hk, ctx):
    import torch
    probs = [tiny_blur(96, 96, 2.0, 7, 1, k=40, s=82, lam=1e-2, sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32")
             for _ in range(4)]
    ops = [make_operator(hk, ctx, P) for P in probs]
    bufs = [_tensors(P) for P in probs]
    need = hk.Solve(ops[0], 40, 82, 1e-2, W.SKETCH_SPARSE_SIGN, 5, probs[0].seed, max_workgroups=CAP).workspace_bytes()
    srv = hk.Server(ctx, slots=4, budget_bytes=int(need * 1.5))
    tickets = [_submit(srv, op, P, b, x) for op, P, (b, x) in zip(ops, probs, bufs)]
    # a request that needs more than the whole budget fails without blocking
    big = tiny_blur(256, 256, 2.0, 7, 1, k=120, s=242, lam=0.0, sketch=W.SKETCH_SPARSE_SIGN, zeta=5, dtype="f32")
    bop = make_operator(hk, ctx, big)
    bb, bx = _tensors(big)
    tbig = _submit(srv, bop, big, bb, bx)
    for t in tickets:
        srv.wait(t)
    with pytest.raises(hk.HKError):
        srv.wait(tbig)
    res = [srv.result(t) for t in tickets]
    rbig = srv.result(tbig)
    srv.close()
    _flush(f"  budget {int(need * 1.5)} B: statuses {[r['status'] for r in res]} big {rbig['status']} "
           f"max concurrent {_max_concurrent(res)}")
    assert all(r["status"] == 0 for r in res)
    assert rbig["status"] == hk.HK_ENOMEM
    assert _max_concurrent(res) == 1
    xa = _alone(hk, ops[0], probs[0], bufs[0][0])
    assert all(torch.equal(x, xa) for _, x in bufs)
    for op in ops + [bop]:
        op.close()
