"""Serving: continuous batching of hp-DG solves on one GPU.

CPU tests cover the admission policy (memory gate), argument errors of the
batch C ABI that return before any device work, and the device-byte count
of operators that are not on the device. GPU tests check that every result
is bitwise the same alone and in the mix (all reductions have a fixed
order), that admission by memory and by slots holds, the error statuses of
retired solves, and a few results against the oracle's exact solution.
"""
import threading
import time

import numpy as np
import pytest

import hpinputs as H
import paper_2009_01287_amd as G
from paper_2009_01287_amd import serving as S


def small_requests(n=8, seed=5011, dof_lo=300, dof_hi=4000):
    out = []
    for r in H.serving_stream(n, seed=seed, dof_lo=dof_lo, dof_hi=dof_hi):
        md = H.request_mesh(r)
        nd = H.ndof(md)
        out.append(S.Request(id=r["id"], mesh=md, form=r["form"], f=H.gaussian_rhs(nd, r["rhs_seed"]),
                             t_arrive=r["t_arrive"]))
    return out


# ------------------------------------------------------------------ CPU
def test_gate_blocks_until_release():
    g = S.MemoryGate(100)
    assert g.acquire(60)
    got = []

    def w():
        got.append(g.acquire(60))

    t = threading.Thread(target=w)
    t.start()
    time.sleep(0.05)
    assert not got                       # 60 + 60 > 100: waits
    g.release(60)
    t.join(2.0)
    assert got == [True] and g.used == 60 and g.peak == 60
    assert g.acquire(50, timeout=0.01) is False
    g.release(60)
    assert g.used == 0


def test_gate_refuses_oversize_and_close():
    g = S.MemoryGate(10)
    with pytest.raises(MemoryError):
        g.acquire(11)
    assert g.acquire(10)
    res = []

    def w():
        try:
            g.acquire(5)
        except RuntimeError as e:
            res.append(str(e))

    t = threading.Thread(target=w)
    t.start()
    time.sleep(0.02)
    g.close()
    t.join(2.0)
    assert res and "stopped" in res[0]


def test_batch_create_rejects_bad_slots():
    for bad in (0, -1, 65):
        with pytest.raises(G.HpdgError) as e:
            G.Batch(bad)
        assert e.value.code == -1


def test_device_bytes_counting_pass():
    md = H.random_mesh(2, 4, 0.3, 2, 1, 6, seed=77)
    m = G.Mesh(md)
    o64 = G.Operator(m, host_only=True)
    o32 = G.Operator(m, host_only=True, prec_fp32=True)
    b64, b32 = o64.device_bytes(), o32.device_bytes()
    # at least the four FP64 CG vectors; the FP32 preconditioner is smaller
    assert b64 > 32 * m.ndof and b32 < b64
    assert o64.device_bytes() == b64          # deterministic, no state change
    # more right-hand sides: more vector storage
    o4 = G.Operator(m, host_only=True, max_nrhs=4)
    assert o4.device_bytes() > b64
    # still host-only: operator calls are refused without device work
    assert o64.summary()["device_bytes"] == 0
    # fused levels and the dense tail add their matrices to the count
    oa = G.Operator(m, host_only=True, auto_cycle=True)
    assert oa.device_bytes() > b64


def test_summarize():
    rs = [S.Result(id=i, status=0, ndof=10, iters=5, t_arrive=0.0, t_done=1.0 + i, true_rel_res=1e-9)
          for i in range(4)]
    rs.append(S.Result(id=9, status=-5))
    s = S.summarize(rs, wall=2.0)
    assert s["ok"] == 4 and s["solves_per_s"] == 2.0 and s["dofs"] == 40
    assert s["p50_s"] == pytest.approx(2.5)


# ------------------------------------------------------------------ GPU
def alone(req, prec_fp32=True):
    """The blocking solve of a request with the server's operator options."""
    import torch
    m = G.Mesh(req.mesh)
    eta = 1.0 if req.form == "sipg" else 0.0
    op = G.Operator(m, form=req.form, eta=eta, prec_fp32=prec_fp32, max_block=256 if m.dim == 3 else 0,
                    auto_cycle=True)
    f = torch.from_numpy(np.ascontiguousarray(req.f)).cuda()
    b = torch.empty_like(f)
    op.rhs(f, b)
    x = torch.zeros_like(b)
    code, info = op.pcg_solve(b, x, rtol=req.rtol, maxit=req.maxit, raise_on_error=False)
    return code, info[0], x.cpu().numpy()


@pytest.mark.gpu
@pytest.mark.parametrize("graph", [False, True])
def test_mix_equals_alone_bitwise(graph):
    reqs = small_requests(10)
    srv = S.Server(max_active=4, workers=4, realtime=False, keep_x=True, min_batch=len(reqs), graph=graph)
    res = srv.run(reqs)
    assert srv.max_concurrent == 4
    for q, r in zip(reqs, res):
        print(f"request {q.id}: dim {r.dim} {r.form} ndof {r.ndof} iters {r.iters} status {r.status}", flush=True)
        assert r.status == 0, r.error
        code, info, x = alone(q)
        assert code == 0
        assert r.iters == info["iters"]
        assert np.array_equal(r.x, x), f"request {q.id}: result differs alone and in the mix"
        assert r.true_rel_res <= 1e-8


@pytest.mark.gpu
def test_admission_by_memory_and_fp64():
    reqs = small_requests(6, seed=5013)
    big = S.Server(max_active=8, workers=3, realtime=False, keep_x=True, prec_fp32=False)
    r_all = big.run(reqs)
    need = max(r.device_bytes for r in r_all)
    tight = S.Server(max_active=8, workers=3, realtime=False, keep_x=True, prec_fp32=False,
                     mem_budget=need + need // 4)
    r_tight = tight.run(reqs)
    assert tight.gate.peak <= tight.gate.budget
    for a, b, q in zip(r_all, r_tight, reqs):
        assert a.status == 0 and b.status == 0
        assert np.array_equal(a.x, b.x)
        code, info, x = alone(q, prec_fp32=False)
        assert np.array_equal(a.x, x)
    # a request larger than the budget is refused, the others still run
    tiny = S.Server(max_active=2, workers=2, realtime=False, mem_budget=need // 2)
    rr = tiny.run(reqs[:2])
    assert all(r.status in (0, -1) for r in rr)
    assert any(r.status == -1 and "budget" in r.error for r in rr) or all(r.device_bytes <= need // 2 for r in rr)


@pytest.mark.gpu
def test_batch_slots_and_statuses():
    import torch
    md = H.random_mesh(2, 4, 0.3, 2, 1, 5, seed=91)
    m = G.Mesh(md)
    ops = [G.Operator(m, host_only=True) for _ in range(3)]
    f = torch.from_numpy(H.gaussian_rhs(m.ndof, 92)).cuda()
    bt = G.Batch(1)
    bs, xs = [], []
    with pytest.raises(G.HpdgError) as e:                    # not on the device yet
        bt.admit(ops[0], f, torch.zeros_like(f))
    assert e.value.code == -6
    for op in ops:
        op.upload()
        b = torch.empty_like(f)
        op.rhs(f, b)
        bs.append(b)
        xs.append(torch.zeros_like(f))
    torch.cuda.synchronize()
    assert bt.admit(ops[0], bs[0], xs[0], maxit=500, tag=10)
    assert not bt.admit(ops[1], bs[1], xs[1], tag=11)        # one slot: busy
    done = []
    t0 = time.time()
    while not done and time.time() - t0 < 30:
        bt.step(wait_us=500)
        done += bt.poll()
    assert done and done[0][0] == 10 and done[0][1] == 0
    # maxit reached: NOT_CONVERGED with the iterations done
    assert bt.admit(ops[1], bs[1], xs[1], maxit=3, tag=11)
    # non-finite right-hand side: INVALID, no iteration
    bad = bs[2].clone()
    bad[5] = float("nan")
    torch.cuda.synchronize()
    got = {}
    t0 = time.time()
    while len(got) < 2 and time.time() - t0 < 30:
        na, nd = bt.step(wait_us=500)
        for tag, code, info in bt.poll():
            got[tag] = (code, info)
        if na == 0 and 12 not in got:
            assert bt.admit(ops[2], bad, xs[2], tag=12)
    assert got[11][0] == -5 and got[11][1]["iters"] == 3
    assert got[12][0] == -1
    # the batch's result equals the blocking solve
    x_ref = torch.zeros_like(f)
    info = ops[0].pcg_solve(bs[0], x_ref, rtol=1e-8, maxit=500)
    assert torch.equal(x_ref, xs[0]) and info[0]["iters"] == done[0][2]["iters"]


@pytest.mark.gpu
def test_admitted_operator_is_held_and_guarded():
    """While a solve is in flight, apply_B and pcg_solve on its operator are
    refused (they share its work vectors); the binding keeps the operator
    and vectors alive until poll() returns the tag, even when the caller
    drops its own references."""
    import gc
    import torch
    md = H.random_mesh(2, 4, 0.3, 2, 1, 5, seed=93)
    m = G.Mesh(md)
    op = G.Operator(m)
    f = torch.from_numpy(H.gaussian_rhs(m.ndof, 94)).cuda()
    b = torch.empty_like(f)
    op.rhs(f, b)
    x = torch.zeros_like(f)
    torch.cuda.synchronize()
    bt = G.Batch(2)
    assert bt.admit(op, b, x, maxit=500, tag=5)
    with pytest.raises(ValueError):
        bt.admit(op, b, x, tag=5)
    r = torch.ones_like(f)
    z = torch.empty_like(f)
    with pytest.raises(G.HpdgError) as e:
        op.apply_B(r, z)
    assert e.value.code == -1 and "in flight" in str(e.value)
    with pytest.raises(G.HpdgError) as e:
        op.pcg_solve(b, torch.zeros_like(f))
    assert e.value.code == -1
    ref_b = b.clone()
    del op, b, x
    gc.collect()
    assert 5 in bt._held
    done = []
    t0 = time.time()
    while not done and time.time() - t0 < 30:
        bt.step(wait_us=500)
        done += bt.poll()
    assert done and done[0][0] == 5 and done[0][1] == 0 and 5 not in bt._held
    # a fresh blocking solve of the same system gives the same iteration count
    op2 = G.Operator(m)
    x2 = torch.zeros_like(f)
    info = op2.pcg_solve(ref_b, x2, rtol=1e-8, maxit=500)
    assert info[0]["iters"] == done[0][2]["iters"]


@pytest.mark.gpu
def test_served_results_match_oracle():
    import scipy.sparse.linalg as spla

    import oracle as O
    from oracle import dg
    reqs = small_requests(4, seed=5017, dof_hi=1500)
    srv = S.Server(max_active=4, workers=2, realtime=False, keep_x=True)
    res = srv.run(reqs)
    for q, r in zip(reqs, res):
        assert r.status == 0
        m = O.Mesh(q.mesh)
        opts = O.Opts(q.form, 0, 1.0 if q.form == "sipg" else 0.0)
        A = dg.assemble_sparse(m, opts).tocsc()
        b = dg.rhs(m, q.f)
        xs = spla.spsolve(A, b)
        err = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
        print(f"request {q.id}: dim {m.dim} {q.form} ndof {m.ndof} rel err {err:.2e}", flush=True)
        assert err < 1e-5


@pytest.mark.gpu
def test_realtime_arrivals():
    reqs = small_requests(12, seed=5019)
    rate = 200.0
    t = 0.0
    rng = np.random.default_rng(3)
    for q in reqs:
        t += rng.exponential(1.0 / rate)
        q.t_arrive = t
    srv = S.Server(max_active=4, workers=4, realtime=True)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    s = S.summarize(res, wall)
    assert s["ok"] == len(reqs)
    for r in res:
        assert r.t_done >= r.t_arrive and r.t_admit >= r.t_arrive
