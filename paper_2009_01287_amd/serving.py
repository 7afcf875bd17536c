"""Continuous-batching server for hp-DG solves on one GPU.

Each request carries a mesh (leaf arrays: level, anchor, degree, k), the
form (SIPG or BR2) and nodal load values f; the answer is the DG solution of
A x = M f to a relative residual rtol by PCG with the subspace-correction
preconditioner.

Pipeline of a request:
  1. setup worker (host thread; the native setup releases the GIL): mesh
     topology, operator and preconditioner on the host (host_only), then the
     exact device bytes the operator will hold (a counting pass of the upload);
  2. admission by device memory: the worker waits until those bytes plus the
     request's vectors fit in the budget, then uploads the operator, forms
     b = M f on a stream of its own and hands the request over;
  3. the native batch executor keeps up to max_active solves on the GPU, each
     on its own stream, starts new ones as slots free up and retires
     converged ones; memory is returned to the budget at retirement.

Latency of a request = retirement - arrival: queueing, host setup, admission
wait, upload and solve. Every reduction in the solve has a fixed order, so a
request's result does not depend on what runs beside it.
"""
from __future__ import annotations

import queue
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import Batch, HpdgError, Mesh, Operator


class MemoryGate:
    """Device-memory budget in bytes. acquire blocks until the request fits;
    a request larger than the whole budget is refused."""

    def __init__(self, budget):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self.waiters = 0
        self._cv = threading.Condition()
        self._closed = False

    def acquire(self, n, timeout=None):
        n = int(n)
        if n > self.budget:
            raise MemoryError(f"request needs {n} bytes, budget is {self.budget}")
        with self._cv:
            self.waiters += 1
            try:
                ok = self._cv.wait_for(lambda: self._closed or self.used + n <= self.budget, timeout)
            finally:
                self.waiters -= 1
            if self._closed:
                raise RuntimeError("server stopped")
            if not ok:
                return False
            self.used += n
            self.peak = max(self.peak, self.used)
            return True

    def release(self, n):
        with self._cv:
            self.used -= int(n)
            assert self.used >= 0
            self._cv.notify_all()

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()


@dataclass
class Request:
    id: int
    mesh: dict
    form: str = "sipg"
    f: np.ndarray | None = None      # nodal load values (ndof,)
    t_arrive: float = 0.0            # seconds after the start of the run
    rtol: float = 1e-8
    maxit: int = 5000
    eta: float | None = None         # None: 1 for SIPG, automatic for BR2


@dataclass
class Result:
    id: int
    status: int
    ndof: int = 0
    dim: int = 0
    form: str = ""
    iters: int = 0
    true_rel_res: float = float("nan")
    t_arrive: float = 0.0
    t_setup: float = 0.0             # host setup seconds
    t_admit: float = 0.0             # time the solve started on the GPU
    t_done: float = 0.0
    device_bytes: int = 0
    x: np.ndarray | None = None
    error: str = ""

    @property
    def latency(self):
        return self.t_done - self.t_arrive


@dataclass
class _Ready:
    req: Request
    mesh: object
    op: object
    f: object
    b: object
    x: object
    nbytes: int
    t_setup: float
    res: Result = field(default=None)


class Server:
    """Serve a list of requests; run() returns one Result per request.

    max_active   solves in flight on the GPU (streams of the batch)
    mem_budget   device bytes for operators and vectors of admitted requests
    workers      host setup threads
    prec_fp32    FP32 preconditioner under FP64 PCG (else all FP64)
    max_block    V_e components above this size use point Jacobi (3D)
    realtime     honour the arrival times (else every request arrives at 0)
    keep_x       return each solution on the host
    min_batch    hold admission until this many requests are prepared (or no
                 more can be: all prepared, or a worker waits for memory)
    auto_cycle   fused V-cycle levels and a small dense tail without timing
                 (fewer launches per iteration; the solves are small and
                 launch bound)
    graph        replay each solve's chunks of CG iterations from HIP graphs
                 (one launch per chunk instead of one per kernel). A capture
                 must not overlap device calls of other threads on the legacy
                 stream (allocations, synchronous copies), so with graphs the
                 workers' uploads and the batch steps take turns on a lock.
    """

    def __init__(self, max_active=16, mem_budget=64 << 30, workers=8, prec_fp32=True, max_block=256,
                 realtime=True, keep_x=False, min_batch=1, graph=False, auto_cycle=True):
        self.max_active = max_active
        self.gate = MemoryGate(mem_budget)
        self.workers = workers
        self.prec_fp32 = prec_fp32
        self.max_block = max_block
        self.realtime = realtime
        self.keep_x = keep_x
        self.min_batch = min_batch
        self.graph = graph
        self.auto_cycle = auto_cycle
        self._dev_lock = threading.Lock() if graph else None
        self.max_concurrent = 0

    # -- worker side ---------------------------------------------------
    def _prepare(self, req: Request, t0: float, ready: queue.Queue, streams):
        import torch
        res = Result(id=req.id, status=0, t_arrive=req.t_arrive, form=req.form, dim=int(req.mesh["dim"]))
        try:
            ts = time.perf_counter()
            mesh = Mesh(req.mesh)
            eta = req.eta if req.eta is not None else (1.0 if req.form == "sipg" else 0.0)
            op = Operator(mesh, form=req.form, eta=eta, prec_fp32=self.prec_fp32, host_only=True,
                          max_block=self.max_block if mesh.dim == 3 else 0, graph=self.graph,
                          auto_cycle=self.auto_cycle,
                          setup_threads=1)     # the workers already run setups in parallel
            res.ndof = mesh.ndof
            nbytes = op.device_bytes() + 3 * 8 * mesh.ndof
            res.device_bytes = nbytes
            res.t_setup = time.perf_counter() - ts
            f = np.ascontiguousarray(req.f, dtype=np.float64).reshape(-1)
            if f.shape[0] != mesh.ndof:
                raise ValueError(f"request {req.id}: f has {f.shape[0]} values, mesh has {mesh.ndof} DOFs")
            self.gate.acquire(nbytes)
            try:
                s = streams.get()
                lock = self._dev_lock
                if lock:
                    lock.acquire()
                try:
                    with torch.cuda.stream(s):
                        op.upload(stream=s.cuda_stream)
                        fd = torch.from_numpy(f).to("cuda", non_blocking=False)
                        b = torch.empty_like(fd)
                        x = torch.zeros_like(fd)
                        op.rhs(fd, b, stream=s.cuda_stream)
                    s.synchronize()
                finally:
                    if lock:
                        lock.release()
                    streams.put(s)
            except BaseException:
                self.gate.release(nbytes)
                raise
            ready.put(_Ready(req, mesh, op, fd, b, x, nbytes, res.t_setup, res))
        except Exception as e:      # reported per request
            res.status = getattr(e, "code", -1)
            res.error = str(e)
            res.t_done = time.perf_counter() - t0
            ready.put(res)

    # -- main loop -----------------------------------------------------
    def run(self, requests):
        import torch
        reqs = sorted(requests, key=lambda r: (r.t_arrive if self.realtime else 0.0, r.id))
        ready: queue.Queue = queue.Queue()
        streams: queue.Queue = queue.Queue()
        for _ in range(self.workers):
            streams.put(torch.cuda.Stream())
        batch = Batch(self.max_active)
        results = {}
        inflight = {}          # tag -> _Ready
        waiting = []           # prepared, not yet admitted (slots full)
        pool = ThreadPoolExecutor(max_workers=self.workers)
        t0 = time.perf_counter()
        i = 0
        n = len(reqs)
        try:
            while len(results) < n:
                now = time.perf_counter() - t0
                while i < n and (not self.realtime or reqs[i].t_arrive <= now):
                    pool.submit(self._prepare, reqs[i], t0, ready, streams)
                    i += 1
                while True:
                    try:
                        item = ready.get_nowait()
                    except queue.Empty:
                        break
                    if isinstance(item, Result):
                        results[item.id] = item
                    else:
                        waiting.append(item)
                # admit at chunk boundaries while slots are free
                left = n - len(results) - len(inflight)
                hold = (len(waiting) < min(self.min_batch, left) and self.gate.waiters == 0)
                lock = self._dev_lock
                while waiting and not hold:
                    it = waiting[0]
                    if lock:
                        with lock:
                            ok = batch.admit(it.op, it.b, it.x, rtol=it.req.rtol, maxit=it.req.maxit, tag=it.req.id)
                    else:
                        ok = batch.admit(it.op, it.b, it.x, rtol=it.req.rtol, maxit=it.req.maxit, tag=it.req.id)
                    if not ok:
                        break
                    it.res.t_admit = time.perf_counter() - t0
                    inflight[it.req.id] = it
                    waiting.pop(0)
                self.max_concurrent = max(self.max_concurrent, len(inflight))
                if inflight:
                    if lock:
                        with lock:
                            _, nd = batch.step(wait_us=200)
                    else:
                        _, nd = batch.step(wait_us=200)
                    if nd:
                        for tag, code, info in batch.poll():
                            it = inflight.pop(tag)
                            r = it.res
                            r.t_done = time.perf_counter() - t0
                            r.status = code
                            r.iters = info["iters"]
                            r.true_rel_res = info["true_rel_res"]
                            if self.keep_x:
                                if lock:
                                    with lock:
                                        r.x = it.x.cpu().numpy()
                                else:
                                    r.x = it.x.cpu().numpy()
                            results[tag] = r
                            del it.op, it.mesh, it.f, it.b, it.x
                            self.gate.release(it.nbytes)
                else:
                    # nothing on the GPU: wait for the next prepared request or arrival
                    timeout = 0.002
                    if self.realtime and i < n and ready.empty():
                        timeout = max(0.0, min(0.05, reqs[i].t_arrive - (time.perf_counter() - t0)))
                    try:
                        item = ready.get(timeout=timeout)
                        ready.put(item)
                    except queue.Empty:
                        pass
        finally:
            self.gate.close()
            pool.shutdown(wait=True)
            del batch
        return [results[r.id] for r in requests]


def summarize(results, wall):
    """solves/s, p50/p99 latency (s) and totals of a run."""
    ok = [r for r in results if r.status == 0]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    return {
        "requests": len(results),
        "ok": len(ok),
        "wall_s": wall,
        "solves_per_s": len(ok) / wall if wall > 0 else float("nan"),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "dofs": int(sum(r.ndof for r in ok)),
        "iters_mean": float(np.mean([r.iters for r in ok])) if ok else float("nan"),
        "max_true_rel_res": float(max((r.true_rel_res for r in ok), default=float("nan"))),
        "host_setup_s": float(sum(r.t_setup for r in results)),
        "errors": sorted({f"{r.status}: {r.error}" for r in results if r.status != 0})[:5],
    }


__all__ = ["MemoryGate", "Request", "Result", "Server", "summarize", "HpdgError"]
