"""Benchmark: PCG solves of the hp-DG system on one MI355X.

A step is one full solve of the cfg2 workload (2D random hp mesh, 32x32 base
quads refined with probability 0.3 up to 3 levels, p ~ U{1..8}, SIPG, k=1,
f = seeded Gaussian nodal values, 155,228 DOFs) from x0 = 0 to 1e-8 relative
residual with the FP64 subspace-correction preconditioner: every iteration
applies the matrix-free DG operator and B = B_J + B_E + P V(A~_C) P^T.
Inputs are resident on the GPU before the timed region.

Prints one JSON line. Besides the contract fields it reports the DG apply
rate (GDOF/s) and its fraction of the HBM roofline measured with HIP events
on the library's stream, a rocprof-comparable per-kernel figure for the
dominant kernel, and the oracle's CPU time on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X
WORKLOADS = {2: "cfg2_random2d_32x32_q0.3_L3_p1-8_sipg_fp64",
             3: "cfg3_random3d_16^3_q0.2_L2_p1-6_br2_fp32prec",
             4: "cfg4_cfg2mesh_64rhs_fp32prec"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import hpinputs as H
    import paper_2009_01287_amd as G

    cfg = args.config
    c = H.CONFIGS[cfg]
    md = H.config_mesh(cfg)
    nrhs = c["nrhs"]
    t0 = time.time()
    mesh = G.Mesh(md)
    op = G.Operator(mesh, form=c["form"], penalty_rule=c["penalty_rule"], eta=c["eta"],
                    prec_fp32=bool(c["prec_fp32"]), max_nrhs=nrhs,
                    max_block=256 if md["dim"] == 3 else 0)
    t_setup = time.time() - t0
    n = mesh.ndof
    f = torch.from_numpy(np.ascontiguousarray(H.config_rhs(cfg, n).reshape(-1))).cuda()
    b = torch.empty_like(f)
    op.rhs(f, b, nrhs=nrhs)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()

    infos = None
    for _ in range(args.warmup):
        x.zero_()
        infos = op.pcg_solve(b, x, nrhs=nrhs, rtol=c["rtol"], maxit=5000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        infos = op.pcg_solve(b, x, nrhs=nrhs, rtol=c["rtol"], maxit=5000)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    solves_per_s = nrhs / dt

    # DG apply rate, HIP events on the stream the library launches on
    y = torch.empty_like(b)
    for _ in range(10):
        op.apply_A(b, y, nrhs=nrhs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.apply_reps):
        op.apply_A(b, y, nrhs=nrhs)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / 1e3 / args.apply_reps
    apply_bytes = 16.0 * n * nrhs
    gdofs = n * nrhs / t_apply / 1e9
    it = infos[0]["iters"]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(md, c, it)

    out = {
        "metric": "DG apply GDOF/s + %HBM peak; solves/s and p50/p99 latency at 1e-8 residual",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not c["prec_fp32"] else "f64 (A, CG) + f32 (B)",
        "data": "synthetic",
        "config": {"workload": WORKLOADS.get(cfg, str(cfg)), "ndof": n, "nrhs": nrhs,
                   "elements": int(len(md["level"])), "rtol": c["rtol"]},
        "solve": {"iters": it, "true_rel_res": max(i["true_rel_res"] for i in infos),
                  "cond_est": infos[0]["cond_est"], "setup_s": t_setup},
        "apply": {"gdof_per_s": gdofs, "us_per_apply": t_apply * 1e6,
                  "hbm_frac_16B_per_dof": apply_bytes / t_apply / HBM_PEAK},
        "roofline": {"bound": "hbm", "achieved": apply_bytes / t_apply / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": apply_bytes / t_apply / HBM_PEAK, "traffic": None,
                     "kernel": "apply_A (volume + face kernels), 16 B/DOF"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(md, c, gpu_iters):
    """The oracle (numpy/scipy FP64) on this host: setup excluded, a bounded
    sample of PCG iterations (one A apply and one B apply each), scaled to
    the GPU's iteration count to give solves/s."""
    import numpy as np
    import oracle as O
    from oracle import dg, precond
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    m = O.Mesh(md)
    opts = O.Opts(c["form"], c["penalty_rule"], c["eta"])
    pc = precond.Preconditioner(m, opts)
    r = np.random.default_rng(0).standard_normal(m.ndof)
    k = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 15.0 and k < 50:
        y = dg.apply(m, opts, r)
        r = pc.apply(y / np.linalg.norm(y))
        k += 1
    per_it = (time.perf_counter() - t0) / k
    return {"value": 1.0 / (per_it * gpu_iters), "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{k} oracle PCG iterations (matrix-free A + B) on the full mesh, "
                      f"{per_it:.2f} s each, scaled to {gpu_iters} iterations; setup excluded; "
                      f"host cores {os.cpu_count()}"}


if __name__ == "__main__":
    main()
