"""Throughput benchmark of the GPU phipm solver.

One step = one full adaptive solve u = sum_k t^k phi_k(tA) b_k to t_end on a
synthetic workload whose inputs are already resident in HBM.  Prints one JSON
line with solves/s, the roofline position of the solver kernel (algorithmic
bytes per solve / measured solve time against the 8 TB/s HBM peak) and the CPU
oracle timed on a bounded sample of the same solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per solver launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE
# (scaled against a plain device copy), keyed by workload and by the hash of
# the kernel sources they were measured on; reported only while that hash
# still matches (the summaries with their commands are under profiles/).
MEASURED_TRAFFIC = {
    "convdiff2d-512": ("c2d2b00fa1ec1447", 753978081505.0),
}


def kernel_source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_0907_4631_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

WORKLOADS = {
    # name: (builder, description, basis precision)
    "convdiff2d-512": ("config2", "2D upwind convection-diffusion 512x512 (n=262144, D=1, "
                       "v=(50,50)), p=2, t=1e-2, tol=1e-8, Arnoldi, FP64", "fp64"),
    "laplace3d-128": ("config3", "3D 7-point Laplacian 128^3 (n=2097152), p=3, t=1e-4, "
                      "tol=1e-6, Lanczos", "fp64"),
    "laplace2d-30": ("config1", "2D 5-point Laplacian 30x30 (n=900), p=1, t=1e-3, tol=1e-7, "
                     "Lanczos, FP64", "fp64"),
}


def build_problem(name):
    import workloads as W
    return getattr(W, WORKLOADS[name][0])()


def cpu_baseline(pb, gpu_attempts, budget_s=20.0):
    """The oracle on the host cores, timed on the first attempts of the same
    solve and scaled to the attempts the GPU solve needed."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    _, st = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol, max_attempts=2, allow_limit=True)
    t_probe = time.perf_counter() - t0
    per = t_probe / max(1, st["steps"] + st["rejected"])
    k = int(max(2, min(gpu_attempts, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    _, st = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol, max_attempts=k, allow_limit=True)
    dt = time.perf_counter() - t0
    done = max(1, st["steps"] + st["rejected"])
    per_solve = dt * gpu_attempts / done
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"first {done} of the {gpu_attempts} attempts of one solve "
                      f"({dt:.1f} s), scaled by attempt count"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff2d-512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (3 times), so that "
                         "HBM byte counters can be scaled against a known transfer")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this solver runs each solve on a single "
              "MI355X (multi-GPU sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0907_4631_amd as pk

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "calibrate_copy_bytes_written": n * 8,
                          "launches": 3}), flush=True)
        return

    pb = build_problem(args.workload)
    A = pk.DeviceCSR(pb.A, device="cuda")
    b = torch.as_tensor(np.ascontiguousarray(pb.b.T), device="cuda")
    u = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    precision = pk.FP32_BASIS if WORKLOADS[args.workload][2] == "fp32" else pk.FP64
    solver = pk.Solver(A, pb.p, tol=pb.tol, precision=precision, workgroups=args.workgroups,
                       validate=1)
    st = None
    for _ in range(max(1, args.warmup)):
        st = solver(pb.t, b, u, stats=True)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        solver(pb.t, b, u, stats=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    status = pk.lib().phipm_last_status()
    if status != 0:
        raise pk.PhipmError(status, "timed solve")

    per_solve_s = ms / 1e3
    achieved = st["bytes"] / per_solve_s / 1e9
    traffic = None
    if args.workload in MEASURED_TRAFFIC:
        sha, nbytes = MEASURED_TRAFFIC[args.workload]
        if sha == kernel_source_hash():
            traffic = nbytes
    attempts = st["steps"] + st["rejected"]
    line = {
        "metric": "phipm solves/s (adaptive Krylov phi-function solve to t_end) and HBM GB/s",
        "value": 1.0 / per_solve_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == pk.FP64 else "f32-basis/f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload][1],
            "n": pb.n, "nnz": int(pb.A.nnz), "p": pb.p, "t": pb.t, "tol": pb.tol,
            "workgroups": st["workgroups"], "lanczos": st["lanczos"],
            "solve_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms",
                                                "m_last")},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_solve (persistent solver)",
            "algorithmic_bytes_per_launch": st["bytes"],
        },
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(pb, attempts)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
