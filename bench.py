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
# the kernel sources and build script they were measured on; reported only while that hash
# still matches (the summaries with their commands are under profiles/).
MEASURED_TRAFFIC = {
    "convdiff2d-512": ("fd823326c946c3f1", 438913824394.0),
}


def kernel_source_hash() -> str:
    """sha256[:16] of the kernel sources and the build script (its flags)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_0907_4631_amd", "csrc", "*"))
                   if os.path.isfile(f))
    files.append(os.path.join(ROOT, "paper_0907_4631_amd", "_build.py"))
    for f in files:
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
    "reaction2d-1024-calls": ("config5", "2D diffusion-reaction Jacobian 1024x1024 "
                              "(Laplacian + diag(1 - 3 u^2), n=1048576), p=2, t=1e-3, tol=1e-6, "
                              "successive calls with new b; learned (tau, m) proposer vs plain "
                              "step control (cold and warm start)", "fp64"),
    "allencahn-1024-ere": ("config5", "Allen-Cahn u_t = Lap u + u - u^3 on the 1024x1024 grid "
                           "(n=1048576) from the config-5 field, exponential Rosenbrock-Euler "
                           "steps h=1e-3, one phipm call per step (p=1, tol=1e-6, Lanczos); "
                           "learned (tau, m) proposer vs plain step control (cold and warm)",
                           "fp64"),
    "heston-100x51": ("heston_problem", "finite-difference Heston operator on the 100x51 grid "
                      "of the paper's Sect. 5.1 (n=5100), p=1, t=T=1, tol=1e-6, Arnoldi, FP64",
                      "fp64"),
    "convdiff2d-batch256": ("config4", "256 independent 2D upwind convection-diffusion solves "
                            "(N_i in 32..256, Peclet in 0..100, p_i in 0..3, t_i in 1e-4..1e-1, "
                            "tol=1e-7) in one persistent autotuned launch replayed from a hipGraph",
                            "fp64"),
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


def cpu_baseline_batch(probs, gpu_stats, budget_s=20.0, seed=7):
    """The oracle on the host cores, timed on a seeded random sample of the
    batch's instances (about budget_s of CPU work) and scaled to the whole
    batch by rows x products (the GPU run's product counts)."""
    import oracle
    oracle.build(force=False)
    order = np.random.default_rng(seed).permutation(len(probs))
    spent, work_done, done = 0.0, 0.0, 0
    for i in order:
        pb = probs[i]
        w = pb.n * max(1, gpu_stats[i]["matvecs"])
        t0 = time.perf_counter()
        oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol)
        spent += time.perf_counter() - t0
        work_done += w
        done += 1
        if spent > budget_s:
            break
    total = sum(pb.n * max(1, s["matvecs"]) for pb, s in zip(probs, gpu_stats))
    per_batch = spent * total / work_done
    return {"value": len(probs) / per_batch, "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{done} randomly chosen of the {len(probs)} instances ({spent:.1f} s), "
                      f"scaled to the batch by rows x products"}


def run_integrator(args):
    """Exponential Rosenbrock-Euler steps of the Allen-Cahn equation whose
    Jacobians the call sequence samples: the learned proposer (the timed
    variant) beside the plain step control cold and warm-started."""
    import torch
    import paper_0907_4631_amd as pk
    from paper_0907_4631_amd import integrator
    from paper_0907_4631_amd import proposer as PR
    import workloads as W
    N, h, tol, steps = 1024, 1e-3, 1e-6, args.steps
    lap = W.laplace2d(N)
    u0 = W.smooth_field(N, 5999)
    res, outs = {}, {}
    for name in ("learned", "plain-cold", "plain-warm"):
        kw = {"proposer": PR.load()} if name == "learned" else {"warm": name == "plain-warm"}
        ig = integrator.AllenCahnERE(lap, u0, h, tol=tol, **kw)
        sts = ig.run(max(1, args.warmup), stats=True)        # untimed, then restart from u0
        ig.u.copy_(torch.as_tensor(u0, device="cuda"))
        if ig.hist is not None:
            ig.hist.zero_()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ig.run(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        if pk.lib().phipm_last_status() != 0:
            raise pk.PhipmError(pk.lib().phipm_last_status(), name)
        outs[name] = ig.u.cpu().numpy()
        ig.u.copy_(torch.as_tensor(u0, device="cuda"))   # statistics from an untimed repeat
        if ig.hist is not None:
            ig.hist.zero_()
        sts = ig.run(steps, stats=True)
        res[name] = {"ms_per_step": ms, "steps_per_s": 1e3 / ms,
                     "solver_steps": sum(x["steps"] for x in sts),
                     "rejected": sum(x["rejected"] for x in sts),
                     "matvecs": sum(x["matvecs"] for x in sts)}
    ref = outs["plain-cold"]
    for name in res:
        res[name]["max_diff_vs_plain_cold"] = float(np.linalg.norm(outs[name] - ref) /
                                                    max(1.0, np.linalg.norm(ref)))
    ms = res["learned"]["ms_per_step"]
    line = {
        "metric": "phipm solves/s (adaptive Krylov phi-function solve to t_end) and HBM GB/s",
        "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["allencahn-1024-ere"][1], "n": N * N, "h": h,
                   "integrator_steps": steps, "variants": res},
    }
    print(json.dumps(line), flush=True)


def run_calls(args):
    """Successive calls on one operator with new right-hand sides: the
    learned proposer (the timed variant) beside the plain step control cold
    and warm-started, and the FP32 basis."""
    import torch
    import paper_0907_4631_amd as pk
    from paper_0907_4631_amd import proposer as PR
    import workloads as W
    A = W.config5_matrix()
    n = A.shape[0]
    t, tol, calls = 1e-3, 1e-6, args.steps
    Ad = pk.DeviceCSR(A)
    bs = [torch.as_tensor(np.ascontiguousarray(W.config5_b(c, n).T), device="cuda")
          for c in range(calls)]
    weights = PR.load()
    variants = [("learned", pk.FP64, True, False), ("plain-cold", pk.FP64, False, False),
                ("plain-warm", pk.FP64, False, True), ("learned-fp32-basis", pk.FP32_BASIS, True,
                                                        False)]
    res, outs = {}, {}
    for name, prec, learned, warm in variants:
        s = pk.Solver(Ad, 2, tol=tol, precision=prec)
        hist = torch.zeros(4, dtype=torch.float64, device="cuda")
        if warm:
            s.opts.history = hist.data_ptr()
        if learned:
            s.opts.proposer = weights.data_ptr()
        us = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(calls)]
        for w in range(max(1, args.warmup)):
            s(t, bs[w % calls], us[0], stats=False)
        hist.zero_()
        torch.cuda.synchronize()
        tot = {"steps": 0, "rejected": 0, "matvecs": 0, "fp64_fallbacks": 0}
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for c in range(calls):
            s(t, bs[c], us[c], stats=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / calls
        if pk.lib().phipm_last_status() != 0:
            raise pk.PhipmError(pk.lib().phipm_last_status(), name)
        for c in range(calls):   # statistics from an untimed repeat of every call
            st = s(t, bs[c], us[c])
            for k in ("steps", "rejected", "matvecs"):
                tot[k] += st[k]
            tot["fp64_fallbacks"] += st["fp64_fallback"]
        outs[name] = [u.cpu().numpy() for u in us]
        res[name] = {"ms_per_call": ms, "calls_per_s": 1e3 / ms, **tot}
    ref = outs["plain-cold"]
    for name in res:
        res[name]["max_diff_vs_plain_cold"] = max(
            float(np.linalg.norm(a - b) / max(1.0, np.linalg.norm(b)))
            for a, b in zip(outs[name], ref))
    ms = res["learned"]["ms_per_call"]
    line = {
        "metric": "phipm solves/s (adaptive Krylov phi-function solve to t_end) and HBM GB/s",
        "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1, "steps": calls,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["reaction2d-1024-calls"][1], "n": n, "nnz": int(A.nnz),
                   "calls": calls, "variants": res},
    }
    if not args.no_cpu:
        class _P:
            pass
        pb = _P()
        pb.A, pb.b, pb.t, pb.tol = A, W.config5_b(0, n), t, tol
        line["cpu_baseline"] = cpu_baseline(pb, max(1, res["plain-cold"]["steps"] +
                                                     res["plain-cold"]["rejected"]) // calls)
        line["cpu_baseline"]["sample"] += " (plain step control, one call)"
    print(json.dumps(line), flush=True)


def run_batch(args):
    import torch
    import paper_0907_4631_amd as pk
    import workloads as W
    specs = W.config4_specs()
    probs = [W.config4_problem(s) for s in specs]
    As = [pk.DeviceCSR(pb.A) for pb in probs]
    bs = [torch.as_tensor(np.ascontiguousarray(pb.b.T), device="cuda") for pb in probs]
    us = [torch.empty(pb.n, dtype=torch.float64, device="cuda") for pb in probs]
    precision = pk.FP32_BASIS if args.precision == "fp32" else pk.FP64
    t0 = time.perf_counter()
    plan = pk.Plan(As, [pb.p for pb in probs], [pb.t for pb in probs], bs, us, tol=probs[0].tol,
                   precision=precision, workgroups=args.workgroups,
                   plan_opts=pk.default_plan_opts(autotune=0 if args.no_tune else 1, graph=1))
    create_s = time.perf_counter() - t0
    info = plan.info()
    for _ in range(max(1, args.warmup)):
        plan.execute()
    torch.cuda.synchronize()
    st = plan.stats()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.execute(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    plan.stats()   # raises on a device-side error of the timed runs
    nbytes = sum(s["bytes"] for s in st)
    achieved = nbytes / (ms / 1e3) / 1e9
    line = {
        "metric": "phipm solves/s (adaptive Krylov phi-function solve to t_end) and HBM GB/s",
        "value": len(probs) / (ms / 1e3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == pk.FP64 else "f32-basis/f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS["convdiff2d-batch256"][1],
            "instances": len(probs), "rows": int(sum(pb.n for pb in probs)),
            "nnz": int(sum(pb.A.nnz for pb in probs)),
            "plan": {k: info[k] for k in ("teams", "class_size", "class_teams", "graph",
                                          "cooperative", "candidates", "max_team", "alpha",
                                          "tuned_ms", "default_ms")},
            "plan_create_s": create_s,
            "solve_stats": {"steps": sum(s["steps"] for s in st),
                            "rejected": sum(s["rejected"] for s in st),
                            "matvecs": sum(s["matvecs"] for s in st),
                            "fp64_fallbacks": sum(s["fp64_fallback"] for s in st)},
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_batch (persistent batched solver)",
            "algorithmic_bytes_per_launch": nbytes,
        },
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_batch(probs, st)
    print(json.dumps(line), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff2d-512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="basis precision (default: the workload's)")
    ap.add_argument("--no-tune", action="store_true", help="batched workload: skip the autotuner")
    ap.add_argument("--fixed-m", type=int, default=0, metavar="M",
                    help="single solves: the paper's phip (Krylov dimension fixed at M, only tau "
                         "adapted) instead of phipm")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="single solves: override the workload's tolerance (a different "
                         "workload: named in config.tol)")
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

    if args.precision is None:
        args.precision = WORKLOADS[args.workload][2]
    if args.workload == "convdiff2d-batch256":
        run_batch(args)
        return
    if args.workload == "reaction2d-1024-calls":
        run_calls(args)
        return
    if args.workload == "allencahn-1024-ere":
        run_integrator(args)
        return
    pb = build_problem(args.workload)
    if args.tol > 0.0:
        pb.tol = args.tol
    A = pk.DeviceCSR(pb.A, device="cuda")
    b = torch.as_tensor(np.ascontiguousarray(pb.b.T), device="cuda")
    u = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    precision = pk.FP32_BASIS if args.precision == "fp32" else pk.FP64
    kw = {}
    if args.fixed_m > 0:
        kw = dict(adapt_m=0, m_init=args.fixed_m, m_max=args.fixed_m)
    solver = pk.Solver(A, pb.p, tol=pb.tol, precision=precision, workgroups=args.workgroups,
                       validate=1, **kw)
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
    default_run = (args.fixed_m == 0 and args.tol == 0.0 and args.workgroups == 0 and
                   args.precision == WORKLOADS[args.workload][2])
    if default_run and args.workload in MEASURED_TRAFFIC:
        # the counters were taken on the workload's own configuration only
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
            "workload": WORKLOADS[args.workload][1] +
                        (f" (tolerance overridden: tol={pb.tol:g})" if args.tol > 0.0 else ""),
            "n": pb.n, "nnz": int(pb.A.nnz), "p": pb.p, "t": pb.t, "tol": pb.tol,
            "workgroups": st["workgroups"], "lanczos": st["lanczos"],
            "method": f"phip (m fixed at {args.fixed_m})" if args.fixed_m > 0 else "phipm",
            "solve_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms",
                                                "m_last", "fp64_fallback",
                                                "fp32_error_estimate")},
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
