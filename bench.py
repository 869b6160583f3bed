"""Throughput benchmark of the GPU phipm solver.

One step = one full adaptive solve u = sum_k t^k phi_k(tA) b_k to t_end on a
synthetic workload whose inputs are already resident in HBM.  Prints one JSON
line.  The default run measures the 512^2 convection-diffusion solve (Arnoldi,
FP64, tol 1e-8): solves/s, the roofline position of the solver kernel (the
reference byte model of a plain CGS2 Krylov step per solve / the measured
solve time, against the 8 TB/s HBM peak), the relative error against the CPU
oracle, the oracle's own time on the host cores, and, under "headline", the
200-call sequence of the 1024^2 reaction-diffusion operator at tol 1e-6 with
the learned (tau, m) proposer and the FP32 basis against the plain FP64
method.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20

# HBM bytes per solver launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE
# (scaled against a plain device copy), keyed by workload: (hash of the kernel
# sources and build script they were measured on, bytes, summary file).  A
# value is reported only while that hash still matches.
MEASURED_TRAFFIC = {
    "convdiff2d-512": ("607ea0405b77420a", 460.5872e9, "profiles/k_solve_convdiff2d-512_hbm_counters.md"),
    "laplace3d-128": ("607ea0405b77420a", 8.2482e9, "profiles/k_solve_laplace3d-128_hbm_counters.md"),
}


def log(msg: str) -> None:
    """Progress of a long run on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


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
    # name: (builder, description, basis precision, CSR value type)
    "convdiff2d-512": ("config2", "2D upwind convection-diffusion 512x512 (n=262144, D=1, "
                       "v=(50,50)), p=2, t=1e-2, tol=1e-8, Arnoldi, FP64", "fp64", "f64"),
    "laplace3d-128": ("config3", "3D 7-point Laplacian 128^3 (n=2097152), p=3, t=1e-4, "
                      "tol=1e-6, Lanczos", "fp64", "f32"),
    "laplace2d-30": ("config1", "2D 5-point Laplacian 30x30 (n=900), p=1, t=1e-3, tol=1e-7, "
                     "Lanczos, FP64", "fp64", "f64"),
    "reaction2d-1024": ("config5_call0", "2D diffusion-reaction Jacobian 1024x1024 (Laplacian + "
                        "diag(1 - 3 u^2), n=1048576), p=2, t=1e-3, tol=1e-6, one call, Lanczos",
                        "fp64", "f64"),
    "reaction2d-1024-calls": ("config5", "2D diffusion-reaction Jacobian 1024x1024 "
                              "(Laplacian + diag(1 - 3 u^2), n=1048576), p=2, t=1e-3, tol=1e-6, "
                              "successive calls with new b; learned (tau, m) proposer + FP32 "
                              "basis vs the plain FP64 method (cold and warm start)", "fp64",
                              "f64"),
    "allencahn-1024-ere": ("config5", "Allen-Cahn u_t = Lap u + u - u^3 on the 1024x1024 grid "
                           "(n=1048576) from the reaction-diffusion field, exponential "
                           "Rosenbrock-Euler steps h=1e-3, one phipm call per step (p=1, "
                           "tol=1e-6, Lanczos); learned (tau, m) proposer vs plain step control "
                           "(cold and warm)", "fp64", "f64"),
    "heston-100x51": ("heston_problem", "finite-difference Heston operator on the 100x51 grid "
                      "of the paper's Sect. 4.1 (n=5100), p=1, t=T=1, tol=1e-6, Arnoldi, FP64",
                      "fp64", "f64"),
    "convdiff2d-batch256": ("config4", "256 independent 2D upwind convection-diffusion solves "
                            "(N_i in 32..256, Peclet in 0..100, p_i in 0..3, t_i in 1e-4..1e-1, "
                            "tol=1e-7) in one persistent autotuned launch replayed from a hipGraph",
                            "fp64", "f64"),
}

METRIC = "phipm solves/s (adaptive Krylov phi-function solve to t_end) and HBM GB/s"


def build_problem(name):
    import workloads as W
    b = WORKLOADS[name][0]
    if b == "config5_call0":
        A = W.config5_matrix()
        pb = W.Problem("reaction2d-1024-call0", A, W.config5_b(0, A.shape[0]), 1e-3, 1e-6, True)
        return pb
    return getattr(W, b)()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_reference(pb, runs=3, budget_s=45.0, single_budget_s=10.0):
    """The oracle on the host cores: the whole solve timed `runs` times
    (median; fewer when one run is long), its solution (for the error of the
    GPU result), and a single-thread figure from the first attempts of the
    same solve, scaled by attempt count."""
    import oracle
    oracle.build(force=False)
    threads = oracle.threads()
    times, u, st = [], None, None
    for _ in range(runs):
        t0 = time.perf_counter()
        u, st = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol)
        times.append(time.perf_counter() - t0)
        if sum(times) > budget_s:
            break
    per_solve = float(np.median(times))
    attempts = st["steps"] + st["rejected"]
    # one thread, bounded sample: the first k attempts
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, s1 = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol, max_attempts=1, allow_limit=True)
        t1 = time.perf_counter() - t0
        k = int(max(1, min(attempts, single_budget_s / max(t1, 1e-9))))
        if k > 1:
            t0 = time.perf_counter()
            _, s1 = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol, max_attempts=k, allow_limit=True)
            t1 = time.perf_counter() - t0
        done = max(1, s1["steps"] + s1["rejected"])
        single = t1 * attempts / done
    finally:
        oracle.set_threads(threads)
    base = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole solve, {len(times)} run(s), median {per_solve:.2f} s "
                      f"({attempts} attempts); single thread: the first {done} attempts "
                      f"({t1:.1f} s) scaled by attempt count",
            "single_thread_value": 1.0 / single, "cpu_model": cpu_model(),
            "build": "gcc " + " ".join(oracle.CFLAGS[:3]),
            "oracle_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms")}}
    return u, base


def rel_err(u, ref):
    return float(np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-300))


def time_solves(solver, t, b, u, steps, warmup):
    import torch
    st = None
    for _ in range(max(1, warmup)):
        st = solver(t, b, u, stats=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        solver(t, b, u, stats=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, st


def fixed_m_kw(args):
    """Solver options of the paper's phip (Krylov dimension fixed, only the
    step size adapted) when --fixed-m is given; phipm's otherwise."""
    if args.fixed_m > 0:
        return dict(adapt_m=0, m_init=args.fixed_m, m_max=args.fixed_m)
    return {}


def method_name(args):
    return f"phip (m fixed at {args.fixed_m})" if args.fixed_m > 0 else "phipm"


def run_single(args, with_headline):
    import torch
    import paper_0907_4631_amd as pk
    pb = build_problem(args.workload)
    if args.tol > 0.0:
        pb.tol = args.tol
    precision = pk.FP32_BASIS if args.precision == "fp32" else pk.FP64
    vdt = np.float32 if args.values == "f32" else np.float64
    if vdt == np.float32 and not np.array_equal(pb.A.data.astype(np.float32).astype(np.float64),
                                                pb.A.data):
        vdt = np.float64   # the operator is not exact in float32: keep it as it is
    A = pk.DeviceCSR(pb.A, device="cuda", dtype=vdt)
    b = torch.as_tensor(np.ascontiguousarray(pb.b.T), device="cuda")
    u = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    kw = fixed_m_kw(args)
    solver = pk.Solver(A, pb.p, tol=pb.tol, precision=precision, workgroups=args.workgroups,
                       validate=1, **kw)
    log(f"{args.workload}: {args.warmup} warmup + {args.steps} timed solves")
    ms, st = time_solves(solver, pb.t, b, u, args.steps, args.warmup)
    log(f"{args.workload}: {ms:.3f} ms per solve")
    status = pk.lib().phipm_last_status()
    if status != 0:
        raise pk.PhipmError(status, "timed solve")
    u_gpu = u.cpu().numpy()

    sec = ms / 1e3
    achieved = st["bytes_ref"] / sec / 1e9
    traffic, traffic_src = None, None
    default_run = (args.fixed_m == 0 and args.tol == 0.0 and args.workgroups == 0 and
                   args.precision == WORKLOADS[args.workload][2])
    if default_run and args.workload in MEASURED_TRAFFIC:
        sha, nbytes, src = MEASURED_TRAFFIC[args.workload]
        if sha == kernel_source_hash():
            traffic, traffic_src = nbytes, src
    s = 4.0 if precision == pk.FP32_BASIS else 8.0
    sv = 4.0 if vdt == np.float32 else 8.0
    work_set = ((sv + 4.0) * pb.A.nnz + 4.0 * (pb.n + 1) +
                s * pb.n * (st["m_last"] + 3) + 8.0 * pb.n * (pb.p + 2))
    line = {
        "metric": METRIC, "value": 1.0 / sec, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == pk.FP64 else "f32-basis/f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload][1] +
                        (f" (tolerance overridden: tol={pb.tol:g})" if args.tol > 0.0 else ""),
            "n": pb.n, "nnz": int(pb.A.nnz), "p": pb.p, "t": pb.t, "tol": pb.tol,
            "workgroups": st["workgroups"], "lanczos": st["lanczos"],
            "csr_values": "f32" if vdt == np.float32 else "f64",
            "method": method_name(args),
            "solve_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms",
                                                "m_last", "fp64_steps",
                                                "fp32_error_estimate")},
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_solve (persistent solver: CSR products, Krylov steps, small "
                      "exponential, control)",
            "algorithmic_bytes_per_launch": st["bytes_ref"],
            "bytes_model": "reference plain-CGS2 model: per basis vector j+1 the CSR product "
                           "(s+4) nnz + 4(n+1) + 2 s n plus (4(j+1)+8) s n (Arnoldi) or 16 s n "
                           "(Lanczos); per step p products + 3p vectors (w-recurrence) and "
                           "(p+m+2) vectors (update)",
            "streamed_bytes_per_launch": st["bytes"],
            "frac_streamed": st["bytes"] / sec / 1e9 / HBM_PEAK_GBS,
            "working_set_bytes": work_set,
            "fits_infinity_cache": bool(work_set <= INFINITY_CACHE_BYTES),
        },
    }
    if traffic_src:
        line["roofline"]["traffic_source"] = traffic_src
    if st.get("krylov_seconds", 0.0) > 0.0:
        # the Krylov builds alone (CSR products + orthogonalisation), timed on
        # the device by the solve's first workgroup in an untimed solve
        kb, ks = st["krylov_bytes_ref"], st["krylov_seconds"]
        line["roofline"]["krylov_phase"] = {
            "bytes_ref": kb, "seconds": ks, "achieved": kb / ks / 1e9,
            "frac": kb / ks / 1e9 / HBM_PEAK_GBS, "share_of_solve": ks / sec}
    if not args.no_cpu:
        log(f"{args.workload}: CPU oracle")
        ref, base = oracle_reference(pb)
        line["err_vs_oracle"] = rel_err(u_gpu, ref)
        line["cpu_baseline"] = base
    if with_headline and not args.no_headline:
        line["headline"] = run_calls_block(args, calls=args.calls, warmup=1,
                                           oracle_calls=not args.no_cpu)
    print(json.dumps(line), flush=True)


CALL_VARIANTS = [
    # name, basis, proposer, warm start
    ("plain-fp64-cold", "fp64", False, False),
    ("plain-fp64-warm", "fp64", False, True),
    ("learned-fp64", "fp64", True, False),
    ("plain-fp32", "fp32", False, False),
    ("learned-fp32", "fp32", True, False),
]


def run_calls_block(args, calls, warmup, oracle_calls=True):
    """Successive calls on the 1024^2 reaction-diffusion operator with new
    right-hand sides (call c draws b from seed 5000 + c), t = 1e-3, tol = 1e-6,
    in every variant; calls/s from HIP events around all calls, the step
    counters from an untimed repeat, and the relative error against the oracle
    on evenly spaced calls."""
    import torch
    import paper_0907_4631_amd as pk
    from paper_0907_4631_amd import proposer as PR
    import workloads as W
    A = W.config5_matrix()
    n = A.shape[0]
    t, tol = 1e-3, 1e-6
    Ad = pk.DeviceCSR(A)
    bs = [torch.as_tensor(np.ascontiguousarray(W.config5_b(c, n).T), device="cuda")
          for c in range(calls)]
    weights = PR.load()
    check = sorted(set(np.linspace(0, calls - 1, min(calls, 6)).astype(int).tolist()))
    res, outs = {}, {}
    for name, basis, learned, warm in CALL_VARIANTS:
        log(f"call sequence: variant {name}, {calls} calls")
        s = pk.Solver(Ad, 2, tol=tol, precision=pk.FP32_BASIS if basis == "fp32" else pk.FP64,
                      **fixed_m_kw(args))
        hist = torch.zeros(4, dtype=torch.float64, device="cuda")
        if warm:
            s.opts.history = hist.data_ptr()
        if learned:
            s.opts.proposer = weights.data_ptr()
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        for w in range(max(1, warmup)):
            s(t, bs[w % calls], u, stats=False)
        hist.zero_()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for c in range(calls):
            s(t, bs[c], u, stats=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / calls
        if pk.lib().phipm_last_status() != 0:
            raise pk.PhipmError(pk.lib().phipm_last_status(), name)
        hist.zero_()
        tot = {"steps": 0, "rejected": 0, "matvecs": 0, "fp64_steps": 0}
        outs[name] = {}
        for c in range(calls):   # counters (and the checked solutions) from an untimed repeat
            st = s(t, bs[c], u)
            for k in tot:
                tot[k] += st[k]
            if c in check:
                outs[name][c] = u.cpu().numpy()
        res[name] = {"ms_per_call": ms, "calls_per_s": 1e3 / ms, **tot}
    block = {"workload": WORKLOADS["reaction2d-1024-calls"][1], "calls": calls,
             "method": method_name(args),
             "timed_variant": "learned-fp32", "baseline_variant": "plain-fp64-cold",
             "variants": res}
    block["speedup_vs_plain_fp64"] = (res["learned-fp32"]["calls_per_s"] /
                                      res["plain-fp64-cold"]["calls_per_s"])
    if oracle_calls:
        import oracle
        oracle.build(force=False)
        errs = {name: [] for name in res}
        for c in check:
            log(f"call sequence: CPU oracle on call {c}")
            ref, _ = oracle.phipm(t, A, W.config5_b(c, n), tol=tol)
            for name in res:
                errs[name].append(rel_err(outs[name][c], ref))
        for name in res:
            res[name]["max_err_vs_oracle"] = max(errs[name])
            res[name]["mean_err_vs_oracle"] = float(np.mean(errs[name]))
        block["err_checked_calls"] = check
    return block


def run_calls(args):
    block = run_calls_block(args, calls=args.steps, warmup=args.warmup,
                            oracle_calls=not args.no_cpu)
    v = block["variants"]["learned-fp32"]
    line = {
        "metric": METRIC, "value": v["calls_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": v["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-basis/f64", "data": "synthetic",
        "config": {"workload": block["workload"], "method": block["method"], "n": 1048576,
                   "calls": args.steps,
                   "variants": block["variants"],
                   "speedup_vs_plain_fp64": block["speedup_vs_plain_fp64"]},
    }
    print(json.dumps(line), flush=True)


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
        ig.run(max(1, args.warmup), stats=True)        # untimed, then restart from u0
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
    cpu = err = None
    if not args.no_cpu:
        # the first steps against the same integrator driven by the CPU oracle
        # (also its time per step on the host cores)
        import oracle
        import scipy.sparse as sp
        oracle.build(force=False)
        k = 3
        log(f"integrator: {k} steps with the CPU oracle")
        u = np.array(u0, dtype=np.float64)
        t0 = time.perf_counter()
        for _ in range(k):
            F = lap @ u + u - u ** 3
            J = sp.csr_matrix(lap + sp.diags(1.0 - 3.0 * u * u))
            J.sort_indices()
            du, _ = oracle.phipm(h, J, np.stack([np.zeros(N * N), F], axis=1), tol=tol, symm=1)
            u = u + du
        sec = (time.perf_counter() - t0) / k
        cpu = {"value": 1.0 / sec, "unit": "solves/s", "cores": oracle.threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"the first {k} integrator steps (plain step control)"}
        err = {"steps": k}
        for name in ("learned", "plain-cold"):
            kw = {"proposer": PR.load()} if name == "learned" else {}
            ig = integrator.AllenCahnERE(lap, u0, h, tol=tol, **kw)
            ig.run(k)
            g = ig.u.cpu().numpy()
            err[name] = float(np.linalg.norm(g - u) / np.linalg.norm(u))
    line = {
        "metric": METRIC, "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["allencahn-1024-ere"][1], "n": N * N, "h": h,
                   "integrator_steps": steps, "variants": res},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
        line["err_vs_oracle"] = err
    print(json.dumps(line), flush=True)


def cpu_baseline_batch(probs, gpu_stats, us=None, budget_s=20.0, seed=7):
    """The oracle on the host cores, timed on a seeded random sample of the
    batch's instances (about budget_s of CPU work) and scaled to the whole
    batch by rows x products (the GPU run's product counts).  With the GPU's
    outputs us, also the error of those instances against the oracle: the
    largest ||u - u_ref|| / (10 tol max(1, ||u_ref||)) (the batch's parity
    gate; below 1 passes) and the largest relative 2-norm error."""
    import oracle
    oracle.build(force=False)
    order = np.random.default_rng(seed).permutation(len(probs))
    spent, work_done, done = 0.0, 0.0, 0
    worst_gate, worst_rel = 0.0, 0.0
    for i in order:
        pb = probs[i]
        w = pb.n * max(1, gpu_stats[i]["matvecs"])
        t0 = time.perf_counter()
        ref, _ = oracle.phipm(pb.t, pb.A, pb.b, tol=pb.tol)
        spent += time.perf_counter() - t0
        work_done += w
        done += 1
        if us is not None:
            u = us[i].cpu().numpy()
            nr = float(np.linalg.norm(ref))
            d = float(np.linalg.norm(u - ref))
            worst_gate = max(worst_gate, d / (10.0 * pb.tol * max(1.0, nr)))
            worst_rel = max(worst_rel, d / max(nr, 1e-300))
        if spent > budget_s:
            break
    total = sum(pb.n * max(1, s["matvecs"]) for pb, s in zip(probs, gpu_stats))
    per_batch = spent * total / work_done
    out = {"value": len(probs) / per_batch, "unit": "solves/s", "cores": oracle.threads(),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{done} randomly chosen of the {len(probs)} instances ({spent:.1f} s), "
                     f"scaled to the batch by rows x products"}
    if us is not None:
        out["sampled_err"] = {"instances": done, "max_err_over_gate": worst_gate,
                              "max_rel_err": worst_rel}
    return out


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
                   precision=precision, workgroups=args.workgroups, **fixed_m_kw(args),
                   plan_opts=pk.default_plan_opts(autotune=0 if args.no_tune else 1, graph=1))
    create_s = time.perf_counter() - t0
    info = plan.info()
    log(f"batch: plan made in {create_s:.1f} s; {args.warmup} warmup + {args.steps} timed runs")
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
    nref = sum(s["bytes_ref"] for s in st)
    nbytes = sum(s["bytes"] for s in st)
    achieved = nref / (ms / 1e3) / 1e9
    line = {
        "metric": METRIC, "value": len(probs) / (ms / 1e3), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == pk.FP64 else "f32-basis/f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS["convdiff2d-batch256"][1],
            "method": method_name(args),
            "instances": len(probs), "rows": int(sum(pb.n for pb in probs)),
            "nnz": int(sum(pb.A.nnz for pb in probs)),
            "plan": {k: info[k] for k in ("teams", "class_size", "class_teams", "graph",
                                          "cooperative", "candidates", "max_team", "alpha",
                                          "tuned_ms", "default_ms")},
            "plan_create_s": create_s,
            "solve_stats": {"steps": sum(s["steps"] for s in st),
                            "rejected": sum(s["rejected"] for s in st),
                            "matvecs": sum(s["matvecs"] for s in st),
                            "fp64_steps": sum(s["fp64_steps"] for s in st)},
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_batch (persistent batched solver)",
            "algorithmic_bytes_per_launch": nref,
            "streamed_bytes_per_launch": nbytes,
            "frac_streamed": nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        },
    }
    if not args.no_cpu:
        log("batch: CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline_batch(probs, st, us)
        line["err_vs_oracle"] = line["cpu_baseline"]["sampled_err"]
    print(json.dumps(line), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff2d-512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-headline", action="store_true",
                    help="default workload: skip the 200-call learned + FP32 comparison")
    ap.add_argument("--calls", type=int, default=200,
                    help="calls of the headline comparison (default 200)")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="basis precision (default: the workload's)")
    ap.add_argument("--values", choices=["f64", "f32"], default=None,
                    help="CSR value type on the device (default: the workload's; float32 only "
                         "when every value is exact in float32)")
    ap.add_argument("--no-tune", action="store_true", help="batched workload: skip the autotuner")
    ap.add_argument("--fixed-m", type=int, default=0, metavar="M",
                    help="the paper's phip (Krylov dimension fixed at M, only tau adapted) "
                         "instead of phipm, for any workload but the integrator")
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
    if args.values is None:
        args.values = WORKLOADS[args.workload][3]
    if args.workload == "convdiff2d-batch256":
        run_batch(args)
    elif args.workload == "reaction2d-1024-calls":
        run_calls(args)
    elif args.workload == "allencahn-1024-ere":
        run_integrator(args)
    else:
        run_single(args, with_headline=args.workload == "convdiff2d-512")
    # release the library's device resources while the runtime is up
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
