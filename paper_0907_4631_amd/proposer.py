"""Training pipeline of the learned (tau, m) proposer, on the GPU.

1. Traces: the plain adaptive solver (FP64 basis) records every accepted
   step (features at the start of the step, the step's outcome and its
   Hessenberg matrix) on a family of problems of the kinds of the three
   single-solve workloads: 2D 5-point Laplacians, 2D upwind
   convection-diffusion and 3D 7-point Laplacians, over ranges of size, t,
   tol and p.
2. Labels: hindsight (tau*, m*) of every recorded step (phipm_label_steps),
   the pair of least time per unit of t under a time model of the step on
   this device: barrier latency and streaming bandwidth of the solver (from
   its roofline measurements) and the small exponential's time per order,
   timed here on the device.
3. Training: Adam on the mean squared error (phipm_mlp_train), with a
   held-out tenth of the rows for validation.

Every numeric step runs in the library's kernels; this module only chooses
the problems and moves tensors.  Command line:

    python -m paper_0907_4631_amd.proposer --out paper_0907_4631_amd/proposer_weights.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import (FP64, M_CAP, MLP_IN, MLP_OUT, MLP_PARAMS, P_MAX, DeviceCSR, LabelCosts, Solver,
               alloc_trace, expm, label_steps, mlp_forward, mlp_train)

# Solver timing constants on MI355X (one 1024-thread workgroup per CU), fitted
# to the phase clocks of the solver for the step-time model of the labels.
# The model counts three team synchronisations and (4K + 8) vectors of
# traffic per Krylov step; the solver does one reduction and one neighbour
# synchronisation (about 15 us together on the full grid) and streams about
# half those bytes, so the constants are per modelled synchronisation and per
# modelled byte: 5 us, and 7.5e12 (3e10 per workgroup) modelled bytes/s.  One
# workgroup alone synchronises in 1.5 us.
SYNC_S = 5e-6
SYNC1_S = 1.5e-6
BW_BYTES_PER_S = 7.5e12
WG_BYTES_PER_S = 3.0e10

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "proposer_weights.npy")


def _workloads():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads
    return workloads


def training_problems(count: int = 96, seed: int = 6000, scale: float = 1.0):
    """Seeded list of (name, A, b, t, tol) covering the three operator
    families.  scale < 1 shrinks the grids (for quick runs)."""
    W = _workloads()
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        fam = i % 3
        p = int(g.integers(0, 4))
        tol = float(10.0 ** -g.integers(6, 9))
        if fam == 0:
            N = int(max(8, round(int(g.choice([30, 64, 128, 256])) * scale)))
            A = W.laplace2d(N)
            t = float(10.0 ** g.uniform(-4.0, -1.0))
            name = f"lap2d-{N}"
        elif fam == 1:
            N = int(max(8, round(int(g.choice([64, 128, 256, 512])) * scale)))
            v = float(g.choice([10.0, 35.0, 50.0, 70.0]))
            A = W.convdiff2d(N, v, v)
            t = float(10.0 ** g.uniform(-3.0, -1.5))
            name = f"convdiff-{N}-v{v:g}"
        else:
            N = int(max(6, round(int(g.choice([32, 64, 128])) * scale)))
            A = W.laplace3d(N)
            t = float(10.0 ** g.uniform(-4.5, -2.5))
            name = f"lap3d-{N}"
        b = W.rng(seed + 1000 + i).standard_normal((A.shape[0], p + 1))
        out.append((f"{name}-p{p}-t{t:.2g}-tol{tol:g}", A, b, t, tol))
    return out


def measure_costs(device="cuda", workgroups: int = 256) -> LabelCosts:
    """Time model of a solver step: the constants above and the small
    exponential's time for every order N (timed on the device at a set of
    orders, linear in between)."""
    import torch
    Ns = [2, 4, 8, 12, 16, 24, 32, 48, 64, 80, 92, 93, 100, 110, 120, 128, M_CAP + P_MAX + 1]
    g = np.random.default_rng(1)
    t = []
    for N in Ns:
        H = torch.as_tensor(g.standard_normal((N, N)) * 30.0 / np.sqrt(N), device=device)
        for _ in range(2):
            expm(H)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(8):
            expm(H)
        e1.record()
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1) / 8 / 1e3)
    c = LabelCosts()
    c.sync_s, c.sync1_s = SYNC_S, SYNC1_S
    c.bw_bytes_per_s, c.wg_bytes_per_s = BW_BYTES_PER_S, WG_BYTES_PER_S
    c.workgroups = workgroups
    table = np.interp(np.arange(M_CAP + P_MAX + 2), Ns, t)
    for i, v in enumerate(table):
        c.expm_s[i] = float(v)
    return c


def collect(problems, cap: int = 512, device="cuda", costs=None, log=None):
    """Traces of the plain FP64 solver on `problems`, labelled (under the
    time model `costs`, or eq. 4 if None).  Returns (X, T) float32 device
    tensors and per-problem stats."""
    import torch
    trace = alloc_trace(cap, device=device)
    Xs, Ts, info = [], [], []
    for name, A, b, t, tol in problems:
        Ad = DeviceCSR(A, device=device)
        bd = torch.as_tensor(np.ascontiguousarray(b.T), device=device)
        u = torch.empty(A.shape[0], dtype=torch.float64, device=device)
        s = Solver(Ad, b.shape[1] - 1, tol=tol, precision=FP64)
        s.opts.trace = trace.data_ptr()
        s.opts.trace_cap = cap
        st = s(t, bd, u)
        k = min(cap, st["trace_len"])
        if k > 0:
            X, T = label_steps(trace, k, costs)
            Xs.append(X.clone())
            Ts.append(T.clone())
        info.append({"name": name, "steps": st["steps"], "rejected": st["rejected"],
                     "matvecs": st["matvecs"], "records": k})
        if log:
            log(f"  trace {name}: {st['steps']} steps, {st['rejected']} rejected, {k} records")
    torch.cuda.synchronize()
    return torch.cat(Xs), torch.cat(Ts), info


def init_params(seed: int = 0, device="cuda"):
    """Glorot-uniform weights and zero biases (drawn on the host, seeded)."""
    import torch
    g = np.random.default_rng(seed)
    P = np.zeros(MLP_PARAMS, dtype=np.float32)
    off = 0
    for fan_out, fan_in in ((64, MLP_IN), (64, 64), (MLP_OUT, 64)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        P[off:off + fan_out * fan_in] = g.uniform(-lim, lim, fan_out * fan_in)
        off += fan_out * fan_in + fan_out
    return torch.as_tensor(P, device=device)


def train(X, T, epochs: int = 400, lr: float = 2e-3, batch: int = 64, seed: int = 0,
          holdout: float = 0.1, log=None):
    """Shuffle (seeded), hold out a validation tenth, train with Adam.
    Returns (params, history dict)."""
    import torch
    rows = X.shape[0]
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(rows), device=X.device)
    X, T = X[perm].contiguous(), T[perm].contiguous()
    nv = int(rows * holdout) if rows >= 20 else 0
    Xv, Tv = X[:nv], T[:nv]
    Xt, Tt = X[nv:].contiguous(), T[nv:].contiguous()
    P = init_params(seed, device=X.device)
    am = torch.zeros_like(P)
    av = torch.zeros_like(P)
    hist = {"train": [], "val": []}
    done, step = 0, 0
    per_call = 50
    while done < epochs:
        e = min(per_call, epochs - done)
        loss = mlp_train(P, am, av, Xt, Tt, e, lr=lr, batch=batch, step0=step)
        step += e * ((Xt.shape[0] + batch - 1) // batch)
        done += e
        hist["train"] += loss.cpu().tolist()
        if nv:
            Y = mlp_forward(P, Xv.contiguous())
            hist["val"].append((done, float(((Y - Tv) ** 2).sum() / (2 * nv))))
        if log:
            log(f"  epoch {done}: train {hist['train'][-1]:.4g}"
                + (f" val {hist['val'][-1][1]:.4g}" if nv else ""))
    return P, hist


def save(params, path: str = DEFAULT_WEIGHTS):
    np.save(path, params.detach().cpu().numpy().astype(np.float32))


def load(path: str = DEFAULT_WEIGHTS, device="cuda"):
    import torch
    P = np.load(path, allow_pickle=False)
    if P.dtype != np.float32 or P.shape != (MLP_PARAMS,):
        raise ValueError(f"{path}: expected {MLP_PARAMS} float32 parameters")
    return torch.as_tensor(P, device=device)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--problems", type=int, default=288)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    say = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    costs = measure_costs()
    say("exponential time per order: " + ", ".join(
        f"{N}: {costs.expm_s[N] * 1e6:.0f} us" for N in (8, 32, 64, 100, 128)))
    X, T, info = collect(training_problems(args.problems, scale=args.scale), costs=costs, log=say)
    say(f"{X.shape[0]} labelled steps from {len(info)} solves in {time.time() - t0:.1f} s")
    t1 = time.time()
    P, hist = train(X, T, epochs=args.epochs, lr=args.lr, seed=args.seed, log=say)
    say(f"trained in {time.time() - t1:.1f} s")
    save(P, args.out)
    say(f"wrote {args.out}")


if __name__ == "__main__":
    main()
