"""Write single_oracle_samples.json: the CPU oracle's solutions of the three
full-size single-solve workloads (512^2 convection-diffusion, 128^3 Laplacian,
call 0 of the 1024^2 reaction-diffusion sequence), each reduced to its 2-norm
and 64 entries at seeded positions.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_single_golden.py  (the 512^2 solve
takes several minutes on 8 cores)."""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_oracle_samples.json")
SAMPLES = 64


def problems():
    import workloads as W
    p2 = W.config2()
    p3 = W.config3()
    A5 = W.config5_matrix()
    b5 = W.config5_b(0, A5.shape[0])
    return [("convdiff2d-512", p2.A, p2.b, p2.t, p2.tol, 9002),
            ("laplace3d-128", p3.A, p3.b, p3.t, p3.tol, 9003),
            ("reaction2d-1024-call0", A5, b5, 1e-3, 1e-6, 9005)]


def main():
    import oracle
    import workloads as W
    oracle.build(force=False)
    recs = []
    for name, A, b, t, tol, seed in problems():
        t0 = time.time()
        u, st = oracle.phipm(t, A, b, tol=tol)
        idx = W.rng(seed).integers(0, A.shape[0], SAMPLES)
        recs.append({"name": name, "n": int(A.shape[0]), "p": int(b.shape[1] - 1), "t": t,
                     "tol": tol, "unorm": float(np.linalg.norm(u)),
                     "samples": [[int(k), float(u[k])] for k in idx],
                     "oracle_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms")},
                     "oracle_seconds": round(time.time() - t0, 1)})
        print(name, recs[-1]["oracle_stats"], recs[-1]["oracle_seconds"], "s", flush=True)
    doc = {"about": "CPU oracle (FP64, default options) on the full-size single-solve "
                    "workloads: 2-norm and 64 sampled entries each",
           "records": recs}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
