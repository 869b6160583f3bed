"""Write config4_oracle_samples.json: the CPU oracle's solution of every
instance of the 256-instance convection-diffusion batch, reduced to its 2-norm
and eight entries at seeded positions.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_batch_golden.py  (about a minute
with 8 processes)."""
from __future__ import annotations

import json
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

TOL = 1e-7
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_oracle_samples.json")
SAMPLES = 8


def sample_positions(spec, n):
    import workloads as W
    return W.rng(spec.seed + 200000).integers(0, n, SAMPLES)


def one(i):
    import oracle
    import workloads as W
    spec = W.config4_specs()[i]
    pb = W.config4_problem(spec, tol=TOL)
    u, st = oracle.phipm(pb.t, pb.A, pb.b, tol=TOL)
    idx = sample_positions(spec, pb.n)
    return {"i": i, "N": spec.N, "p": spec.p, "t": spec.t, "peclet": spec.peclet,
            "n": pb.n, "unorm": float(np.linalg.norm(u)),
            "samples": [[int(k), float(u[k])] for k in idx],
            "oracle_stats": {k: st[k] for k in ("steps", "rejected", "matvecs", "expms")}}


def main():
    from multiprocessing import Pool
    import oracle
    oracle.build(force=False)
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        recs = sorted(pool.map(one, range(256)), key=lambda r: r["i"])
    doc = {"about": "CPU oracle (FP64, tol 1e-7, default options) on the 256 seeded "
                    "convection-diffusion instances: 2-norm and 8 sampled entries each",
           "tol": TOL, "instances": recs}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
