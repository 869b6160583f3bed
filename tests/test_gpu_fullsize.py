"""The full-size single-solve workloads in the benchmark's launch
configuration (default options, one workgroup per CU) against the CPU
oracle's solutions, stored as their 2-norm and 64 seeded entries in
tests/golden/single_oracle_samples.json (written by make_single_golden.py in
that folder, which calls only the oracle).

Gate: |u_k - u_ref,k| and | ||u|| - ||u_ref|| | at most 10 tol max(1, ||u_ref||),
both implied by the 2-norm gate of the other parity tests."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "single_oracle_samples.json")


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_4631_amd as pk
    pk.lib()
    return pk


def records():
    with open(GOLD) as f:
        return {r["name"]: r for r in json.load(f)["records"]}


def problem(name):
    if name == "convdiff2d-512":
        pb = W.config2()
        return pb.A, pb.b, pb.t, pb.tol
    if name == "laplace3d-128":
        pb = W.config3()
        return pb.A, pb.b, pb.t, pb.tol
    A = W.config5_matrix()
    return A, W.config5_b(0, A.shape[0]), 1e-3, 1e-6


def check(u, rec):
    gate = 10.0 * rec["tol"] * max(1.0, rec["unorm"])
    assert abs(np.linalg.norm(u) - rec["unorm"]) <= gate
    for k, v in rec["samples"]:
        assert abs(u[k] - v) <= gate, (k, u[k], v, gate)


@pytest.mark.parametrize("name", ["convdiff2d-512", "laplace3d-128", "reaction2d-1024-call0"])
def test_full_size_matches_oracle_samples(pk, name):
    print("full-size case", name, flush=True)
    rec = records()[name]
    A, b, t, tol = problem(name)
    assert A.shape[0] == rec["n"] and b.shape[1] - 1 == rec["p"]
    Ad = pk.DeviceCSR(A)
    bd = torch.as_tensor(np.ascontiguousarray(b.T), device="cuda")
    u = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    s = pk.Solver(Ad, rec["p"], tol=tol, precision=pk.FP64, validate=1)
    st = s(t, bd, u)
    torch.cuda.synchronize()
    print("  gpu", {k: st[k] for k in ("steps", "rejected", "matvecs", "workgroups")},
          "oracle", rec["oracle_stats"], flush=True)
    assert st["status"] == 0
    check(u.cpu().numpy(), rec)


def test_full_size_learned_proposer_meets_gate(pk):
    """The benchmark's timed variant of the call sequence: the committed
    network seeding every step."""
    from paper_0907_4631_amd import proposer as PR
    rec = records()["reaction2d-1024-call0"]
    A, b, t, tol = problem("reaction2d-1024-call0")
    Ad = pk.DeviceCSR(A)
    bd = torch.as_tensor(np.ascontiguousarray(b.T), device="cuda")
    u = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    weights = PR.load()
    s = pk.Solver(Ad, rec["p"], tol=tol, precision=pk.FP64)
    s.opts.proposer = weights.data_ptr()
    st = s(t, bd, u)
    torch.cuda.synchronize()
    assert st["status"] == 0 and st["proposals"] > 0
    check(u.cpu().numpy(), rec)
