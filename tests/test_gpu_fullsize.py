"""The full-size single-solve workloads in the benchmark's launch
configuration (default options, one workgroup per CU) against the CPU oracle
run live on the same inputs.

Gate (the parity target): the relative 2-norm error of the whole solution,
||u - u_ref||_2 <= 10 tol ||u_ref||_2.  Each case also checks the oracle's
2-norm and 64 seeded entries stored in tests/golden/single_oracle_samples.json
(written by make_single_golden.py in that folder, which calls only the
oracle), so a change of the oracle itself shows up too."""
import json
import os
import time

import numpy as np
import pytest

import oracle
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
    oracle.build(force=False)
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


_REFS = {}


def reference(name):
    """The oracle's solution, computed once per name."""
    if name not in _REFS:
        A, b, t, tol = problem(name)
        t0 = time.perf_counter()
        u, st = oracle.phipm(t, A, b, tol=tol)
        print(f"  oracle {name}: {time.perf_counter() - t0:.1f} s on {oracle.threads()} threads,"
              f" stats {st}", flush=True)
        _REFS[name] = u
    return _REFS[name]


def check(name, u, tol):
    ref = reference(name)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    print(f"  {name}: relative 2-norm error vs oracle {err:.3e} (gate {10 * tol:.0e}),"
          f" ||u_ref|| = {np.linalg.norm(ref):.6g}", flush=True)
    assert err <= 10.0 * tol, err
    rec = records()[name]
    assert abs(np.linalg.norm(ref) - rec["unorm"]) <= 1e-9 * rec["unorm"]
    for k, v in rec["samples"]:
        assert abs(ref[k] - v) <= 1e-9 * max(1.0, rec["unorm"]), (k, ref[k], v)
    return err


def run(pk, name, precision=None, val_dtype=np.float64, proposer=None, **kw):
    A, b, t, tol = problem(name)
    Ad = pk.DeviceCSR(A, dtype=val_dtype)
    bd = torch.as_tensor(np.ascontiguousarray(b.T), device="cuda")
    u = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    s = pk.Solver(Ad, b.shape[1] - 1, tol=tol,
                  precision=pk.FP64 if precision is None else precision, validate=1, **kw)
    if proposer is not None:
        s.opts.proposer = proposer.data_ptr()
    st = s(t, bd, u)
    torch.cuda.synchronize()
    print("  gpu", {k: st[k] for k in ("steps", "rejected", "matvecs", "workgroups",
                                       "fp64_steps")}, flush=True)
    assert st["status"] == 0
    return u.cpu().numpy(), st, tol


@pytest.mark.parametrize("name", ["convdiff2d-512", "laplace3d-128", "reaction2d-1024-call0"])
def test_full_size_matches_oracle(pk, name):
    print("full-size case", name, flush=True)
    u, st, tol = run(pk, name)
    check(name, u, tol)


def test_full_size_learned_proposer_meets_gate(pk):
    """The benchmark's timed variant of the call sequence: the committed
    network seeding every step."""
    from paper_0907_4631_amd import proposer as PR
    print("full-size case reaction2d-1024-call0 learned", flush=True)
    u, st, tol = run(pk, "reaction2d-1024-call0", proposer=PR.load())
    assert st["proposals"] > 0
    check("reaction2d-1024-call0", u, tol)


def test_full_size_fp32_basis_request_builds_fp64_steps(pk):
    """The 128^3 Laplacian with the FP32 basis requested: the phi-part of
    eq. step is far larger than u there, so every step's a-priori rounding
    bound exceeds the budget and the step is built with the FP64 basis; the
    result meets the same gate."""
    print("full-size case laplace3d-128 fp32 basis requested", flush=True)
    u, st, tol = run(pk, "laplace3d-128", precision=pk.FP32_BASIS, val_dtype=np.float32)
    assert st["steps"] >= 1 and st["fp64_steps"] == st["steps"]
    check("laplace3d-128", u, tol)
