"""The GPU exponential Rosenbrock-Euler driver against the same driver on the
CPU oracle (test_integrator_pins.ere_oracle): plain step control, warm start
and the learned proposer, all within the accumulated gate of the steps."""
import numpy as np
import pytest

import workloads as W
from test_integrator_pins import ere_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_4631_amd as pk
    pk.lib()
    return pk


@pytest.mark.parametrize("variant", ["plain", "warm", "learned"])
def test_gpu_driver_matches_oracle_driver(pk, variant):
    from paper_0907_4631_amd import integrator
    from paper_0907_4631_amd import proposer as PR
    print("integrator variant", variant, flush=True)
    N, h, steps, tol = 48, 1e-3, 10, 1e-7
    lap = W.laplace2d(N)
    u0 = W.smooth_field(N, 5999)
    kw = {}
    if variant == "warm":
        kw["warm"] = True
    if variant == "learned":
        kw["proposer"] = PR.load()
    ig = integrator.AllenCahnERE(lap, u0, h, tol=tol, **kw)
    sts = ig.run(steps, stats=True)
    torch.cuda.synchronize()
    u = ig.u.cpu().numpy()
    ref = ere_oracle(lap, u0, h, steps, tol)
    # each call is within 10 tol max(1, ||du||) of the oracle's; over the steps
    # the differences add up (the map is Lipschitz with constant about 1)
    gate = 10 * tol * steps * max(1.0, np.linalg.norm(ref))
    print("  |u - ref|", np.linalg.norm(u - ref), "gate", gate,
          "matvecs", sum(s["matvecs"] for s in sts), flush=True)
    assert all(s["status"] == 0 and s["lanczos"] == 1 for s in sts)
    assert np.linalg.norm(u - ref) <= gate


def test_allen_cahn_update_matches_definition(pk):
    """phipm_allen_cahn_update against its definition in numpy: u += du, then
    F = L u + (u - u^3) and J's diagonal lap_diag + (1 - 3 u^2), on a grid of
    several tiles with a ragged last tile."""
    print("allen_cahn_update case 45x45", flush=True)
    lap = W.laplace2d(45).tocsr()
    lap.sort_indices()
    n = lap.shape[0]
    g = np.random.default_rng(3)
    u0 = g.uniform(-1.2, 1.2, n)
    du = g.standard_normal(n) * 1e-3
    rows = np.repeat(np.arange(n), np.diff(lap.indptr))
    diag = np.nonzero(lap.indices == rows)[0].astype(np.int32)
    L = pk.DeviceCSR(lap, device="cuda")
    J = pk.DeviceCSR(lap, device="cuda")
    u = torch.as_tensor(u0, device="cuda").clone()
    F = torch.empty(n, dtype=torch.float64, device="cuda")
    pk.allen_cahn_update(L, u, du=torch.as_tensor(du, device="cuda"),
                         diag_pos=torch.as_tensor(diag, device="cuda"),
                         lap_diag=torch.as_tensor(lap.data[diag], device="cuda"),
                         J_val=J.val, F=F)
    torch.cuda.synchronize()
    un = u0 + du
    assert np.array_equal(u.cpu().numpy(), un)
    Fr = lap @ un + (un - un * un * un)
    scale = np.abs(lap) @ np.abs(un) + np.abs(un) + np.abs(un) ** 3
    assert np.all(np.abs(F.cpu().numpy() - Fr) <= 1e-14 * scale)
    Jr = lap.data.copy()
    Jr[diag] = lap.data[diag] + (1.0 - 3.0 * un * un)
    Jg = J.val.cpu().numpy()
    off = np.ones(lap.nnz, dtype=bool)
    off[diag] = False
    assert np.array_equal(Jg[off], Jr[off])  # off-diagonal values untouched
    # (the device may contract 1 - 3u^2 into one fused multiply-add)
    tolJ = 1e-15 * (np.abs(lap.data[diag]) + 1.0 + 3.0 * un * un)
    assert np.all(np.abs(Jg[diag] - Jr[diag]) <= tolJ)
