"""phipm_noalloc, the entry point that allocates nothing (its workspace is the
library's fixed device scratch), against phipm() with a caller workspace,
through the C ABI: two calls in a row, the second on a smaller problem, each
equal to phipm()'s result bit for bit (the same kernels and launch shape on
the same inputs), and a problem too large for the scratch refused on the host
before any device work."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0907_4631_amd as pk
    pk.lib()
    return pk


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def both(pk, A, b, t, **kw):
    Ad = pk.DeviceCSR(A)
    bd = dev(b.T)
    u_ref, st_ref = pk.solve(t, Ad, bd, **kw)
    u = torch.full((A.shape[0],), np.nan, dtype=torch.float64, device="cuda")
    st = pk.solve_noalloc(t, Ad, bd, u, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st, u_ref.cpu().numpy(), st_ref


def test_noalloc_matches_phipm_on_two_calls(pk):
    print("noalloc: two calls, the second smaller", flush=True)
    assert pk.lib().phipm_noalloc_scratch_bytes() == 64 << 20
    g = np.random.default_rng(31)
    # first call: 96^2 convection-diffusion, p = 2 (several workgroups)
    A1 = W.convdiff2d(96, 40.0, 20.0)
    b1 = g.standard_normal((A1.shape[0], 3))
    u, st, r, sr = both(pk, A1, b1, 5e-3, tol=1e-8)
    assert st["status"] == 0 and sr["status"] == 0
    assert np.array_equal(u, r)
    assert (st["steps"], st["rejected"], st["matvecs"]) == (sr["steps"], sr["rejected"],
                                                            sr["matvecs"])
    # second call, smaller: 30^2 Laplacian, p = 1 (one workgroup), on the
    # scratch the first call left behind
    pb = W.config1()
    u, st, r, sr = both(pk, pb.A, pb.b, pb.t, tol=pb.tol)
    assert st["status"] == 0
    assert np.array_equal(u, r)
    assert st["matvecs"] == sr["matvecs"]


def test_noalloc_refuses_a_problem_larger_than_its_scratch(pk):
    print("noalloc: too large", flush=True)
    A = W.laplace2d(1024)                     # n = 1,048,576: V alone needs ~850 MB
    Ad = pk.DeviceCSR(A)
    b = torch.zeros((2, A.shape[0]), dtype=torch.float64, device="cuda")
    u = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
    with pytest.raises(pk.PhipmError) as e:
        pk.solve_noalloc(1e-3, Ad, b, u, tol=1e-6)
    assert e.value.status == pk.ESCRATCH
    assert torch.count_nonzero(u).item() == 0   # nothing was written
