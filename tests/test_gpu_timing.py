"""Pass timing inside solves: it times the products a solve launches and changes none of its results."""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _target():
    import paper_1305_6497_amd as dda
    sites, box = dda.make_sites("RCTGLPRSM", (20, 16, 12))
    t = dda.Target(sites, box, m=1.5 + 0.1j, kd=0.3)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1), dda.orient_rhs(0.0, 0.0, 0.0, which=2)]
    return t, rhs


def test_pass_timing_inside_solves():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    t, rhs = _target()
    P0, st0 = t.solve(rhs, tol=1e-6, precision="mixed", solver="cocg")
    P0 = P0.clone()
    t.set_pass_timing(1)
    P1, st1 = t.solve(rhs, tol=1e-6, precision="mixed", solver="cocg")
    avg, n = t.pass_timing("mixed")
    avg64, n64 = t.pass_timing("fp64")
    assert torch.equal(P0, P1)                     # events change no result
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    # one batched FP32 product per COCG iteration of the slowest RHS, one FP64 product per host check
    assert n >= max(s["iters"] for s in st1) and n > 0, (n, st1)
    assert n64 >= max(s["outer"] for s in st1) >= 1, (n64, st1)
    for k in ("x_forward", "y_forward", "z_pass", "y_inverse", "x_inverse"):
        assert avg[k] > 0.0 and avg64[k] > 0.0, (k, avg, avg64)
    assert abs(avg["total"] - sum(avg[k] for k in avg if k != "total")) < 1e-9
    # sampling every 3rd product (FP32 and FP64 in launch order) times about a third of the FP32 ones
    t.set_pass_timing(3)
    t.solve(rhs, tol=1e-6, precision="mixed", solver="cocg")
    _, n3 = t.pass_timing("mixed")
    assert abs(n3 - n / 3) <= n64 + 2, (n3, n, n64)
    # off: nothing is timed; products replayed from a captured graph are not timed either
    t.set_pass_timing(0)
    t.solve(rhs, tol=1e-6, precision="mixed", solver="cocg")
    assert t.pass_timing("mixed")[1] == 0
    t.set_pass_timing(1)
    Pg, stg = t.solve(rhs, tol=1e-6, precision="mixed", solver="bicgstab", use_graph=True, check_every=8)
    assert all(s["status"] == 0 for s in stg)
    assert t.pass_timing("mixed")[1] == 0
    assert t.pass_timing("fp64")[1] >= 1
    t.close()
