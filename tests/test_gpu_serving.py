"""Serving on the GPU: every result is the same alone and in the concurrent mix."""

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_results_identical_alone_and_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1305_6497_amd as dda
    from paper_1305_6497_amd.serving import GpuExecutor, Request, Server

    shapes = [("ELLIPSOID", (18, 18, 18)), ("CYLINDER1", (20, 14, 1)), ("HEX_PRISM", (16, 21, 1)),
              ("ELLIPSOID", (24, 17, 13)), ("RCTGLPRSM", (12, 16, 20)), ("ELLIPSOID", (30, 30, 30)),
              ("CYLINDER1", (26, 18, 1)), ("HEX_PRISM", (22, 17, 1))]
    reqs = [Request(id=i, arrival=0.003 * i, shape=s, shpar=p, m=complex(1.3 + 0.1 * i, 0.02 * i), x=2.0 + 0.5 * i)
            for i, (s, p) in enumerate(shapes)]
    ex = GpuExecutor(tol=1e-6)
    alone = {r.id: Server(ex, slots=1).run([Request(**{**r.__dict__, "arrival": 0.0})])[r.id] for r in reqs}
    for rep in range(3):
        mix = Server(ex, slots=4).run(reqs)
        overlapped = sum(1 for i in range(1, len(reqs)) if mix[i].admitted < mix[i - 1].done)
        assert overlapped >= 1                      # requests really ran concurrently
        for r in reqs:
            a, b = alone[r.id], mix[r.id]
            assert not a.error and not b.error, (a.error, b.error)
            assert all(s["status"] == 0 for s in a.stats + b.stats)
            for qa, qb in zip(a.q, b.q):
                assert qa == qb, (rep, r.id, qa, qb)   # bit-identical: deterministic reductions, private buffers
