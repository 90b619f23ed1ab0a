"""The allocation-free product (dda_apply_noalloc) against dda_apply on the GPU.

dda_apply_noalloc runs the same kernels as dda_apply on work buffers held in a
static device array, so its output must equal dda_apply's bit for bit.  Two
calls follow each other on the shared array, the second on a smaller input,
so a result that depended on what an earlier call left there would show.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _setup(dda, shape, shpar, m, x, comp=False):
    sites, box = dda.make_sites(shape, shpar)
    kd = dda.kd_from_x(x, len(sites))
    if comp:
        cid = (sites[:, 0] < box[0] // 2).astype(np.uint8)
        return dda.Target(sites, box, m=[m, 1.2 + 0.02j], kd=kd, comp=cid), len(sites)
    return dda.Target(sites, box, m=m, kd=kd), len(sites)


CASES = [  # (shape, shpar, m, x, nrhs, two compositions); the second is smaller
    ("RCTGLPRSM", (40, 24, 20), 1.5 + 0.1j, 6.0, 3, True),
    ("ELLIPSOID", (10.2, 10.2, 10.2), 1.33 + 0.01j, 1.0, 1, False),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_product_equals_apply(precision):
    import torch

    import inputs
    import paper_1305_6497_amd as dda
    for shape, shpar, m, x, nrhs, comp in CASES:
        print("noalloc", precision, shape, shpar, nrhs, flush=True)
        t, n = _setup(dda, shape, shpar, m, x, comp)
        bytes0 = t.info()["device_bytes"]
        rhs = [dda.orient_rhs(0.3 * i, 0.7, 0.2 * i, which=1 + i % 2) for i in range(nrhs)]
        P = torch.tensor(inputs.random_polarization(n, nrhs, seed=7), device="cuda")
        out = torch.full_like(P, float("nan"))
        t.apply_noalloc(rhs, P, out, precision)
        torch.cuda.synchronize()
        assert t.info()["device_bytes"] == bytes0          # no workspace of the handle was grown
        ref = t.apply(rhs, P, precision)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (precision, shape, float((out - ref).abs().max()))
        t.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch

    import inputs
    import paper_1305_6497_amd as dda
    print("noalloc limits", flush=True)
    t, n = _setup(dda, "RCTGLPRSM", (64, 64, 64), 1.5 + 0.1j, 10.0)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1)] * 2
    P = torch.tensor(inputs.random_polarization(n, 2, seed=3), device="cuda")
    out = torch.zeros_like(P)
    with pytest.raises(dda.DDAError) as e:                 # 2 x 75.5 MB of FP64 work buffers > 128 MiB
        t.apply_noalloc(rhs, P, out, "fp64")
    assert e.value.code == -4
    assert bool((out == 0).all())                          # nothing was queued
    t.apply_noalloc(rhs[:1], P[:1].contiguous(), out[:1], "fp64")       # one RHS fits
    torch.cuda.synchronize()
    ref = t.apply(rhs[:1], P[:1].contiguous(), "fp64")
    assert torch.equal(out[:1], ref)
    t.close()
    t, n = _setup(dda, "RCTGLPRSM", (6, 6, 6), 1.5 + 0.1j, 1.0)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1)] * 33
    P = torch.zeros((33, n, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dda.DDAError):                      # nrhs * n_comp > 32
        t.apply_noalloc(rhs, P, torch.zeros_like(P), "mixed")
    t.close()
