"""Run the FFT product of a named workload a number of times, for profilers.

Also runs a plain device-to-device copy of a known number of bytes, so that a
counter such as FETCH_SIZE or WRITE_SIZE can be calibrated against traffic
whose size is exact (copy of B bytes: B read, B written).

    python -m paper_1305_6497_amd.profile_matvec block_64 --reps 20 --precision mixed
"""

import argparse
import json
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_args()

    import torch

    import inputs
    import paper_1305_6497_amd as dda

    w = inputs.WORKLOADS[args.workload]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    n = len(sites)
    kd = dda.kd_from_x(w["x"], n)
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1 + (i % 2)) for i in range(args.nrhs)]
    P = torch.tensor(inputs.random_polarization(n, args.nrhs, seed=3), device="cuda")
    out = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        out = t.apply(rhs, P, args.precision)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.reps
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    info = t.info()
    print(json.dumps(dict(workload=args.workload, precision=args.precision, nrhs=args.nrhs, reps=args.reps,
                          ms_per_product=dt * 1e3, box=info["box"], grid=info["grid"], n_sites=n,
                          copy_bytes=nbytes, checksum=float(out.abs().sum().item()))))
    t.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
