"""Run the FFT product of a named workload a number of times, for profilers.

Also runs a plain device-to-device copy of a known number of bytes, so that a
counter such as FETCH_SIZE or WRITE_SIZE can be calibrated against traffic
whose size is exact (copy of B bytes: B read, B written).

    python -m paper_1305_6497_amd.profile_matvec block_64 --reps 20 --precision mixed

``solve`` runs whole solves of a workload instead (kernel statistics of the
iteration):

    python -m paper_1305_6497_amd.profile_matvec solve sphere_d133 --nrhs 2 --solver cocg

``summarize`` turns two rocprofv3 counter runs of that command (one with
--pmc FETCH_SIZE, one with --pmc WRITE_SIZE, both -f csv) into HBM bytes per
launch of each kernel, each counter scaled so that the copy reads and writes
exactly its size:

    python -m paper_1305_6497_amd.profile_matvec summarize FETCH_DIR WRITE_DIR \
        --workload block_64 --kernel k_zpass --json profiles/x.json
"""

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
# Sources the FFT-product kernels are compiled from: a traffic figure measured
# on other sources no longer describes the kernel.
KERNEL_SOURCES = ("passes.hpp", "fft_lds.hpp", "dda_internal.hpp", "reduce.hpp", "matvec_f32.hip", "matvec_f32v.hip",
                  "matvec_f64.hip", "plan_tuned.inc")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _counter_rows(d, counter):
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not path:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path[0])):
        if r["Counter_Name"] != counter:
            continue
        name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("dda::", "").strip()
        out[name].append(float(r["Counter_Value"]) * 1024.0)          # KiB -> bytes
    return out


def summarize(args):
    fetch = _counter_rows(args.fetch_dir, "FETCH_SIZE")
    write = _counter_rows(args.write_dir, "WRITE_SIZE")
    copy_bytes = args.copy_mib << 20
    # the largest copyBuffer dispatch is the calibration copy
    cf = copy_bytes / max(v for k, vs in fetch.items() if "copyBuffer" in k for v in vs)
    cw = copy_bytes / max(v for k, vs in write.items() if "copyBuffer" in k for v in vs)
    rows = {}
    for k in fetch:
        if not k.startswith("k_"):
            continue
        fb = cf * sum(fetch[k]) / len(fetch[k])
        wb = cw * sum(write[k]) / len(write[k]) if k in write else 0.0
        rows[k] = dict(launches=len(fetch[k]), fetch_bytes=fb, write_bytes=wb, traffic_bytes=fb + wb)
    out = dict(workload=args.workload, fetch_scale=cf, write_scale=cw, copy_bytes=copy_bytes, kernels=rows,
               source_sha256=kernel_source_hash())
    if args.kernel:
        sel = [k for k in rows if k.startswith(args.kernel)]
        if len(sel) != 1:
            raise SystemExit(f"kernel {args.kernel!r} matches {sel}")
        out["kernel"] = sel[0]
        out["traffic_bytes"] = rows[sel[0]]["traffic_bytes"]
    print(f"calibration: FETCH_SIZE x {cf:.4f}, WRITE_SIZE x {cw:.4f} ({args.copy_mib} MiB copy)")
    for k, v in rows.items():
        print(f"{k:36s} launches {v['launches']:3d}  fetch {v['fetch_bytes'] / 1e6:9.2f} MB  "
              f"write {v['write_bytes'] / 1e6:9.2f} MB")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    return 0


def solve(args):
    """Solves of a named workload (its first RHS, or both polarizations), for
    kernel statistics of the whole iteration."""
    import torch

    import inputs
    import paper_1305_6497_amd as dda

    w = inputs.WORKLOADS[args.workload]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    kd = dda.kd_from_x(w["x"], len(sites))
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1 + k) for k in range(args.nrhs)]
    P = torch.empty((len(rhs), len(sites), 3), dtype=torch.complex128, device="cuda")
    for rep in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = t.solve(rhs, tol=args.tol, precision=args.precision, out=P, solver=args.solver)
        torch.cuda.synchronize()
        print(json.dumps(dict(workload=args.workload, solver=args.solver, precision=args.precision, rep=rep,
                              seconds=time.perf_counter() - t0, iters=[x["iters"] for x in st])), flush=True)
    t.close()
    return 0


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "solve":
        ap = argparse.ArgumentParser(prog="profile_matvec solve")
        ap.add_argument("workload")
        ap.add_argument("--solver", default="bicgstab")
        ap.add_argument("--precision", default="mixed")
        ap.add_argument("--nrhs", type=int, default=1, choices=(1, 2))
        ap.add_argument("--tol", type=float, default=1e-5)
        ap.add_argument("--reps", type=int, default=1)
        return solve(ap.parse_args(sys.argv[2:]))
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        ap = argparse.ArgumentParser(prog="profile_matvec summarize")
        ap.add_argument("fetch_dir")
        ap.add_argument("write_dir")
        ap.add_argument("--workload", default="block_64")
        ap.add_argument("--kernel", default=None)
        ap.add_argument("--copy-mib", type=int, default=512)
        ap.add_argument("--json", default=None)
        return summarize(ap.parse_args(sys.argv[2:]))
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
