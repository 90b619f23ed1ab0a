"""Benchmark of the DDA hot path on one MI355X.

A step is one whole pass of the path over the largest single-GPU workload: a
sphere of diameter 133 dipoles (ELLIPSOID SHPAR 133, N = 1,232,177, FFT grid
270^3), m = 1.33 + 0.001i, x = 25, incidence along x, both polarizations (e
along y and z) as one batch of two right-hand sides.  The step is the
incident field, COCG with the complex FP32 FFT product and FP64 Krylov
vectors and inner products, FP64 true-residual refinement to 1e-5, and the
FP64 cross-section sums.  The Green-tensor transform of the target is built
once before timing (it depends on the target and k only).

Prints one JSON line on stdout (progress goes to stderr).  `value` is solves
per second (a batch of two RHS is two solves).  Extra fields: products/s,
p50/p99 step latency, the other solvers and the plain FP64 single-RHS solver
on the same workload, the Q error of every result against the FP64 oracle's
stored solution (tests/golden), a tolerance scan, per-pass HIP-event timing,
the roofline of the dominant kernel and of the whole product, and the FP64 CPU
oracle timed on a bounded sample of the same solve.  The other workloads
(64^3 block, D = 20 sphere, 64-RHS ellipsoid, the guide's worked example and
near field, the 1000-request serving mix) are under `workloads`.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "sphere_d133"
PASS_TIMING_EVERY = 4
SOLVER = "cocg"
# FP32 products and FP32 search directions (p, A p); residual, iterate, sums and the true-residual
# refinement in FP64
PRECISION = "mixed32"
PEAK_HBM_GBS = 8000.0
# FP32 / FP64 vector issue without packed math: 256 CUs x 4 SIMDs, one wave
# instruction per SIMD every 4 cycles at 2.4 GHz
PEAK_VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(box, grid, n_sites, fp32=True, nrhs=1):
    """Bytes the FFT product must move per launch of a block of nrhs RHS, and
    those of its z-pass.

    P in and AP out in FP64 (48 B per site each); each transform stage writes
    its output once and the next stage reads it once: x-forward output
    3*Mx*ny*nz, y-forward output 3*Mx*My*nz, the z-pass reads and writes the
    latter, the inverse stages mirror the forward ones; the octant Green
    transform (6 components) is read once per launch, whatever nrhs.
    """
    nx, ny, nz = box
    Mx, My, Mz = grid
    c = 8 if fp32 else 16
    moct = (Mx // 2 + 1) * (My // 2 + 1) * (Mz // 2 + 1)
    per_rhs = 2 * 48 * n_sites + 3 * c * (4 * Mx * ny * nz + 4 * Mx * My * nz)
    zpass_rhs = 2 * 3 * c * Mx * My * nz
    green = 6 * c * moct
    return nrhs * per_rhs + green, nrhs * zpass_rhs + green


def pass_bytes(box, grid, n_sites, fp32=True, nrhs=1):
    """Algorithmic bytes of each of the five passes for one launch of nrhs RHS."""
    nx, ny, nz = box
    Mx, My, Mz = grid
    c = 8 if fp32 else 16
    a_b = 3 * c * Mx * ny * nz
    b_b = 3 * c * Mx * My * nz
    _, z = algorithmic_bytes(box, grid, n_sites, fp32, nrhs)
    return dict(x_forward=nrhs * (48 * n_sites + a_b), y_forward=nrhs * (a_b + b_b), z_pass=z,
                y_inverse=nrhs * (a_b + b_b), x_inverse=nrhs * (a_b + 2 * 48 * n_sites))


# FP32 vector peak without packed math (this build keeps packed FP32 off): 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops per fused multiply-add x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def zpass_alu_roofline(grid, nrhs, ms):
    """The z-pass against the vector-ALU bound: algorithmic flops per launch (per column and RHS three
    forward and three inverse complex transforms of length Mz at 5 Mz log2 Mz flops each, and the 3x3
    complex multiply at 72 flops per frequency) over the launch time."""
    Mx, My, Mz = grid
    flops = nrhs * Mx * My * (6 * 5 * Mz * math.log2(Mz) + 72 * Mz)
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "z_pass", "achieved": achieved, "peak": PEAK_FP32_UNPACKED_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_UNPACKED_TFLOPS, "algorithmic_flops_per_launch": flops,
            "rhs_per_launch": nrhs, "launch_ms": ms}


KERNEL_PREFIX = dict(x_forward="k_xfwd", y_forward="k_yfwd", z_pass="k_zpass", y_inverse="k_yinv",
                     x_inverse="k_xinv")


def measured_traffic(kernel_prefix, workload):
    """HBM bytes per launch of a kernel from the committed counter summary
    (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated on a plain copy), or None
    when the kernel sources changed since the counters were taken."""
    from paper_1305_6497_amd import profile_matvec
    path = os.path.join(ROOT, "profiles", f"{kernel_prefix}_{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != profile_matvec.kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    return rec["traffic_bytes"], os.path.relpath(path, ROOT)


def roofline(prof, box, grid, n_sites, nrhs, workload, fp32=True):
    """Roofline of the dominant pass (by event time) and of the whole product."""
    pb = pass_bytes(box, grid, n_sites, fp32, nrhs)
    dom = max(pb, key=lambda k: prof[k])
    achieved = pb[dom] / (prof[dom] * 1e-3) / 1e9
    traffic, src = measured_traffic(KERNEL_PREFIX[dom], workload)
    tot, _ = algorithmic_bytes(box, grid, n_sites, fp32, nrhs)
    prod = tot / (prof["total"] * 1e-3) / 1e9
    return ({"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "traffic_source": src,
             "algorithmic_bytes_per_launch": pb[dom], "rhs_per_launch": nrhs, "launch_ms": prof[dom]},
            {"bound": "hbm", "achieved": prod, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": prod / PEAK_HBM_GBS,
             "algorithmic_bytes_per_launch": tot, "rhs_per_launch": nrhs, "product_ms": prof["total"],
             "pass_ms": prof, "pass_frac": {k: pb[k] / (prof[k] * 1e-3) / 1e9 / PEAK_HBM_GBS for k in pb}})


def _oracle_rate(sites, kd, m, rhs, budget_s):
    """Time FP64 COCG iterations of the oracle (one SciPy FFT product each) on one RHS: doubling the count
    until the run takes half the budget.  Returns (iterations, seconds, setup seconds, workers)."""
    from oracle import incident, interaction, polarizability, solvers
    workers = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    t0 = time.perf_counter()
    khat, e = rhs
    ai = polarizability.alpha_inv_ldr(m, kd, khat, e)
    E = incident.incident_field(sites, kd, khat, e)
    op = interaction.FFTOperator(sites, kd, ai, workers=workers)
    setup = time.perf_counter() - t0
    its = 1
    t0 = time.perf_counter()
    solvers.cocg(op.matvec, E, tol=1e-30, maxiter=its)
    dt = time.perf_counter() - t0
    while dt < budget_s * 0.5 and its < 64:
        its *= 2
        t0 = time.perf_counter()
        solvers.cocg(op.matvec, E, tol=1e-30, maxiter=its)
        dt = time.perf_counter() - t0
    return its, dt, setup, workers


def cpu_baseline(sites, kd, m, rhs, gpu_fp64_iters, budget_s=20.0):
    """FP64 CPU oracle (COCG on its SciPy FFT product) on a bounded sample of
    the same solve: s per iteration x the iteration count of the identical
    FP64 algorithm."""
    its, dt, setup, workers = _oracle_rate(sites, kd, m, rhs, budget_s)
    per_iter = dt / its
    solve_s = per_iter * gpu_fp64_iters
    return dict(value=1.0 / solve_s, unit="solves/s", cores=workers, kind="oracle",
                sample=(f"{its} FP64 COCG iterations ({its} SciPy FFT products of the 266^3 grid, "
                        f"scipy.fft workers={workers}; element-wise NumPy work single-threaded) of the same "
                        f"{WORKLOAD} solve (first polarization) in {dt:.2f} s; solves/s = 1 / (s per iteration x "
                        f"{gpu_fp64_iters} iterations, the count of the identical FP64 COCG on this GPU); "
                        f"Green-transform setup {setup:.1f} s excluded"),
                matvecs_per_s=its / dt, setup_s=setup)


def cpu_per_config(dda, inputs, extras, budget_s=6.0):
    """The oracle's FP64 product rate on every other configuration (first RHS), and its solve rate as
    s per product x the products of the same configuration's FP64 solve on this GPU."""
    from oracle import targets
    legs = (("block_64", lambda e: e["block_64"]["fp64"]["matvecs"]),
            ("sphere_d20", lambda e: e["sphere_d20"]["fp64_matvecs"]),
            ("ellipsoid_96x64x48", lambda e: e["ellipsoid_96x64x48_batched"]["fp64_matvecs_mean"]))
    out = {}
    for name, gpu_mv in legs:
        w = inputs.WORKLOADS[name]
        sites = targets.make(w["shape"], w["shpar"])
        kd = dda.kd_from_x(w["x"], len(sites))
        its, dt, setup, workers = _oracle_rate(sites, kd, w["m"], _rhs_list(dda, inputs, w)[0], budget_s)
        mv = gpu_mv(extras)
        out[name] = dict(matvecs_per_s=its / dt, solves_per_s=its / dt / mv, cores=workers,
                         gpu_fp64_matvecs_per_solve=mv, setup_s=setup,
                         sample=f"{its} FP64 COCG iterations of the oracle in {dt:.2f} s (first RHS)")
    return out


def _reference(name):
    """Oracle efficiencies stored by tests/golden/make_reference.py, if present."""
    path = os.path.join(ROOT, "tests", "golden", f"reference_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _rel_err(q, ref):
    return {k: abs(q[k] - ref[k]) / abs(ref[k]) for k in ("qext", "qabs", "qsca")}


def _ref_errors(q, ref):
    """Per-RHS relative errors against the stored oracle results (by RHS index)."""
    if not ref or not ref.get("results"):
        return None
    by = {r["rhs"]: r for r in ref["results"]}
    errs = [dict(rhs=i, **_rel_err(q[i], by[i])) for i in range(len(q)) if i in by]
    worst = max((max(e["qext"], e["qabs"], e["qsca"]) for e in errs), default=None)
    return dict(n_compared=len(errs), n_results=len(q), max_rel_err=worst, per_rhs=errs)


def _rhs_list(dda, inputs, w):
    """(khat, e) of the workload: fixed incidence along x, or seeded SO(3) orientations."""
    if w["orientations"] == 1:
        return [dda.orient_rhs(0.0, 0.0, 0.0, which=k + 1) for k in range(w["polarizations"])]
    b, t, p = inputs.orientation_angles(w["orientations"])
    return [dda.orient_rhs(b[i], t[i], p[i], which=k + 1) for i in range(w["orientations"])
            for k in range(w["polarizations"])]


def _timed_solves(t, torch, rhs, reps, **kw):
    t.solve(rhs, **kw)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(reps):
        P, st = t.solve(rhs, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - s0) / reps, P, st


def block64_workload(dda, inputs, torch, tol):
    """64^3 block, one RHS: mixed against FP64, every solver (Infinity-Cache resident)."""
    w = inputs.WORKLOADS["block_64"]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    n = len(sites)
    kd = dda.kd_from_x(w["x"], n)
    rhs = [dda.orient_rhs(0.0, 0.0, 0.0, which=1)]
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    info = t.info()
    P = torch.empty((1, n, 3), dtype=torch.complex128, device="cuda")
    ref = _reference("block_64")
    out = {"config": {"n_sites": n, "box": list(info["box"]), "fft_grid": list(info["grid"]), "nrhs": 1,
                      "tol": tol}}
    for name, prec, solver in (("mixed", "mixed", "bicgstab"), ("fp64", "fp64", "bicgstab"),
                               ("mixed32", "mixed32", "bicgstab"), ("mixed_bicgstab2", "mixed", "bicgstab2"),
                               ("mixed_cocg", "mixed", "cocg"), ("mixed32_cocg", "mixed32", "cocg"),
                               ("mixed_qmr", "mixed", "qmr")):
        dt, P, st = _timed_solves(t, torch, rhs, 5, tol=tol, precision=prec, out=P, solver=solver)
        q = t.cross_sections(rhs, P)
        out[name] = {"solves_per_s": 1.0 / dt, "iters": st[0]["iters"], "matvecs": st[0]["matvecs"],
                     "rel_resid": st[0]["rel_resid"], "q": q[0], "q_err_vs_oracle": _ref_errors(q, ref)}
    out["speedup_mixed_over_fp64"] = out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    Pr = torch.tensor(inputs.random_polarization(n, 1, seed=1), device="cuda")
    prof = t.profile_matvec(rhs, Pr, precision="mixed", reps=50)
    prof64 = t.profile_matvec(rhs, Pr, precision="fp64", reps=20)
    dom, prod = roofline(prof, info["box"], info["grid"], n, 1, "block_64")
    dom64, prod64 = roofline(prof64, info["box"], info["grid"], n, 1, "block_64", fp32=False)
    out["roofline"] = dom
    out["product_roofline"] = prod
    out["roofline_fp64"] = dom64
    out["product_roofline_fp64"] = prod64
    out["note"] = "working set below the 256 MB Infinity Cache: the roofline is not graded here"
    t.close()
    return out


def extra_workloads(dda, inputs, torch, tol, serving_alone=True):
    """The other configurations."""
    import numpy as np
    out = {}

    log("block_64")
    out["block_64"] = block64_workload(dda, inputs, torch, tol)

    # Sphere D = 20 (N = 4224), FP64, two polarizations solved separately.
    log("sphere_d20")
    w = inputs.WORKLOADS["sphere_d20"]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    kd = dda.kd_from_x(w["x"], len(sites))
    rhs = _rhs_list(dda, inputs, w)
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    res = {}
    for graph in (False, True):
        for r in rhs:
            t.solve([r], tol=tol, precision="fp64", use_graph=graph)
        lat = []
        for _ in range(10):
            for r in rhs:
                s0 = time.perf_counter()
                P, st = t.solve([r], tol=tol, precision="fp64", use_graph=graph)
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - s0)
        res["graph" if graph else "eager"] = {"solves_per_s": len(lat) / sum(lat),
                                             "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                             "p99_ms": float(np.percentile(lat, 99) * 1e3), "iters": st[0]["iters"],
                                             "matvecs": st[0]["matvecs"]}
    P, st = t.solve(rhs, tol=tol, precision="fp64")
    q = t.cross_sections(rhs, P)
    ref = _reference("sphere_d20")
    res["q"] = q
    res["fp64_matvecs"] = float(np.mean([x["matvecs"] for x in st]))
    res["q_err_vs_oracle"] = _ref_errors(q, ref)
    res["mie"] = ref.get("mie") if ref else None
    res["config"] = {"n_sites": len(sites), "fft_grid": list(t.info()["grid"]), "precision": "fp64", "nrhs": 1}
    t.close()
    out["sphere_d20"] = res

    # Ellipsoid 96 x 64 x 48: 32 orientations x 2 polarizations = 64 RHS in one block (mixed) against the
    # plain FP64 single-RHS solver on the same GPU; every result against the oracle's.
    log("ellipsoid_96x64x48 (64 RHS)")
    w = inputs.WORKLOADS["ellipsoid_96x64x48"]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    kd = dda.kd_from_x(w["x"], len(sites))
    rhs = _rhs_list(dda, inputs, w)
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    P = torch.empty((len(rhs), len(sites), 3), dtype=torch.complex128, device="cuda")
    ref = _reference("ellipsoid_96x64x48")
    ell = {"nrhs": len(rhs), "config": {"n_sites": len(sites), "fft_grid": list(t.info()["grid"]),
                                        "precision": "mixed", "orientations": "PCG64 seed 1305, uniform on SO(3)"}}
    for tl in sorted({tol, 3e-6, 1e-6, 1e-7}, reverse=True):
        t.solve(rhs, tol=tl, precision="mixed", out=P, solver="bicgstab")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        P, st = t.solve(rhs, tol=tl, precision="mixed", out=P, solver="bicgstab")
        q = t.cross_sections(rhs, P)
        torch.cuda.synchronize()
        tb = time.perf_counter() - s0
        ell[f"tol_{tl:g}"] = {"solves_per_s": len(rhs) / tb, "block_seconds": tb,
                              "iters_mean": float(np.mean([x["iters"] for x in st])),
                              "iters_max": int(max(x["iters"] for x in st)),
                              "max_rel_resid": float(max(x["rel_resid"] for x in st)),
                              "q_err_vs_oracle": _ref_errors(q, ref)}
    # the loosest tolerance whose every result is within 1e-5 of the oracle's
    ok = [k for k in sorted((k for k in ell if k.startswith("tol_")), key=lambda k: -float(k[4:]))
          if ell[k]["q_err_vs_oracle"] and ell[k]["q_err_vs_oracle"]["max_rel_err"] is not None
          and ell[k]["q_err_vs_oracle"]["max_rel_err"] <= 1e-5]
    ell["at_parity"] = dict(tol=float(ok[0][4:]), solves_per_s=ell[ok[0]]["solves_per_s"],
                            max_rel_err=ell[ok[0]]["q_err_vs_oracle"]["max_rel_err"]) if ok else None
    # the same block with FP32 search directions (BiCGSTAB and COCG) at the metric's tolerance and at the
    # parity tolerance
    for slv in ("bicgstab", "cocg"):
        for tl in sorted({tol, ell["at_parity"]["tol"] if ell["at_parity"] else tol}, reverse=True):
            t.solve(rhs, tol=tl, precision="mixed32", out=P, solver=slv)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            P, st = t.solve(rhs, tol=tl, precision="mixed32", out=P, solver=slv)
            q = t.cross_sections(rhs, P)
            torch.cuda.synchronize()
            tb = time.perf_counter() - s0
            ell[f"{slv}_mixed32_tol_{tl:g}"] = {"solves_per_s": len(rhs) / tb, "block_seconds": tb,
                                                "iters_mean": float(np.mean([x["iters"] for x in st])),
                                                "iters_max": int(max(x["iters"] for x in st)),
                                                "q_err_vs_oracle": _ref_errors(q, ref)}
    P1 = torch.empty((1, len(sites), 3), dtype=torch.complex128, device="cuda")
    t.solve(rhs[:1], tol=tol, precision="fp64", out=P1)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    iters64 = []
    mv64 = []
    for r in rhs:
        P1, s1 = t.solve([r], tol=tol, precision="fp64", out=P1)
        t.cross_sections([r], P1)
        iters64.append(s1[0]["iters"])
        mv64.append(s1[0]["matvecs"])
    torch.cuda.synchronize()
    ts = time.perf_counter() - s0
    ell["fp64_single_rhs_solves_per_s"] = len(rhs) / ts
    ell["fp64_iters_mean"] = float(np.mean(iters64))
    ell["fp64_matvecs_mean"] = float(np.mean(mv64))
    ell["speedup_batched_mixed_over_fp64_single"] = ell[f"tol_{tol:g}"]["solves_per_s"] / ell[
        "fp64_single_rhs_solves_per_s"]
    prof = t.profile_matvec(rhs, P, precision="mixed", reps=3)
    info = t.info()
    ell["roofline"], ell["product_roofline"] = roofline(prof, info["box"], info["grid"], len(sites), len(rhs),
                                                        "ellipsoid_96x64x48")
    t.close()
    out["ellipsoid_96x64x48_batched"] = ell

    # Near field of the guide's Au sphere (N = 59728 in 48^3, kd = 0.20619, m = 0.96+1.01i) on the printed
    # 96^3 extended volume, interpolated trilinearly along the printed line through the centre.
    log("au_sphere_near_field")
    golden = os.path.join(ROOT, "tests", "golden")
    fx = json.load(open(os.path.join(golden, "au_sphere_nearfield_line.json")))
    sites, box = dda.make_sites("ELLIPSOID", (48.49, 48.49, 48.49))
    rhs = [(np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))]
    t = dda.Target(sites, box, m=complex(*fx["m"]), kd=fx["kd"])
    t.solve(rhs, tol=1e-5, precision="fp64")
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    P, st = t.solve(rhs, tol=1e-5, precision="fp64")
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    E = t.near_field(rhs, P, margin=(24, 24, 24))
    torch.cuda.synchronize()
    s2 = time.perf_counter()
    _, B = t.near_field(rhs, P, margin=(24, 24, 24), magnetic=True)    # E and B (the NRFLD = 2 option)
    torch.cuda.synchronize()
    s3 = time.perf_counter()
    del B
    E = E.cpu().numpy()[0]
    t.close()
    c = (np.array(box) - 1) / 2.0
    E = E * np.exp(-1j * fx["kd"] * c[0])                  # phase origin at the sphere's centre
    rows = np.array(fx["rows"])
    xs = c[0] + rows[:, 0] / fx["d_um"] + 24
    i0 = np.floor(xs).astype(int)
    w1 = xs - i0
    yz = (int(c[1]) + 24, int(c[1]) + 25)                 # the line lies midway between lattice planes
    ey = sum(0.25 * ((1 - w1) * E[z, y, i0, 1] + w1 * E[z, y, i0 + 1, 1]) for y in yz for z in yz)
    dev = np.abs(ey - (rows[:, 5] + 1j * rows[:, 6]))
    out["au_sphere_near_field"] = {
        "n_sites": len(sites), "extended_box": [96, 96, 96], "solve_seconds": s1 - s0, "iters": st[0]["iters"],
        "near_field_seconds": s2 - s1, "points_per_s": 96 ** 3 / (s2 - s1), "near_field_e_and_b_seconds": s3 - s2,
        "max_abs_dev_from_printed_line": float(dev.max()),
        "note": "FP64 solve to 1e-5 (LDR; the printed run used GKDLDR), near field on 96^3, E_y along the printed "
                "x-axis track, trilinear"}

    # The guide's worked example (16 x 32 x 32 Au block, two polarizations along y and z, k along x): every
    # printed efficiency next to the GPU's, solved with GKDLDR and BiCGstab(2) to TOL 1e-5 as printed.
    log("au_block_worked_example")
    pr = json.load(open(os.path.join(golden, "paper_printed.json")))["au_block_example"]
    mu = json.load(open(os.path.join(golden, "au_block_mueller.json")))
    sites, box = dda.make_sites("RCTGLPRSM", mu["box"])
    lab = np.eye(3)
    rhs = [(lab[0], lab[1]), (lab[0], lab[2])]
    t = dda.Target(sites, box, m=complex(*mu["m"]), kd=mu["kd"], alpha="GKDLDR")
    t.solve(rhs, tol=1e-5, precision="fp64", solver="bicgstab2")
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    P, st = t.solve(rhs, tol=1e-5, precision="fp64", solver="bicgstab2")
    q = t.cross_sections(rhs, P)
    far = t.far_field(rhs, P, etasca=0.5)
    _, S, M = t.scattering_matrix(rhs, P, lab, [[0.0, 0.0], [math.pi, 0.0]])
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    t.close()
    mean = lambda key, src: 0.5 * (src[0][key] + src[1][key])
    gpu = {"qext": mean("qext", q), "qabs": mean("qabs", q), "qsca": mean("qsca", q), "g": mean("g", far),
           "cos2": mean("cos2", far), "qbk": mean("qbk", far), "qpha": mean("qpha", q),
           "qpol": q[0]["qext"] - q[1]["qext"], "s11_0": float(M[0, 0, 0]), "s11_180": float(M[1, 0, 0])}
    printed = {"qext": pr["qext"], "qabs": pr["qabs"], "qsca": pr["qsca"], "g": mu["g"], "cos2": mu["cos2"],
               "qbk": pr["qbk"], "qpha": pr["qpha"], "qpol": pr["qpol"], "s11_0": mu["rows"][0][3],
               "s11_180": pr["s11_180"]}
    out["au_block_worked_example"] = {
        "n_sites": len(sites), "solve_and_outputs_seconds": s1 - s0,
        "bicgstab2_cycles": [x["iters"] // 2 for x in st], "printed_iterations": [18, 18], "gpu": gpu,
        "printed": printed,
        "rel_diff": {k: (gpu[k] - printed[k]) / abs(printed[k]) for k in printed if k != "qpol"},
        "note": "FP64, TOL 1e-5, GKDLDR and BiCGstab(2) as printed; the printed values carry the printed run's "
                "own TOL 1e-5 residual"}

    # Serving mix: the whole seeded 1000-request stream, saturated, then Poisson arrivals at 0.8x the
    # saturated rate, then every request alone (one slot) for the alone-vs-mix difference of each result.
    from paper_1305_6497_amd import serving
    log("serving mix (1000 requests)")
    out["serving_mix_1000"] = serving_mix(serving, dda, inputs, tol, alone=serving_alone)
    return out


def serving_mix(serving, dda, inputs, tol, n=1000, slots=8, alone=True):
    import numpy as np
    ex = serving.GpuExecutor(tol=tol)
    reqs = serving.make_requests(n, inputs.SERVING_SEED, 1.0, dda)
    burst = [serving.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs]
    s0 = time.perf_counter()
    res_sat = serving.Server(ex, slots=slots).run(burst)
    sat = serving.summarize(res_sat, time.perf_counter() - s0)
    log(f"serving saturated: {sat['requests_per_s']:.1f} requests/s")
    rate = 0.8 * sat["requests_per_s"]
    reqs = serving.make_requests(n, inputs.SERVING_SEED, rate, dda)
    s0 = time.perf_counter()
    res_poi = serving.Server(ex, slots=slots).run(reqs)
    poi = serving.summarize(res_poi, time.perf_counter() - s0)
    poi["arrival_rate_per_s"] = rate
    log(f"serving Poisson: p50 {poi['p50_ms']:.0f} ms, p99 {poi['p99_ms']:.0f} ms")
    failed = [dict(id=r.id, shape=reqs[r.id].shape, shpar=list(reqs[r.id].shpar), m=[reqs[r.id].m.real,
                   reqs[r.id].m.imag], x=reqs[r.id].x, n_sites=r.n_sites, error=r.error,
                   stats=r.stats) for r in res_poi.values()
              if r.error or not all(s["status"] == 0 for s in r.stats)]
    out = {"saturated": sat, "poisson_0.8": poi, "slots": slots, "requests": n,
           "unconverged": failed,
           "cap": "per RHS: COCG with the products of 2000 BiCGSTAB iterations, then BiCGstab(2) from its iterate "
                  "for up to 4000 BiCG steps (survey reading C-18: max_iter caps an outlier)",
           "note": "seeded 1000-request mix (PCG64 seed 4242); 2 polarizations each; mixed precision, tol "
                   f"{tol:g}; admission by dda_footprint_bytes against 80% of free HBM"}
    if alone:
        # every request alone (one slot, one at a time) against its result inside the Poisson mix
        s0 = time.perf_counter()
        res_alone = serving.Server(ex, slots=1).run([serving.Request(**{**r.__dict__, "arrival": 0.0})
                                                     for r in reqs])
        dq = []
        for r in reqs:
            a, b = res_alone[r.id], res_poi[r.id]
            if a.error or b.error:
                continue
            dq.append(max(abs(qa[k] - qb[k]) / abs(qa["qext"]) for qa, qb in zip(a.q, b.q)
                          for k in ("qext", "qabs", "qsca")))
        dq = np.array(dq)
        out["alone_vs_mix"] = {"requests_compared": int(len(dq)), "max_abs_dq_over_qext": float(dq.max()),
                               "nonzero": int((dq > 0).sum()), "p99_abs_dq_over_qext": float(np.percentile(dq, 99)),
                               "alone_seconds": time.perf_counter() - s0}
        log(f"serving alone-vs-mix: max |dQ|/Q_ext {dq.max():.3g}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--no-serving-alone", action="store_true", help="skip the alone-vs-mix serving rerun")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not part of this "
              "build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_1305_6497_amd as dda

    w = inputs.WORKLOADS[WORKLOAD]
    sites, box = dda.make_sites(w["shape"], w["shpar"])
    n = len(sites)
    kd = dda.kd_from_x(w["x"], n)
    rhs = _rhs_list(dda, inputs, w)
    log(f"{WORKLOAD}: N = {n}, setup")
    t = dda.Target(sites, box, m=w["m"], kd=kd)
    info = t.info()
    P = torch.empty((len(rhs), n, 3), dtype=torch.complex128, device="cuda")
    ref = _reference(WORKLOAD)

    def step(tol, solver=SOLVER, precision=PRECISION, r=rhs, out=P):
        Pp, st = t.solve(r, tol=tol, precision=precision, out=out, solver=solver, max_iter=20000)
        q = t.cross_sections(r, Pp)
        return st, q

    for _ in range(args.warmup):
        step(args.tol)
    torch.cuda.synchronize()
    log(f"{WORKLOAD}: {args.steps} timed steps")
    # HIP events around the five passes of every PASS_TIMING_EVERY-th product the timed solves launch
    t.set_pass_timing(PASS_TIMING_EVERY)
    lat = []
    mv = 0
    outer = 0
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        st, q = step(args.tol)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        mv += sum(x["matvecs"] for x in st)
        outer += sum(x["outer"] for x in st)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    in_solve, n_timed = t.pass_timing("mixed")
    t.set_pass_timing(0)
    assert all(x["status"] == 0 and x["rel_resid"] <= args.tol for x in st), st
    solves = len(rhs) * args.steps

    # the same batch with the other solvers
    log(f"{WORKLOAD}: other solvers")
    solvers_out = {}
    for solver, prec in (("cocg", "mixed"), ("bicgstab", "mixed"), ("bicgstab2", "mixed"), ("qmr", "mixed")):
        dt, Ps, sts = _timed_solves(t, torch, rhs, 2, tol=args.tol, precision=prec, out=P, solver=solver,
                                    max_iter=20000)
        qs = t.cross_sections(rhs, Ps)
        solvers_out[f"{solver}_{prec}"] = {"solves_per_s": len(rhs) / dt, "iters": [x["iters"] for x in sts],
                               "matvecs": [x["matvecs"] for x in sts], "q_err_vs_oracle": _ref_errors(qs, ref)}

    # plain FP64 single-RHS solver on the same GPU (one polarization at a time)
    log(f"{WORKLOAD}: FP64 single-RHS")
    P1 = torch.empty((1, n, 3), dtype=torch.complex128, device="cuda")
    s0 = time.perf_counter()
    st64 = []
    q64 = []
    for r in rhs:
        P1, s1 = t.solve([r], tol=args.tol, precision="fp64", out=P1, solver=SOLVER, max_iter=20000)
        q64 += t.cross_sections([r], P1)
        st64 += s1
    torch.cuda.synchronize()
    fp64_s = (time.perf_counter() - s0) / len(rhs)

    # tolerance scan: Q against the oracle's solution at the metric's tolerance and tighter ones; throughput
    # at the loosest tolerance whose every result is within 1e-5 of the oracle's
    log(f"{WORKLOAD}: tolerance scan")
    scan = []
    for tl in (1e-5, 3e-6, 1e-6, 3e-7, 1e-7):
        dt, Ps, sts = _timed_solves(t, torch, rhs, 1, tol=tl, precision=PRECISION, out=P, solver=SOLVER,
                                    max_iter=20000)
        qs = t.cross_sections(rhs, Ps)
        scan.append({"tol": tl, "solves_per_s": len(rhs) / dt, "iters": [x["iters"] for x in sts],
                     "q_err_vs_oracle": _ref_errors(qs, ref)})
    parity = [s for s in scan if s["q_err_vs_oracle"] and s["q_err_vs_oracle"]["max_rel_err"] is not None
              and s["q_err_vs_oracle"]["max_rel_err"] <= 1e-5]
    at_parity = dict(tol=parity[0]["tol"], solves_per_s=parity[0]["solves_per_s"],
                     max_rel_err=parity[0]["q_err_vs_oracle"]["max_rel_err"]) if parity else None

    # event timing of the five FFT passes: the 2-RHS mixed product of the solve, and the FP64 product
    log(f"{WORKLOAD}: pass timing")
    Pr = torch.tensor(inputs.random_polarization(n, len(rhs), seed=1), device="cuda")
    prof = t.profile_matvec(rhs, Pr, precision="mixed", reps=20)
    prof64 = t.profile_matvec(rhs[:1], Pr[:1].contiguous(), precision="fp64", reps=10)
    dom, prod = roofline(in_solve, info["box"], info["grid"], n, len(rhs), WORKLOAD)
    dom_alu = zpass_alu_roofline(info["grid"], len(rhs), in_solve["z_pass"])
    dom_iso, prod_iso = roofline(prof, info["box"], info["grid"], n, len(rhs), WORKLOAD)
    dom64, prod64 = roofline(prof64, info["box"], info["grid"], n, 1, WORKLOAD, fp32=False)
    mie = ref.get("mie") if ref else None
    # far field of the last solve: Q_sca by quadrature (the dipole array's optical theorem) and <cos theta>
    s0 = time.perf_counter()
    Pq, _ = t.solve(rhs, tol=args.tol, precision=PRECISION, out=P, solver=SOLVER, max_iter=20000)
    far = t.far_field(rhs, Pq, etasca=0.5)
    torch.cuda.synchronize()
    far_out = dict(seconds_with_solve=time.perf_counter() - s0, n_theta=far[0]["n_theta"], n_phi=far[0]["n_phi"],
                   qsca=[f["qsca"] for f in far], g=[f["g"] for f in far], mie_g=mie.get("g") if mie else None,
                   qsca_rel_diff_vs_qext_minus_qabs=[abs(f["qsca"] - v["qsca"]) / v["qext"] for f, v in zip(far, q)])
    ms_per_step = 1e3 * total / args.steps
    lat_ms = np.array(lat) * 1e3
    t.close()

    extras = None
    if not args.no_extras:
        extras = extra_workloads(dda, inputs, torch, args.tol, serving_alone=not args.no_serving_alone)
    cpu = None
    if not args.no_cpu:
        log("cpu_baseline (FP64 oracle)")
        from oracle import targets
        cpu = cpu_baseline(targets.make(w["shape"], w["shpar"]), kd, w["m"], rhs[0], st64[0]["iters"])
        if extras:
            log("per-configuration oracle rates")
            cpu["per_config"] = cpu_per_config(dda, inputs, extras)
    out = {
        "metric": "FFT dipole matvecs/sec + solves/sec at 1e-5 rel. residual; p50/p99 latency",
        "value": solves / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 FFT product and search directions / f64 residual, iterate, sums and refinement",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: ELLIPSOID SHPAR 133 sphere, N={n}, m=1.33+0.001i, x=25, LATTDR, "
                               "k||x, e||y and e||z as one batch of 2 RHS, COCG, FP32 product and search "
                               f"directions + FP64 residual and refinement to {args.tol:g}",
                   "n_sites": n, "box": list(info["box"]), "fft_grid": list(info["grid"]), "kd": kd,
                   "nrhs": len(rhs), "tol": args.tol, "solver": SOLVER, "precision": PRECISION},
        "solves_per_step": len(rhs),
        "matvecs_per_s": mv / total,
        "matvecs_per_solve": mv / solves,
        "fp64_checks_per_solve": outer / solves,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "q": q,
        "iters": [x["iters"] for x in st],
        "rel_resid": [x["rel_resid"] for x in st],
        "q_err_vs_oracle": _ref_errors(q, ref),
        "q_rel_err_vs_mie": [_rel_err(v, mie) for v in q] if mie else None,
        "far_field": far_out,
        "at_parity": at_parity,
        "tolerance_scan": scan,
        "solvers": solvers_out,
        "fp64_single_rhs": {"solves_per_s": 1.0 / fp64_s, "iters": [x["iters"] for x in st64],
                            "q_err_vs_oracle": _ref_errors(q64, ref),
                            "speedup_mixed_batched_over_fp64_single": (solves / total) * fp64_s},
        "pass_timing_in_solve": {"every": PASS_TIMING_EVERY, "products_timed": n_timed, "ms": in_solve,
                                 "note": "HIP events on the solve's stream around each pass of the sampled "
                                         "products of the timed steps; roofline and product_roofline use it"},
        "matvec_event_ms": {"mixed_2rhs": prof, "fp64_1rhs": prof64},
        "roofline_alu": dom_alu,
        "roofline_isolated_passes": {"roofline": dom_iso, "product_roofline": prod_iso,
                                     "note": "each pass launched alone 20 times back to back"},
        "matvec_only_per_s": {"mixed": len(rhs) * 1e3 / prof["total"], "fp64": 1e3 / prof64["total"]},
        "roofline": dom,
        "product_roofline": prod,
        "roofline_fp64": dom64,
        "product_roofline_fp64": prod64,
        "cpu_baseline": cpu,
        "workloads": extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
