"""Write reference efficiencies of the full-size workloads with the FP64 oracle.

Only ``oracle/`` and the seeded ``inputs`` module are used: every stored value
is the oracle's.  Each workload is solved with the oracle's BiCGSTAB on its
FFT product to a true relative residual of 1e-10 (dense LU is out of reach at
these sizes) and the efficiencies Q_ext, Q_abs, Q_sca = Q_ext - Q_abs are
written to ``reference_<name>.json`` beside this script, together with the
iteration count, the residual and the Mie efficiencies of spheres.

Usage:  python tests/golden/make_reference.py block_64 [ellipsoid_96x64x48:4] ...
(``name:k`` limits a multi-orientation workload to its first k right-hand
sides, ``name:a-b`` solves right-hand sides a .. b-1 only; ``name:mie``
writes only the Mie efficiencies of a sphere workload).

Each finished right-hand side is merged into the stored file at once, under
a file lock, replacing an earlier result of the same index: several
processes may fill disjoint ranges of one workload side by side, and an
interrupted run keeps what it finished.
"""

import fcntl
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import inputs  # noqa: E402
from oracle import cross_sections, incident, interaction, mie, polarizability, solvers, targets  # noqa: E402

TOL = 1e-10


def right_hand_sides(w):
    """(khat, e) pairs: fixed incidence along x, or seeded SO(3) orientations."""
    e1, e2 = incident.polarization_pair([0, 1, 0])
    pols = [e1, e2][: w["polarizations"]]
    if w["orientations"] == 1:
        return [incident.incident_in_tf(0.0, 0.0, 0.0, e) for e in pols]
    b, t, p = inputs.orientation_angles(w["orientations"])
    out = []
    for i in range(w["orientations"]):
        for e in pols:
            out.append(incident.incident_in_tf(b[i], t[i], p[i], e))
    return out


def header(name, w, n, kd):
    out = dict(workload=name, n_sites=n, kd=kd, aeff=targets.aeff(n), tol=TOL, m=[w["m"].real, w["m"].imag],
               x=w["x"], results=[],
               note="FP64 oracle: BiCGSTAB on the FFT product to true relative residual <= 1e-10; "
                    "LATTDR polarizability; Q_sca = Q_ext - Q_abs")
    if w["shape"] == "ELLIPSOID" and len(set(w["shpar"])) == 1:
        out["mie"] = mie.mie_q(w["m"], w["x"])
    return out


def merge(path, head, result):
    """Add one result to the stored file (read-modify-write under a lock)."""
    with open(path + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        data = head
        if os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
            if old.get("tol") == TOL and old.get("n_sites") == head["n_sites"]:
                data = old
        data["results"] = sorted([r for r in data["results"] if r["rhs"] != result["rhs"]] + [result],
                                 key=lambda r: r["rhs"])
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
        fcntl.flock(lk, fcntl.LOCK_UN)


def run(name, first=0, stop=None, workers=None):
    w = inputs.WORKLOADS[name]
    sites = targets.make(w["shape"], w["shpar"])
    n = len(sites)
    kd = targets.kd_from_x(w["x"], n)
    rhs = right_hand_sides(w)
    stop = len(rhs) if stop is None else min(stop, len(rhs))
    path = os.path.join(HERE, f"reference_{name}.json")
    head = header(name, w, n, kd)
    for r in range(first, stop):
        khat, e = rhs[r]
        t0 = time.time()
        ai = polarizability.alpha_inv_ldr(w["m"], kd, khat, e)
        E = incident.incident_field(sites, kd, khat, e)
        op = interaction.FFTOperator(sites, kd, ai, workers=workers)
        P, info = solvers.bicgstab(op.matvec, E, tol=TOL, maxiter=20000)
        q = cross_sections.efficiencies(n, kd, E, ai, P)
        res = dict(rhs=r, khat=list(map(float, khat)), e_re=list(map(float, np.real(e))),
                   e_im=list(map(float, np.imag(e))), qext=q["qext"], qabs=q["qabs"], qsca=q["qsca"],
                   iters=int(info["iters"]), rel_resid=float(info["rel_resid"]), seconds=time.time() - t0)
        print(name, r, res, flush=True)
        merge(path, dict(head, results=[]), res)
    return path


def mie_only(name):
    w = inputs.WORKLOADS[name]
    n = len(targets.make(w["shape"], w["shpar"]))
    out = dict(workload=name, n_sites=n, kd=targets.kd_from_x(w["x"], n), aeff=targets.aeff(n),
               m=[w["m"].real, w["m"].imag], x=w["x"], results=[], mie=mie.mie_q(w["m"], w["x"]),
               note="Mie efficiencies of the sphere of the same size parameter (oracle.mie)")
    path = os.path.join(HERE, f"reference_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return path


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        name, _, k = arg.partition(":")
        workers = int(os.environ.get("ORACLE_WORKERS", "-1"))
        if k == "mie":
            print(mie_only(name))
        elif "-" in k:
            a, b = k.split("-")
            print(run(name, int(a), int(b), workers=workers))
        else:
            print(run(name, 0, int(k) if k else None, workers=workers))
