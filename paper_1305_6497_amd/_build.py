"""Build the HIP library libdda.so for gfx950 in-tree with hipcc."""

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdda.so")
OBJDIR = os.path.join(HERE, "_build")

# Packed-FP32 instructions are disabled for all device code; host.cpp (the
# site rules) is compiled without floating-point contraction.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-command-line-argument"]
SOURCES = {
    "matvec_f32.hip": [],
    "matvec_f32v.hip": [],
    "matvec_f64.hip": [],
    "fft_generic.hip": [],
    "krylov.hip": [],
    "farfield.hip": [],
    "nearfield.hip": [],
    "api.hip": [],
    "host.cpp": ["-ffp-contract=off"],
    "devmem.cpp": [],
    "tuned.cpp": [],
}


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    cmds = []
    objs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(OBJDIR, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([hipcc()] + DEVICE_FLAGS + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
        return r.stderr

    with cf.ThreadPoolExecutor(max_workers=min(max(1, (os.cpu_count() or 4)), len(cmds))) as ex:
        for msg in ex.map(run, cmds):
            if verbose and msg:
                print(msg)
    tmp = LIB + ".tmp"
    run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
