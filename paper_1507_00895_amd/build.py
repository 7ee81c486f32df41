"""Build libdf.so (HIP, gfx950) in-tree.

    python -m paper_1507_00895_amd.build            # build
    python -m paper_1507_00895_amd.build --check    # build, then list exported symbols

hipcc compiles every .hip source of csrc/ for gfx950 only.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdf.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Ladder kernels: no machine-level loop-invariant code motion.  In the item
# loop of the queue and persistent builds it hoisted values out of the loop
# and held them across the whole unrolled item (the three-wave FP64 build went
# from 0 to 260 bytes of spills per lane); the one-item builds are unchanged.
LADDER_FLAGS = ["-mllvm", "-disable-machine-licm"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source to an object, link libdf.so; returns its path."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="libdf_build_")
    try:
        objs = [os.path.join(tmp, os.path.basename(src) + ".o") for src in sources()]

        def compile_one(src, obj):
            extra = LADDER_FLAGS if os.path.basename(src).startswith("df_ladder_") else []
            cmd = [cc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
                   "-I", INCLUDE, "-I", CSRC, *DEVICE_FLAGS, *extra, src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
            return src, r.returncode, r.stdout.decode(errors="replace")

        # the slowest translation units first, so that they do not finish last
        order = sorted(zip(sources(), objs), key=lambda so: -os.path.getsize(so[0]) -
                       (10 ** 6 if "_np" in so[0] else 0))
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, code, text in ex.map(lambda so: compile_one(*so), order):
                _report(src, code, text)
        out_tmp = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


def _report(src, code, text):
    if code != 0:
        raise RuntimeError(f"compile of {os.path.basename(src)} failed:\n{text}")
    # hipcc's host pass does not know the packed-fp32 target feature
    for line in text.splitlines():
        if line.strip() and "packed-fp32-ops" not in line and "warning: unknown" not in line:
            print(line)


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
    if "--check" in sys.argv:
        out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
        print("\n".join(l for l in out.splitlines() if " T df_" in l))
