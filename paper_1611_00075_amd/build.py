"""Build libmd.so (HIP, gfx950 only) in-tree with hipcc.

    python -m paper_1611_00075_amd.build

Flags: -O3, no FMA contraction (cell and neighbour decisions are compared bit
for bit with the FP64 oracle; FMAs the kernels want are written explicitly),
packed FP32 instructions disabled.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libmd.so (always recompiles)."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in sources():
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", src, "-o", obj,
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE), src))
        objs.append(obj)
    for p, src in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(err.decode())
            raise RuntimeError(f"hipcc failed on {src}")
        msg = err.decode()
        msg = "\n".join(l for l in msg.splitlines()
                        if "packed-fp32-ops" not in l and l.strip())
        if msg and verbose:
            sys.stderr.write(msg + "\n")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
