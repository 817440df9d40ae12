"""Build step of libps.so (HIP, gfx950) in-tree, next to this file.

    python -m paper_2312_17396_amd.build      # or: build() from Python

Every .hip / .cpp file under csrc/ is compiled with hipcc for gfx950 and
linked into one shared library with a C ABI (include/ps.h)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libps.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False) -> str:
    """Compile and link libps.so; returns its path.  Always recompiles."""
    objs = []
    odir = os.path.join(HERE, "_build")
    os.makedirs(odir, exist_ok=True)
    for src in sources():
        obj = os.path.join(odir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
        cmd = [HIPCC, *FLAGS, "-c", *lang, src, "-o", obj]
        cmd = [c for c in cmd if c != "-shared"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in (r.stderr or "").splitlines() if "not a recognized feature" not in l)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
