"""Build libdop.so (HIP kernels + C ABI + serving engine) in-tree for gfx950.

Usage: python -m paper_2505_22313_amd.build   (or build() from Python)
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdop.so")

SOURCES = ["asm_kernels.hip", "upsample_kernels.hip", "probe_kernels.hip", "dop_api.cpp",
           "dop_serve.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    print("[build]", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(jobs=None, verbose=True):
    """Compile every source to an object in _build/ and link libdop.so."""
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [cc] + HIPCC_FLAGS + lang + ["-I", os.path.join(ROOT, "include"),
                                          "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print("[build]", " ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [p.wait() for p in procs]
    if any(bad):
        raise RuntimeError("compilation failed")
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
