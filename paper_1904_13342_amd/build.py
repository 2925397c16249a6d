"""Build libpyrohip.so for gfx950 with hipcc (in-tree, no JIT cache).

    python paper_1904_13342_amd/build.py

Run it as a script (importing the package loads the library it builds).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpyrohip.so")
SOURCES = ["abi.cpp", "proj2d.hip", "cone_bp.hip", "cone_fp.hip", "filter.hip", "adjoint.hip",
           "corrector.hip", "tv.hip", "noalloc.hip", "widen.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # never emit packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-result",
]


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    return obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = [_compile(s) for s in SOURCES]
    objs = []
    failed = False
    for (obj, p), src in zip(jobs, SOURCES):
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 target feature; harmless
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n{text}\n")
        elif verbose and text.strip():
            sys.stderr.write(f"--- {src}\n{text}\n")
        objs.append(obj)
    if failed:
        raise RuntimeError("hipcc compilation failed")
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
