"""Compile the package's native libraries in-tree.

* ``libspgraph.so``: seeded graph generators and the CSR builder (host C++,
  g++).
* ``libsp.so``: the gfx950 BC library (HIP C++, hipcc), exporting the C ABI of
  ``include/sp.h``.

Floating-point contraction is off (``-ffp-contract=off``) so every sigma/delta
operation rounds separately, and packed FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
SP_LIB = os.path.join(HERE, "libsp.so")
GRAPH_LIB = os.path.join(HERE, "libspgraph.so")

HIP_SOURCES = ["api.hip", "source_path.hip", "batch_path.hip", "server.hip", "profile.hip", "autotune.hip",
               "sssp_path.hip", "pr_path.hip",
               "tc_path.hip", "noalloc.hip", "wg_path.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build_graphgen() -> str:
    tmp = GRAPH_LIB + ".tmp%d" % os.getpid()
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
          "-o", tmp, os.path.join(CSRC, "graphgen.cpp")])
    os.replace(tmp, GRAPH_LIB)
    return GRAPH_LIB


def header_hash() -> int:
    """First 8 bytes of the sha256 of include/sp.h: compiled into the library
    (sp_header_hash) and checked by the binding when it loads, so a library
    built from another version of the header is refused instead of
    exchanging structs of the wrong size."""
    import hashlib
    with open(os.path.join(ROOT, "include", "sp.h"), "rb") as f:
        return int.from_bytes(hashlib.sha256(f.read()).digest()[:8], "little")


def build_sp(jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    flags = HIP_FLAGS + ["-DSP_HEADER_HASH=%#xull" % header_hash()]
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = SP_LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, SP_LIB)
    return SP_LIB


def build_all() -> None:
    build_graphgen()
    build_sp()


if __name__ == "__main__":
    build_all()
    print("built", GRAPH_LIB, SP_LIB)
