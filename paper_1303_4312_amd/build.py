"""Build libcorank_merge.so in-tree with hipcc for gfx950.

Usage: python -m paper_1303_4312_amd.build  (or __graft_entry__.build()).
The shared library is written next to this file and is what the Python
binding loads; nothing is installed elsewhere.
"""
from __future__ import annotations

import concurrent.futures
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libcorank_merge.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)

HIP_SOURCES = ["launch.hip", "launch_keys_u32.hip", "launch_keys_u64.hip", "launch_keys_f32.hip",
               "sort.hip"]
CXX_SOURCES = ["api.cpp", "host_co_rank.cpp", "server.cpp"]

# -packed-fp32-ops: keep the compiler from emitting packed fp32 VALU ops.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build_id() -> str:
    """First 16 hex digits of a SHA-256 over the library's sources and
    header (names and contents): the library's build identity, compiled in
    and written into saved tuning tables."""
    h = hashlib.sha256()
    files = sorted(os.listdir(CSRC))
    for name in files:
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode() + b"\0")
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    with open(os.path.join(INCLUDE, "corank_merge.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def compile_command(src: str, obj: str, bid: str) -> list:
    """The compile command of one source file of the library."""
    if src.endswith(".cpp"):
        return [hipcc(), "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-I", INCLUDE,
                f'-DCM_BUILD_ID="{bid}"', "-c", os.path.join(CSRC, src), "-o", obj]
    return [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
            "-o", obj]


def build(verbose: bool = False) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cmds, objs = [], []
    bid = build_id()
    for src in HIP_SOURCES + CXX_SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmds.append(compile_command(src, obj, bid))
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # the translation units are independent: compile them side by side
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for cmd, res in zip(cmds, pool.map(lambda c: subprocess.run(c), cmds)):
            if res.returncode != 0:
                raise subprocess.CalledProcessError(res.returncode, cmd)
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
