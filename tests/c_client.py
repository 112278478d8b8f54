"""Builds tests/c_abi_client.c against the shared library and the oracle's
C source (a C program, no Python, using the library through its header)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(ROOT, "paper_1303_4312_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out_dir):
    exe = os.path.join(out_dir, "c_abi_client")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "c_abi_client.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-o", exe, "-L", LIB_DIR, "-lcorank_merge", f"-Wl,-rpath,{LIB_DIR}",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe
