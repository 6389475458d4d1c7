"""Compiles libbht.so for gfx950 with hipcc (in-tree, next to this file)."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "bht.hip")]
LIB = os.path.join(HERE, "libbht.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed fp32 instructions stay off on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"),
                                  "-I", os.path.join(HERE, "csrc"), "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libbht.so")
    os.replace(tmp, LIB)
    return LIB


def device_asm(out_path: str) -> str:
    """gfx950 assembly of the kernels (for instruction-level checks)."""
    cmd = [hipcc()] + [f for f in HIP_FLAGS if f not in ("-shared", "-fPIC")] + [
        "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
        "-I", os.path.join(HERE, "csrc"), "-o", out_path] + SOURCES
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path


if __name__ == "__main__":
    print(build(verbose=True))
