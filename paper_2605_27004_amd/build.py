"""Build the HIP library ``paper_2605_27004_amd/lib/liblbm.so`` for gfx950, in-tree.

    python paper_2605_27004_amd/build.py

Host code (the C ABI) is compiled with g++, the kernels with hipcc for gfx950 only, and the
two are linked into one shared library that the Python binding loads with ctypes.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
OUT = os.path.join(OUT_DIR, "liblbm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
             # packed FP32 instructions are kept out of every kernel
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs, objs = [], []
    for name in sorted(os.listdir(CSRC)):
        stem, ext = os.path.splitext(name)
        if ext == ".hip":
            cmd = [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, name), "-o", os.path.join(bdir, stem + "_hip.o")]
        elif ext == ".cpp":
            cmd = ["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, name), "-o", os.path.join(bdir, stem + ".o")]
        else:
            continue
        objs.append(cmd[-1])
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, proc in jobs if proc.wait() != 0]
    if failed:
        raise RuntimeError("compilation failed: " + "; ".join(" ".join(c) for c in failed))
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
