"""Compiles the HIP library libjatam.so for gfx950, in-tree.

    python -m paper_2205_15311_amd.build_lib [-v]
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjatam.so")
SOURCES = ["jatam_plain.hip", "jatam_batched.hip", "jatam_ga.hip", "jatam_mlp.hip",
           "jatam_select.hip", "jatam_tally.hip", "jatam_static.hip", "jatam_truth.hip",
           "jatam_neighbourhood.hip", "jatam_roulette.hip", "jatam_api.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (the integer kernels need none)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: cannot build the gfx950 library")
    return path


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links the library."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def compile_one(name):
        obj = os.path.join(objdir, name + ".o")
        cmd = [hipcc()] + compile_flags + ["-c", "-o", obj, os.path.join(CSRC, name)]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        return obj, res

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(compile_one, SOURCES))
    failed = [res for _, res in results if res.returncode != 0]
    if failed:
        for res in failed:
            sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to compile libjatam.so's sources")
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + \
        [obj for obj, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link libjatam.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
