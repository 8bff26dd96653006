"""Builds the CPU oracle into oracle/libjatam_oracle.so with gcc.

Test infrastructure: the oracle is the independent CPU checker of the HIP
library; this script only compiles it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "jatam_oracle.c"), os.path.join(HERE, "jatam_ga_oracle.c")]
LIB = os.path.join(HERE, "libjatam_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-Werror", "-o", LIB + ".tmp"] + SRCS
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
