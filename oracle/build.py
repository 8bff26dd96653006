"""Builds the CPU oracle into oracle/libjatam_oracle.so with gcc.

Test infrastructure: the oracle is the independent CPU checker of the HIP
library; this script only compiles it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "jatam_oracle.c"), os.path.join(HERE, "jatam_ga_oracle.c"),
        os.path.join(HERE, "jatam_roulette_oracle.c")]
LIB = os.path.join(HERE, "libjatam_oracle.so")


# -O3 for the CPU baseline's timing; x86-64-v3 (AVX2, BMI2, POPCNT) rather than
# -march=native because the library is built here and loaded on other hosts
# (any AVX2-capable x86-64 runs it).
def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-Werror", "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
