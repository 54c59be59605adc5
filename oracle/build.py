"""Compile the CPU oracle (plain C, FP64, no FMA contraction) into oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cqsim_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source with AddressSanitizer and UndefinedBehaviorSanitizer (CPU
# checks of the oracle: load it with CQ_ORACLE_LIB and libasan preloaded)
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

CFLAGS = ["-O2", "-msse4.1", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, *(SAN_FLAGS if sanitize else []), "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
