"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no fast-math and no floating-point contraction, so every operation
rounds exactly as written in mpdata_oracle.c.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["mpdata_oracle.c"]
OUT = os.path.join(HERE, "liboracle.so")
# the same source with its stage loops shared among threads (OpenMP over the
# outermost loop): the multi-core CPU baseline; same bits as OUT
OUT_OMP = os.path.join(HERE, "liboracle_omp.so")


def _gcc(out, extra, verbose):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra"] + extra + ["-o", out + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    _gcc(OUT_OMP, ["-fopenmp"], verbose)
    return _gcc(OUT, ["-Wno-unknown-pragmas"], verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
