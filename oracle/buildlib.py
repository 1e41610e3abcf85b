"""Build step for the FP64 CPU oracle (test infrastructure only).

gcc with plain IEEE double arithmetic (no -ffast-math, no FMA contraction, so
every multiply and add rounds as written) and OpenMP over independent views or
rows.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lfsr_oracle.c")
OUT = os.path.join(HERE, "liblfsr_oracle.so")


def build_oracle(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_oracle(verbose=True))
