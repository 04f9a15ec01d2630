"""Build the FP64 CPU oracle (test infrastructure only) with the host C compiler.

    python oracle/build.py          # writes oracle/liboracle.so

The oracle is plain C compiled by gcc with OpenMP over collision cells and
libquadmath for the binary128 boosts; it shares no source with the GPU library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "compton_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [
        os.environ.get("CC", "gcc"), "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC, "-o", tmp, "-lquadmath", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
