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
OUT_SANITIZED = os.path.join(HERE, "liboracle_sanitized.so")


def build(verbose: bool = False, sanitized: bool = False) -> str:
    """sanitized: an AddressSanitizer + UndefinedBehaviorSanitizer build (any
    report aborts) for running the oracle's tests under the sanitizers; a
    process that loads it needs libasan preloaded."""
    out = OUT_SANITIZED if sanitized else OUT
    tmp = out + ".tmp"
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all"] if sanitized else ["-O2"]
    cmd = [
        os.environ.get("CC", "gcc"), *opt, "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC, "-o", tmp, "-lquadmath", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitized="--sanitized" in sys.argv))
