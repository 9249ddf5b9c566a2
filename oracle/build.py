"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

compiles ``moa_oracle.c`` into ``oracle/liboracle.so`` with gcc, OpenMP and
no FP contraction, so every floating-point operation in it is one IEEE
operation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "moa_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = OUT, sanitize: bool = False) -> str:
    """Build the oracle library at `out`. sanitize: instrument it with
    AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal); the
    process that loads it must preload gcc's libasan."""
    tmp = out + ".tmp%d" % os.getpid()
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter"] + san + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
