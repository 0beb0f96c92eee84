"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain C, gcc, -O2 with floating-point contraction off so that every
expression is evaluated in the order it is written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vup_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
SAN_SRC = os.path.join(HERE, "san_check.c")
SAN_OUT = os.path.join(HERE, "san_check")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def build_sanitized(verbose: bool = False) -> str:
    """The oracle with its sanitizer harness (san_check.c) as one host
    executable under AddressSanitizer and UndefinedBehaviorSanitizer, every
    report fatal. CPU only; the GPU library is never built this way."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas", SRC, SAN_SRC,
           "-o", SAN_OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_OUT + ".tmp", SAN_OUT)
    return SAN_OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
