"""Build the oracle's C part (test infrastructure) with gcc.

The oracle is plain FP64 C compiled with -O3 -ffp-contract=off so that its
rounding does not depend on FMA contraction, for x86-64-v3 (AVX2; the
library is built once and also runs on other x86 hosts, so it is not tied
to the build machine with -march=native).  It is independent of the HIP
library: no shared sources, headers or build steps.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["aqif_lcp.c"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    """Build if the library is missing or older than a source."""
    if os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(os.path.join(HERE, s)) <= t for s in SOURCES):
            return LIB
    return build()


if __name__ == "__main__":
    print(build(verbose=True))
