"""Build the oracle shared library (test infrastructure only) with g++."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["hlbm_oracle.cpp", "hlbm_oracle_adjoint.cpp"]
HEADERS = ["hlbm_oracle.hpp", "hlbm_oracle_sim.hpp"]


def build(force: bool = True) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-o", LIB + ".tmp"] + srcs
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    """Build only when the library is missing or older than a source."""
    deps = [os.path.join(HERE, s) for s in SOURCES + HEADERS if os.path.exists(os.path.join(HERE, s))]
    if os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    return build()


if __name__ == "__main__":
    print(build())
    sys.exit(0)
