"""Build the CPU oracle library (test infrastructure only).

Compiles ``acbm_oracle.c`` with the system C compiler into
``liboracle_acbm.so`` next to this file.  Plain ``-O2``: no intrinsics, no
vectorisation pragmas, no threads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "acbm_oracle.c")
LIB = os.path.join(HERE, "liboracle_acbm.so")
CFLAGS = ["-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, *CFLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
