"""Build the SAD-instruction probe, a standalone measurement executable.

The probe is not part of libacbm: it backs the peak the benchmark divides by
(issue cost of the packed SAD instructions and the shader clock while they
run).  ``python probe/build.py`` writes ``probe/probe_sad`` next to its source;
``bench.py`` runs it when it is there.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "probe_sad.hip")
BIN = os.path.join(HERE, "probe_sad")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    tmp = BIN + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on the probe:\n{p.stderr}")
    os.replace(tmp, BIN)
    return BIN


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
