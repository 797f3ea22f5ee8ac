"""Build the gfx950 shared library libpdlp_hip.so in place (hipcc, no torch extension).

    python -m paper_2106_04756_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdlp_hip.so")

SOURCES = ["pdlp_solver.hip", "host_prep.cpp"]
HEADERS = ["pdlp_kernels.hip", "pdlp_batch.hip", "pdlp_batch_host.hip", "pdlp_unroll.hip", "pdlp_device.h", "pdlp_internal.h",
           "host_prep.h"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the float64 arithmetic is kept unfused so the rounding of each PDHG formula matches a
    # plain evaluation of it term by term
    "-ffp-contract=off",
    # packed fp32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile the library (always; the output is replaced atomically)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
