"""Compile the HIP library libsdpdem.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("sdpdem_kernels.hip", "sdpdem_neighbors.hip",
                                                   "sdpdem_api.hip", "sdpdem_mlp.hip")]
LIB = os.path.join(HERE, "libsdpdem.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-I" + os.path.join(ROOT, "include"),
    # packed FP32 instructions stay disabled
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# measurement helpers of the benchmark (ALU and copy peaks), a library of
# their own: not part of the particle method's ABI
PEAKS_SOURCES = [os.path.join(HERE, "csrc", "sdpdem_peaks.hip")]
PEAKS_LIB = os.path.join(HERE, "libsdpdem_peaks.so")


def _hipcc(sources, lib, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = lib + ".tmp"
    cmd = [hipcc] + FLAGS + sources + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _hipcc(PEAKS_SOURCES, PEAKS_LIB, verbose)
    return _hipcc(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
