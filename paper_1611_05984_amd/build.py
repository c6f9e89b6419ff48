"""Build libwavestep.so (the gfx950 time step) and libwsprobe.so (HBM
streaming ceilings the benchmark measures beside it) in-tree with hipcc.

Packed FP32 instructions are disabled (-packed-fp32-ops); the libraries are
position independent and link only the HIP runtime.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "wavestep.hip")
LIB = os.path.join(HERE, "libwavestep.so")
PROBE_SRC = os.path.join(HERE, "csrc", "ws_probe.hip")
PROBE_LIB = os.path.join(HERE, "libwsprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def _hipcc(src: str, lib: str, verbose: bool) -> str:
    cmd = [HIPCC] + FLAGS + ["-o", lib + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building %s" % os.path.basename(lib))
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    _hipcc(PROBE_SRC, PROBE_LIB, verbose)
    return _hipcc(SRC, LIB, verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
