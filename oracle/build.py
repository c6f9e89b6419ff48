"""Build the FP64 CPU oracle library (test infrastructure) with gcc.

The oracle is plain C; it is compiled without fast-math and without
floating-point contraction so its results do not depend on the host's FMA
support.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wave_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source, loaded
# instead of LIB when WAVESTEP_ORACLE_SANITIZE=1 (the Python process then needs
# the ASan runtime preloaded: LD_PRELOAD=$(gcc -print-file-name=libasan.so)).
SAN_LIB = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = SAN_LIB if sanitize else LIB
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"] + san + [
           "-o", lib + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
