"""Build the FP64 CPU oracle (test infrastructure) with gcc: the 2D method
(oracle.c) and the lattice of its 3D extension (oracle3d.c) in one library.

The oracle is plain C; it is compiled without fast-math or FMA contraction so
that its double-precision arithmetic follows the source order.  OpenMP splits
its independent per-node loops over threads (results do not depend on the
thread count).  ``build(sanitize=True)`` writes a separate copy built with
AddressSanitizer and UndefinedBehaviorSanitizer for the CPU sanitizer test.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle3d.c")]
    out = LIB_SAN if sanitize else LIB
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function"]
    if sanitize:
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd += srcs + ["-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
