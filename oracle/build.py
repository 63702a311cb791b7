"""Build the oracle's shared library (plain C, gcc).

TEST INFRASTRUCTURE ONLY.  The oracle is the CPU reference the GPU library
is checked against; building it is part of building the checker, and nothing
in the product path loads it.

The same source is compiled three times, for double, long double and
__float128, with -ffp-contract=off and no fast-math so that every operation
is one IEEE-rounded operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

# -ftree-vectorize lets gcc run the elementwise loops (the block update) on
# vector registers: each element still gets the same IEEE operations in the
# same order (no contraction, no reassociation), so results are unchanged.
# -fopenmp: the threaded block driver (pivots of a step on several threads).
CFLAGS = ["-O2", "-ftree-vectorize", "-fopenmp", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-std=gnu11", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False, srcdir=HERE, lib=LIB):
    """Compile the oracle sources in srcdir into lib (always rebuilds)."""
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    units = [
        ("ordering.c", [], "ordering.o"),
        ("jacobi.c", [], "jacobi_d.o"),
        ("jacobi.c", ["-DORC_LONG"], "jacobi_l.o"),
        ("jacobi.c", ["-DORC_QUAD"], "jacobi_q.o"),
    ]
    objs = []
    for src, defs, obj in units:
        out = os.path.join(objdir, obj)
        cmd = ["gcc", *CFLAGS, *defs, "-c", os.path.join(srcdir, src), "-o", out]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(out)
    tmp = lib + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
