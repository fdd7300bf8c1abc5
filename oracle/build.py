"""Build the CPU oracle shared library (oracle/liboracle.so) with gcc.

TEST INFRASTRUCTURE ONLY.  The oracle is compiled at -O2 with FMA
contraction off, IEEE semantics (no fast-math), and OpenMP over nodes; the
step source is compiled twice, once in real and once in complex arithmetic
(complex-step derivatives).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose=False):
    objs = []
    units = [("lbm_oracle.c", [], "oracle_re.o"),
             ("lbm_oracle.c", ["-DORC_COMPLEX"], "oracle_cx.o"),
             ("thermo.c", [], "thermo.o")]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src, defs, obj in units:
        out = os.path.join(bdir, obj)
        cmd = ["gcc", *CFLAGS, *defs, "-c", os.path.join(HERE, src), "-o", out]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(out)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
