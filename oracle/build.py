"""Build the CPU oracle libraries (fp32 and fp64) with gcc.

Test infrastructure: compiled here so the checker exists on every machine
that runs the tests; the product library never links or loads it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIBS = {"f32": os.path.join(HERE, "liboracle_f32.so"),
        "f64": os.path.join(HERE, "liboracle_f64.so")}
REALS = {"f32": "float", "f64": "double"}


def build(verbose: bool = False) -> None:
    for prec, out in LIBS.items():
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-std=c99", "-Wall", "-DREAL=%s" % REALS[prec], SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def built() -> bool:
    return all(os.path.exists(p) and os.path.getmtime(p) >= os.path.getmtime(SRC)
               for p in LIBS.values())


if __name__ == "__main__":
    build(verbose=True)
