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


def _gcc(src: str, out: str, prec: str, verbose: bool = False) -> None:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-DREAL=%s" % REALS[prec], src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> None:
    for prec, out in LIBS.items():
        _gcc(SRC, out, prec, verbose)


def build_planted(old: str, new: str, workdir: str, prec: str) -> str:
    """Compile a copy of oracle.c in which the one occurrence of ``old`` is
    replaced by ``new`` (a deliberate mistake), into ``workdir``; returns the
    library's path.  Used by tests that show a pin fails on a wrong oracle."""
    text = open(SRC).read()
    if text.count(old) != 1:
        raise ValueError("planted mistake must replace exactly one occurrence of %r" % old)
    src = os.path.join(workdir, "planted.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    out = os.path.join(workdir, "liboracle_planted_%s.so" % prec)
    _gcc(src, out, prec)
    return out


def built() -> bool:
    return all(os.path.exists(p) and os.path.getmtime(p) >= os.path.getmtime(SRC)
               for p in LIBS.values())


if __name__ == "__main__":
    build(verbose=True)
