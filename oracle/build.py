"""Build the CPU oracle library (test infrastructure only).

    python oracle/build.py

Compiles ``oracle/fhtp_oracle.c`` with gcc and OpenMP into
``oracle/liboracle_fhtp.so``.  No ``-march=native``: the library is built here
and may run on another host.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fhtp_oracle.c")
OUT = os.path.join(HERE, "liboracle_fhtp.so")


def build(verbose: bool = False, src: str = SRC, out: str = OUT) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
