"""Build the oracle's C line operator (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` compiles
``oracle/lines.c`` with gcc into ``oracle/_oracle_lines.so``.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lines.c")
LIB = os.path.join(HERE, "_oracle_lines.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
