"""Build ``liboracle.so`` from ``fj_oracle.c`` (host C, FP64, OpenMP).

Test infrastructure: building the checker is not using it.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "fj_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
           src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
