"""Compile the plain C oracle (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(force=True):
    out = os.path.join(HERE, "liboracle.so")
    if not force and os.path.exists(out):
        return out
    srcs = [os.path.join(HERE, f) for f in ("symmspmv.c", "gauss_seidel.c", "kaczmarz.c")]
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, *srcs], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
