"""Builds liboracle.so (lbm_oracle.c, D2Q9) and liboracle3.so (lbm_oracle3.c,
D3Q19) with gcc (test infrastructure)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SRC3 = os.path.join(HERE, "lbm_oracle3.c")
LIB3 = os.path.join(HERE, "liboracle3.so")


def _build_one(src, lib, force):
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(src):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-std=c11", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


NATIVE_FLAGS = ["-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11"]


def build_native(out: str) -> str:
    """The D2Q9 oracle compiled for the host it runs on (-O3 -march=native;
    contraction stays off, so the arithmetic is that of the in-tree build),
    for timing the CPU baseline."""
    tmp = out + ".tmp"
    r = subprocess.run(["gcc", *NATIVE_FLAGS, "-o", tmp, SRC, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    _build_one(SRC3, LIB3, force)
    return _build_one(SRC, LIB, force)


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
