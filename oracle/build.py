"""Build step of the CPU oracles (stixels and the semi-global matching stage):
plain gcc, FP64, no fast-math, OpenMP over columns."""

from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build_oracle(force: bool = True) -> str:
    out = os.path.join(_HERE, "libstixel_oracle.so")
    srcs = [os.path.join(_HERE, "stixel_oracle.c"), os.path.join(_HERE, "sgm_oracle.c")]
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-fPIC",
           "-shared", "-fopenmp", *srcs, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(force=True))
