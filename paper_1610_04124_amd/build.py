"""Build step of the HIP library: hipcc for gfx950 into an in-tree shared object.

    python -m paper_1610_04124_amd.build                  libstixels.so
    python -m paper_1610_04124_amd.build --phase-timing   libstixels_phases.so: the
        same kernels with shader-clock stamps at each phase of a column task in
        the persistent kernel (profiling only; loaded when STIXELS_PHASE_TIMING=1)
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB = os.path.join(_HERE, "libstixels.so")
PHASES_LIB = os.path.join(_HERE, "libstixels_phases.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",                       # keep the exact-grid arithmetic un-fused
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    """Every HIP unit, the per-slot-count kernel units with the most rows
    (the slowest to compile) first."""
    def key(path):
        name = os.path.basename(path)
        if name.startswith("inst_s"):
            return (0, -int(name[len("inst_s"):-len(".hip")]))
        return (1, name)
    return sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")), key=key)


def build(verbose: bool = False, phase_timing: bool = False) -> str:
    """Compiles every source to an object in parallel, then links the library."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(_HERE, "csrc")]
    if phase_timing:
        inc.append("-DSTX_PHASE_TIMING=1")
    lib_path = PHASES_LIB if phase_timing else LIB
    with tempfile.TemporaryDirectory(prefix="stixels_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[HIPCC, *FLAGS, *inc, "-c", src, "-o", obj]
                for src, obj in zip(sources(), objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            list(ex.map(run, cmds))
        tmp = lib_path + ".tmp"
        run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
        os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_timing="--phase-timing" in sys.argv))
