"""Build libsmm.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsmm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# gfx950 only; packed FP32 instructions disabled for the device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    units = (
        ("host_setup.cpp", ["-x", "hip", *DEVICE_FLAGS, "-ffp-contract=off"]),
        ("api.cpp", ["-x", "hip", *DEVICE_FLAGS]),
        ("typed.cpp", ["-x", "hip", *DEVICE_FLAGS, "-ffp-contract=off"]),
        ("batch.cpp", ["-x", "hip", *DEVICE_FLAGS]),
        ("cnn.cpp", ["-x", "hip", *DEVICE_FLAGS]),
        ("mg.cpp", ["-x", "hip", *DEVICE_FLAGS]),
        ("cg_smm.cpp", ["-x", "hip", *DEVICE_FLAGS, "-ffp-contract=off"]),
        ("cg_smm.hip", DEVICE_FLAGS),
        ("kernels.hip", DEVICE_FLAGS),
        ("cnn_kernels.hip", DEVICE_FLAGS),
    )
    objs = [os.path.join(objdir, src + ".o") for src, _ in units]
    cmds = [[HIPCC, *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj] for (src, flags), obj in zip(units, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        list(ex.map(_run, cmds))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
