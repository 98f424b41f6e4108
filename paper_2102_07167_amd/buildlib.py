"""Build the gfx950 shared library ``libkur.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libkur.so")
SOURCES = ["kur_kernels.hip", "ens_kernels.hip", "persist_kernels.hip", "io_kernels.hip", "noalloc.hip", "kur_api.cpp", "graph_build.cpp", "autotune.cpp",
           "ensemble.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-pthread",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP/C++ source of the library into libkur.so (always, when force)."""
    if not force and os.path.exists(SO):
        return SO
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
