"""Build the HIP library ``libplds.so`` for gfx950 (and the workload generator).

``hipcc`` cross-compiles without a GPU.  The built library sits next to this
file so that it travels with the source tree.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "plds.hip")
LIB = os.path.join(HERE, "libplds.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PLDS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # no packed fp32 instructions anywhere (there is no float arithmetic on the path)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build_hip():
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + SRC)
    os.replace(tmp, LIB)
    return LIB


def build():
    from . import workloads
    workloads.build(force=True)
    return build_hip()


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_2106_03824_amd import build as b
    print(b.build())
