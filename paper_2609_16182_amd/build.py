"""Build libpsl.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2609_16182_amd.build

Flags: -ffp-contract=off keeps every a*b+c as a separate multiply and add
(the round semantics are defined in IEEE double without fused operations);
no fast-math, so double division stays correctly rounded; packed FP32
instructions are disabled.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpsl.so")
ARCH = os.environ.get("PSL_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-pthread", "-Wl,--no-undefined",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: libpsl needs the ROCm toolchain")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


PROBE = os.path.join(HERE, "libpsl_probe.so")


def build_probe(verbose=False):
    """Compile the gather-rate probe (probe/*.hip) into libpsl_probe.so."""
    tmp = PROBE + f".tmp{os.getpid()}"
    cmd = [hipcc(), *FLAGS, *sorted(glob.glob(os.path.join(HERE, "probe", "*.hip"))), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpsl_probe.so")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose=False):
    """Compile every HIP source into libpsl.so (always rebuilds)."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *FLAGS, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpsl.so")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
