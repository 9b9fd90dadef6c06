"""Builds the HIP library ``librelaybp.so`` in-tree for gfx950, and the LDS
bandwidth probe ``liblds_peak.so`` that measures the LDS roofline's peak.

Flags: -ffp-contract=off keeps the canonical FP32 operation order (no fused
multiply-add); the packed-FP32 target feature is switched off so the compiler
never emits packed FP32 arithmetic.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librelaybp.so")
LDS_PEAK_LIB = os.path.join(HERE, "liblds_peak.so")
SOURCES = ["relay_kernels.hip", "relay_block.hip", "relay_block16.hip", "relay_large.hip", "relay_train.hip",
           "relay_api.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def _hipcc(out: str, sources, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-shared", "-o", tmp] + [os.path.join(CSRC, s) for s in sources]
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if verbose or res.returncode != 0:
        print(res.stdout)
        print(res.stderr)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(LDS_PEAK_LIB, ["lds_peak.hip"], verbose)
    return _hipcc(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
