"""Compile the HIP library (and its test-hook library) for gfx950, in tree.

Flags that matter for the results:
  -ffp-contract=off      no implicit fused multiply-adds (the rule spells its FMAs out)
  (no fast-math)         '/' and sqrtf stay correctly rounded, denormals are kept
  -packed-fp32-ops off   no v_pk_*_f32 instructions are generated
"""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "librotvote.so"
PROBE_LIB = PKG / "librotvote_probe.so"

ARCH = os.environ.get("ROTVOTE_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or Path(c).exists()):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> list[Path]:
    """Build librotvote.so and librotvote_probe.so next to this file."""
    hipcc = _hipcc()
    jobs = [
        (LIB, [CSRC / "rv_kernels.hip", CSRC / "rv_bin.hip", CSRC / "rv_batch.hip",
               CSRC / "rv_refine.hip", CSRC / "rv_multi.hip", CSRC / "rv_rigid.hip",
               CSRC / "rv_static.hip", CSRC / "rv_api.cpp",
               CSRC / "rv_serve.cpp"]),
        (PROBE_LIB, [CSRC / "rv_probe.hip", CSRC / "rv_ceil.hip"]),
    ]
    out = []
    for lib, srcs in jobs:
        tmp = lib.with_suffix(".so.tmp")
        cmd = [hipcc, *HIPCC_FLAGS, "-o", str(tmp), *map(str, srcs)]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
        out.append(lib)
    return out


if __name__ == "__main__":
    for p in build(verbose=True):
        print("built", p)
