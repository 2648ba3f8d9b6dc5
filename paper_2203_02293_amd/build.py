"""Build the gfx950 HIP library (``librt_mi355x.so``) in-tree with hipcc."""
from __future__ import annotations

import os
import pathlib
import subprocess

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "librt_mi355x.so"
SOURCES = [CSRC / "rt_kernels.hip", CSRC / "rt_deep.hip", CSRC / "rt_optics.hip", CSRC / "rt_api.hip"]
HEADERS = [CSRC / "rt_internal.hpp", CSRC / "rt_math.hpp", CSRC / "rt_physics.hpp",
           CSRC / "rt_wave.hpp", ROOT / "include" / "rt.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: the kernels use scalar FP32 forms only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def stale() -> bool:
    if not LIB.exists():
        return True
    t = LIB.stat().st_mtime
    return any(p.stat().st_mtime > t for p in SOURCES + HEADERS)


def build(verbose: bool = False) -> pathlib.Path:
    """Compile every HIP source into the shared library (always recompiles)."""
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, *FLAGS, f"-I{ROOT / 'include'}", f"-I{CSRC}",
           *map(str, SOURCES), "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
