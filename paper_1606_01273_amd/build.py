"""Build libcaspt2.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["engine.cpp", "kernels.hip", "couple.hip", "couple_ccvv.hip", "couple_cavv.hip", "gemm_f32.hip", "pcg_kernels.hip", "density.hip", "noalloc.hip", "caspt2.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-fvisibility=hidden", "-fvisibility-inlines-hidden",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wl,--no-undefined"]   # every referenced symbol must be defined or in a linked library


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "libcaspt2.so")
    tmp = out + ".tmp"
    cmd = ["hipcc", *FLAGS, *[os.path.join(HERE, "csrc", s) for s in SRC], "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=False))
