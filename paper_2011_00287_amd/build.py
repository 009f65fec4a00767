"""Build the HIP library for gfx950: ``python -m paper_2011_00287_amd.build``.

Compiles csrc/lb_api.hip (the 3D coupled step; it includes every 3D kernel
header) and csrc/nematic2d.hip (the 2D active nematic) into lib/liblbchiral.so
with hipcc.  Packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRCS = [os.path.join(PKG, "csrc", "lb_api.hip"), os.path.join(PKG, "csrc", "nematic2d.hip")]
OUT = os.path.join(PKG, "lib", "liblbchiral.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# sources the 3D step's kernels and their launch configuration are built from
STEP_SOURCES = ("physics.hpp", "storage.hpp", "kernels_fused.hpp", "kernels_step.hpp", "kernels_pc.hpp",
                "kernels_site.hpp", "kernels_reduce.hpp", "kernels_adjoint.hpp", "kernels_pc_adjoint.hpp",
                "adjoint.hpp", "lb_api.hip")


def kernel_source_hash() -> str:
    """Hash of the 3D step's HIP sources without comments and blank lines: hardware counters are valid only
    for the code they were taken on, and an edit of a comment leaves that code as it was."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(PKG, "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(line.rstrip() for line in text.splitlines() if line.strip()).encode())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
