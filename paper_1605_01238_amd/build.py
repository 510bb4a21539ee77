"""Build the HIP library ``libwq.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["wq_plan.hip", "wq_setup_kernels.hip", "wq_contract.hip"]
LIB = os.path.join(HERE, "libwq.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, out: str = LIB, defines=()) -> str:
    """Compile every source into libwq.so (always recompiles).  ``defines``
    are extra -D settings (tuning knobs of the kernels)."""
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           # packed FP32 instructions are kept out of the device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-o", tmp] + [f"-D{d}" for d in defines] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
