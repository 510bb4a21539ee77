"""Build the HIP library ``libwq.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["wq_plan.hip", "wq_setup_kernels.hip", "wq_contract.hip", "wq_batch.hip"]
LIB = os.path.join(HERE, "libwq.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, out: str = LIB, defines=()) -> str:
    """Compile every source into libwq.so (always recompiles; one hipcc per
    source, in parallel, then one link).  ``defines`` are extra -D settings
    (tuning knobs of the kernels)."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    flags = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             # packed FP32 instructions are kept out of the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include")] + [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory() as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc()] + flags + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        tmp = out + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(len(cmds)) as ex:
            results = list(ex.map(run, cmds))
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed")
        r = run(link)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc link failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
