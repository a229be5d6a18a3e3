"""Build the HIP solver library ``libbse.so`` in-tree for gfx950.

Run ``python -m paper_2008_08825_amd.build`` (or ``__graft_entry__.build()``).
Every call recompiles all sources.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbse.so")

SOURCES = ["capi.hip", "gemm.hip", "chol.hip", "jacobi.hip", "finalize.hip", "refine.hip",
           "adjoint.hip", "batched.hip", "checks.hip",
           "noalloc.hip", "window.hip", "form2.hip"]

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP solver cannot be built")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object, link ``libbse.so``, return its path."""
    cc = hipcc()
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs[:1])
            procs = procs[1:]
    _drain(procs)
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        raise RuntimeError("link of libbse.so failed:\n" + out.stdout)
    os.replace(tmp, LIB)
    return LIB


def _drain(procs):
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
        lines = [ln for ln in text.splitlines()
                 if "packed-fp32-ops" not in ln and ln.strip()]
        if lines:
            sys.stderr.write(f"[{src}]\n" + "\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
