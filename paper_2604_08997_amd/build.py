"""Build the HIP library ``libsipo.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2604_08997_amd.build`` (or ``__graft_entry__.build()``).
Every ``csrc/*.hip`` source is compiled and linked into one shared library next
to this file.  Packed FP32 instructions are disabled for every kernel.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsipo.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object, then link libsipo.so; returns its path."""
    srcs = sources()
    tmp = tempfile.mkdtemp(prefix="sipo_build_")
    objs = []
    procs = []
    for src in srcs:
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        errs = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(errs))
        if verbose and errs:
            print("\n".join(errs))
    tmp_lib = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp_lib, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmp)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
