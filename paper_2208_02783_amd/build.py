"""Builds librst.so (gfx950) in-tree with hipcc.  ``python -m paper_2208_02783_amd.build``.

Each kernel instance (stencil radius x positions per thread) is its own
translation unit so the instances compile in parallel; the host runtime is
one more unit; all are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librst.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
INSTANCES = [(2, 1), (2, 2), (6, 1), (6, 2)]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value", "-Wno-pass-failed",
]


def build(verbose: bool = False, jobs: int | None = None, out: str = LIB, defines=()) -> str:
    jobs = jobs or min(8, os.cpu_count() or 4)
    objdir = tempfile.mkdtemp(prefix="rstbuild_")
    units = []
    # heaviest first: the preconditioned solvers, then the plain solvers, then apply
    for kind in (4, 2, 6, 3, 0, 5, 1, 7):
        for rad, q in INSTANCES:
            units.append((os.path.join(CSRC, "kern_inst.hip"),
                          os.path.join(objdir, f"k{kind}_r{rad}_q{q}.o"),
                          [f"-DRST_RAD={rad}", f"-DRST_Q={q}", f"-DRST_KIND={kind}"]))
    procs = []
    units.append((os.path.join(CSRC, "rst_cnn.hip"), os.path.join(objdir, "rst_cnn.o"), []))
    units.append((os.path.join(CSRC, "rst_lib.hip"), os.path.join(objdir, "rst_lib.o"), []))
    pending = list(units)
    objs = []
    while pending or procs:
        while pending and len(procs) < jobs:
            src, obj, defs = pending.pop(0)
            cmd = [HIPCC, *FLAGS, *defs, *[f"-D{d}" for d in defines], "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), cmd))
            objs.append(obj)
        p, cmd = procs.pop(0)
        text = p.communicate()[0].decode(errors="replace")
        # hipcc's host pass warns that it does not know the device-only feature flag
        msgs = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            for q, _ in procs:
                q.wait()
            raise RuntimeError("hipcc failed: " + " ".join(cmd) + "\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs), flush=True)
    tmp = out + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    os.rmdir(objdir)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
