"""Build libfc.so (HIP kernels + host planner + C ABI) for gfx950 in-tree.

Usage: python -m paper_2008_00672_amd.build   (or __graft_entry__.build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfc.so")

# (source, extra defines): the device code is built once per I/O storage type
UNITS = [("fc_kern_io.hip", ["-DFC_IO=0"]), ("fc_kern_io.hip", ["-DFC_IO=1"]), ("fc_kern_io.hip", ["-DFC_IO=2"]),
         ("fc_launch.cpp", []), ("fc_plan.cpp", []), ("fc_graph.cpp", []), ("fc_scratch.hip", [])]

# Packed FP32 VALU forms are kept out of the generated code; the compiler
# otherwise forms them from float2 arithmetic.
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose=False, jobs=None):
    """Compile every unit to an object (in parallel), then link libfc.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for k, (src, defs) in enumerate(UNITS):
        obj = os.path.join(objdir, "%d_%s.o" % (k, os.path.splitext(src)[0]))
        cmd = [hipcc()] + HIP_FLAGS + defs + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
                                              os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(" ".join(cmd) + "\n" + out + err)
    if failed:
        raise RuntimeError("hipcc failed building libfc.so")
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIP_FLAGS + ["-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libfc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
