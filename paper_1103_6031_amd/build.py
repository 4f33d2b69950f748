"""Build libmgic.so (HIP for gfx950) in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only, with FP contraction off (the arithmetic
order written in the kernels is the order executed) and packed FP32 instructions disabled.
`build(out=..., csrc=...)` builds a variant library from another source directory (A/B timing).
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmgic.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]
SOURCES = ["k_multigrid.hip", "k_levels.hip", "k_lpt.hip", "k_highorder.hip", "k_fft.hip", "k_density.hip",
           "solver.cpp", "spectral.cpp", "density.cpp", "batch_hier.cpp"]


def _compile(args):
    src, objdir, defines, csrc = args
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = ([HIPCC] + FLAGS + ["-I" + csrc] + ["-D" + d for d in defines] + lang +
           ["-c", os.path.join(csrc, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=True, out=LIB, defines=(), csrc=CSRC):
    tag = "_".join(defines) if defines else "default"
    if csrc != CSRC:
        tag += "_" + os.path.basename(os.path.dirname(os.path.abspath(csrc)))
    objdir = os.path.join(ROOT, "_build", tag)
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, [(s, objdir, list(defines), csrc) for s in SOURCES]))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
