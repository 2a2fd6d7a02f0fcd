"""Builds libmpk.so (HIP kernels for gfx950 + host planner + C ABI) in-tree.

Each source is compiled to its own object in parallel, then one link step
makes the shared library."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpk.so")
SOURCES = [os.path.join(HERE, "csrc", "planner.cpp"), os.path.join(HERE, "csrc", "mpk.hip"),
           os.path.join(HERE, "csrc", "server.cpp"), os.path.join(HERE, "csrc", "gmres.hip"),
           os.path.join(HERE, "csrc", "cache.cpp")]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="mpk_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", s, "-o", o]
                for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(len(cmds)) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed compiling a libmpk.so source")
        tmp = LIB + ".tmp"
        link = [hipcc, *FLAGS, "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libmpk.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
