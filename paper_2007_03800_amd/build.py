"""Build libsdl.so (HIP, gfx950 only) in-tree with hipcc.

Usage: python -m paper_2007_03800_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsdl.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain scalar/vector FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed (exit %d): %s" % (res.returncode, cmd[-1]))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object (in parallel; no device code crosses files),
    then link the shared library.  Always a full rebuild."""
    from concurrent.futures import ThreadPoolExecutor

    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    cflags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="sdl_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src)[:-4] + ".o") for src in sources()]
        cmds = [[HIPCC, *cflags, *inc, "-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        n = jobs or min(8, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=n) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
