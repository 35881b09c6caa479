"""Build the S^5 HIP library ``libs5.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libs5.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


# the write-check build: the same library with every output write counted
# (s5_debug_count_writes); used by the tests only
OUT_WCHECK = os.path.join(PKG, "libs5_wcheck.so")


def _compile(src, extra=(), tag=""):
    obj = os.path.join(BUILD_DIR, src + tag + ".o")
    out = _run([HIPCC, "-x", "hip", *DEVICE_FLAGS, *extra, "-c", os.path.join(CSRC, src),
                "-o", obj])
    return obj, out


def _link(objs, out):
    tmp = out + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = {}
    for src in ("s5_kernels.hip", "s5_learn.hip", "s5_host.cpp"):
        objs[src], out = _compile(src)
        if verbose and out.strip():
            print(out)
    _link(list(objs.values()), OUT)
    wc, _ = _compile("s5_kernels.hip", ("-DS5_COUNT_WRITES",), ".wcheck")
    _link([wc, objs["s5_learn.hip"], objs["s5_host.cpp"]], OUT_WCHECK)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
