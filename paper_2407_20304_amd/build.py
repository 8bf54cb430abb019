"""Build libholo.so (HIP kernels + host runtime) and libholo_plain.so (the
plain per-angle ray sums of the comparison baseline) for gfx950, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libholo.so")
SOURCES = ["holo_kernels.hip", "holo_radon.hip", "holo_api.cpp", "holo2d.hip", "holo2d_api.cpp", "holo_multires.hip",
           "holo_fs.hip"]
PLAIN_LIB = os.path.join(HERE, "libholo_plain.so")
PLAIN_SOURCES = [os.path.join("plain", "plain_radon.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 (v_pk_*_f32) is disabled for every device pass.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0].replace(os.sep, "_") + ".o")
    cmd = [HIPCC] + DEVICE_FLAGS + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, lib)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PLAIN_SOURCES
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(_compile, srcs))
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], PLAIN_LIB)
    if verbose:
        print("built", LIB, "and", PLAIN_LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
