"""Builds liblbsc.so (the HIP library behind include/lbsc.h) for gfx950.

    python -m paper_1905_09554_amd.build

The library is compiled in-tree with hipcc; it is loaded by the ctypes
binding in this package.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbsc.so")
PROBE = os.path.join(PKG, "hbm_probe")
SOURCES = ["lbsc_device.hip", "lbsc_api.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # Packed FP32 instructions stay off: the compiler must not form them.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def hipcc():
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def build(verbose=False):
    """Compiles every source and links liblbsc.so; raises on failure."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + HIPCC_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    # Bandwidth calibration program (streaming kernels of known traffic).
    cmd = [hipcc(), os.path.join(CSRC, "hbm_probe.hip"), "-o", PROBE + ".tmp"] + [
        f for f in HIPCC_FLAGS if f not in ("-fPIC",)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE + ".tmp", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
