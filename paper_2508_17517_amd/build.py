"""Build libairg.so (HIP, gfx950) and the host-only test library in-tree.

    python -m paper_2508_17517_amd.build [--jobs N]

Every HIP translation unit is compiled with hipcc for gfx950 without FMA
contraction (the setup reproduces a sequential summation order bit for bit)
and without packed-FP32 instructions, then linked into one shared library.
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libairg.so")
HOST_LIB = os.path.join(HERE, "libairg_dense_host.so")
# the same host-only routines built with AddressSanitizer and UBSan (g++ only,
# for the CPU tests that run them under the sanitizers)
HOST_SAN_LIB = os.path.join(HERE, "libairg_dense_host_san.so")
GXX_SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"]

HIP_SOURCES = ["vec.hip", "spmv.hip", "cf.hip", "spgemm.hip", "order.hip", "fv.hip", "probe.hip", "coarse.hip",
               "dense.cpp", "hierarchy.cpp", "solve.cpp", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("AIRG_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + HIP_FLAGS
        _run(cmd)
        if verbose:
            print("compiled", src, flush=True)
        return obj

    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, HIP_SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, LIB)
    # host-only build of the dense routines for CPU tests
    gxx = shutil.which("g++") or "g++"
    _run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
          "-I", INCLUDE, "-I", CSRC, os.path.join(CSRC, "dense.cpp"),
          os.path.join(CSRC, "dense_host_shim.cpp"), "-o", HOST_LIB + ".tmp"])
    os.replace(HOST_LIB + ".tmp", HOST_LIB)
    host_sources = [os.path.join(CSRC, "dense.cpp"), os.path.join(CSRC, "dense_host_shim.cpp")]
    _run([gxx, "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-I", INCLUDE, "-I", CSRC]
         + GXX_SANITIZE + host_sources + ["-o", HOST_SAN_LIB + ".tmp"])
    os.replace(HOST_SAN_LIB + ".tmp", HOST_SAN_LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args(argv)
    print(build(a.jobs, verbose=True))


if __name__ == "__main__":
    sys.exit(main())
