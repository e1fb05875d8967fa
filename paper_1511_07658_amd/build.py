"""Build libgvm.so (and the micro-benchmark) for gfx950 with hipcc.

    python -m paper_1511_07658_amd.build [--clean]

Objects go to ``_build/`` at the repository root; the library lands next to
this file as ``libgvm.so`` so that it travels with the source tree.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgvm.so")
MICROBENCH = os.path.join(PKG, "gvm_microbench")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Every HIP translation unit is built for gfx950 only.  Packed FP32 is turned
# off in the device code generator: hipcc would otherwise form v_pk_* FP32
# instructions by itself.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{INCLUDE}", f"-I{CSRC}",
              "-I/opt/rocm/include"]

LIB_SOURCES = [
    ("stream_kernels.hip", "hip"),
    ("sgemm.hip", "hip"),
    ("ep_kernels.hip", "hip"),
    ("device_hip.cpp", "hip"),
    ("plain.cpp", "hip"),
    ("plain_noalloc.hip", "hip"),
    ("batch_plan.cpp", "host"),
    ("device_loopback.cpp", "host"),
    ("manager.cpp", "host"),
    ("rank.cpp", "host"),
    ("shm.cpp", "host"),
    ("common.cpp", "host"),
    ("copy_pool.cpp", "host"),
    ("abi.cpp", "host"),
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in p.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in line)
    return p.returncode, out


def _compile(src, kind):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if kind == "hip":
        cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = ["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    rc, out = _run(cmd)
    return src, rc, out, obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libgvm.so; returns the library path."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        results = list(ex.map(lambda s: _compile(*s), LIB_SOURCES))
    errors = [(s, out) for s, rc, out, _ in results if rc != 0]
    for s, rc, out, _ in results:
        if verbose and out.strip():
            print(f"[{s}]\n{out}")
    if errors:
        msg = "\n".join(f"--- {s}\n{out}" for s, out in errors)
        raise RuntimeError(f"compilation failed:\n{msg}")
    objs = [o for *_, o in results]
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrt", "-lpthread", "-ldl"])
    if rc != 0:
        raise RuntimeError(f"link failed:\n{out}")
    os.replace(tmp, LIB)
    rc, out = _run([HIPCC, *HIP_FLAGS, os.path.join(CSRC, "microbench.hip"), "-o", MICROBENCH + ".tmp"])
    if rc != 0:
        raise RuntimeError(f"micro-benchmark build failed:\n{out}")
    os.replace(MICROBENCH + ".tmp", MICROBENCH)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--clean", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    if a.clean and os.path.isdir(BUILD):
        shutil.rmtree(BUILD)
    print(build(verbose=a.verbose))
    return 0


if __name__ == "__main__":
    sys.exit(main())
