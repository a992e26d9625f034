"""Build libmofem.so in-tree for gfx950.

Host C++ (assembly, eigen-solver) is compiled with g++; the HIP sources
(kernels and the C-ABI layer) with hipcc for gfx950 only.  Packed FP32
instructions are disabled for all device code.  Usage:
    python -m paper_2109_01173_amd.build            # build
    python -m paper_2109_01173_amd.build --clean    # remove objects first
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmofem.so")

HOST_SOURCES = ["host_fem.cpp", "host_eigen.cpp", "host_chol.cpp"]
HIP_SOURCES = ["k_band_kb2.hip", "k_band_kb3.hip", "k_band_kb4.hip", "k_band_kb1.hip",
               "k_band.hip", "k_gemm.hip", "k_ozaki.hip", "k_vec.hip", "k_bchol.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")
ARCH = "gfx950"

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-mavx2", "-mfma", "-Wall", "-Wno-unused-function"]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass of hipcc warns that it does not know the packed-fp32 feature
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (p.returncode, " ".join(cmd), out))
    return out


def _stale(src, obj):
    """Object older than its source or any header / include file of csrc."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".inl"))]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "mofem.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def build(verbose=False, jobs=8, force=True):
    """Compile every source (force=True) or only stale objects, then link."""
    os.makedirs(BUILD, exist_ok=True)
    jobs_list = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        if force or _stale(os.path.join(CSRC, src), obj):
            jobs_list.append([CXX] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        if force or _stale(os.path.join(CSRC, src), obj):
            jobs_list.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, jobs_list))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(BUILD, s + ".o") for s in HOST_SOURCES + HIP_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--clean" in sys.argv and os.path.isdir(BUILD):
        shutil.rmtree(BUILD)
    print(build(verbose=True, force="--incremental" not in sys.argv))
