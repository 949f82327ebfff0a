"""Builds libwvl.so in this package directory for gfx950 (MI355X).

    python -m paper_1401_7441_amd.build

Steps: regenerate csrc/wvl_filters.h (gen_filters), compile the HIP kernels
with hipcc (packed FP32 instructions disabled), compile the host side with g++
(-ffp-contract=off: the sphere membership test must round as written), link
against the HIP runtime that torch loads (one runtime per process).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwvl.so")
BENCH_BIN = os.path.join(HERE, "wvl_bench")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-mllvm", "-pragma-unroll-threshold=1000000",
               "-Wall", "-Wno-unused-result"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _torch_lib_dir():
    """The HIP runtime must be the one torch loads: torch's streams and device
    pointers belong to it, and a second runtime in the process sees no device."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        raise RuntimeError("torch is required: its HIP runtime hosts the library")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def build(regen_filters: bool = True) -> str:
    if regen_filters:
        from . import gen_filters
        gen_filters.write_header(os.path.join(CSRC, "wvl_filters.h"))
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    kobjs = []
    for src in ("wvl_kernels.hip", "wvl_fused.hip", "wvl_static.hip"):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        _run([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        kobjs.append(obj)
    hobj = os.path.join(bdir, "wvl_host.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fopenmp", "-Wall",
          "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c",
          os.path.join(CSRC, "wvl_host.cpp"), "-o", hobj])
    tmp = LIB + ".tmp"
    tlib = _torch_lib_dir()
    # plain host link: the device code is already embedded in wvl_kernels.o
    _run(["g++", "-shared", "-fPIC", "-fopenmp", "-o", tmp, *kobjs, hobj, f"-L{tlib}", "-l:libamdhip64.so",
          f"-Wl,-rpath,{tlib}", "-Wl,--no-undefined"])
    os.replace(tmp, LIB)
    # native driver (own HIP runtime from the ROCm install, no torch)
    bobj = os.path.join(bdir, "wvl_bench_main.o")
    _run([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "wvl_bench_main.hip"), "-o", bobj])
    tmpb = BENCH_BIN + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-fopenmp", "-o", tmpb, bobj, *kobjs, hobj])
    os.replace(tmpb, BENCH_BIN)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
