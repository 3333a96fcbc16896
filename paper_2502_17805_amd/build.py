"""Build the gfx950 library in-tree: paper_2502_17805_amd/libsdmhd.so.

The HIP kernels and the C ABI are compiled with hipcc for gfx950 (packed FP32
instructions disabled); the host mesh/metric code is compiled with g++ and
OpenMP and linked in.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsdmhd.so")
ARCH = os.environ.get("SDM_OFFLOAD_ARCH", "gfx950")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True, defines=(), out=None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    host_o = os.path.join(BUILD, "sdm_host.o")
    kern_o = os.path.join(BUILD, "sdm_kernels.o")
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-fopenmp", "-Wall", "-c",
          os.path.join(CSRC, "sdm_host.cpp"), "-o", host_o])
    _run(["hipcc", f"--offload-arch={ARCH}", "-std=c++17", "-O3", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, "sdm_kernels.hip"), "-o", kern_o])
    lib = out or LIB
    tmp = lib + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, kern_o, host_o, "-lgomp"])
    os.replace(tmp, lib)
    if out is None:
        build_c_driver(lib)
    return lib


def build_c_driver(lib=LIB) -> str:
    """The plain C caller of the ABI that the GPU tests run
    (tests/c/abi_step.c): HIP runtime API only, linked against the library."""
    root = os.path.dirname(HERE)
    src = os.path.join(root, "tests", "c", "abi_step.c")
    exe = os.path.join(root, "tests", "c", "abi_step")
    if not os.path.exists(src):
        return ""
    _run(["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", exe,
          f"-L{os.path.dirname(lib)}", "-lsdmhd", "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,$ORIGIN/../../paper_2502_17805_amd", "-Wl,-rpath,/opt/rocm/lib"])
    return exe


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--define", action="append", default=[], metavar="NAME=VALUE",
                    help="extra preprocessor definition for the kernels (e.g. SDM_MFMA_INTERP=1)")
    build(defines=ap.parse_args().define)
    sys.exit(0)
