"""Build the HIP library liblbfe.so for gfx950 in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liblbfe.so")
SOURCES = ["lbfe_api.hip", "lbfe_kernels.hip", "lbfe_chain.hip", "lbfe_fused.hip", "lbfe_moment.hip", "lbfe_mask.hip",
           "lbfe_adjoint.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, so a
    # device function compiles to the same rounding wherever it is inlined
    # (the fused and unfused step paths then agree bit for bit)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, extra=()):
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building liblbfe.so")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    build_c_example()
    return LIB


C_EXAMPLE_SRC = os.path.join(ROOT, "tests", "c_abi_droplet.c")
C_EXAMPLE = os.path.join(OUT_DIR, "c_abi_droplet")


def build_c_example():
    """The plain-C program of tests/c_abi_droplet.c against liblbfe.so and
    the HIP runtime (gcc, no HIP device code), next to the library."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), C_EXAMPLE_SRC, "-o", C_EXAMPLE, "-L", OUT_DIR, "-llbfe",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("gcc failed building the C ABI example")
    return C_EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
