"""Build of the HIP library libcmlbm.so for gfx950 (in-tree, next to this file).

Run ``python -m paper_1202_6081_amd.build``.  Every call compiles from source.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcmlbm.so")

SOURCES = ["api.cpp", "kernels.hip", "checks.hip"]
# -packed-fp32-ops: no v_pk_* FP32 instructions are generated.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libcmlbm.so")
    os.replace(tmp, LIB)
    return LIB


C_TEST_SRC = os.path.join(ROOT, "tests", "c", "abi_from_c.c")
C_TEST_BIN = os.path.join(ROOT, "tests", "c", "abi_from_c")


def build_c_test(verbose=False):
    """The C program that drives the library's C ABI from C alone (a GPU test
    runs it): plain C11 against include/cmlbm.h and the HIP runtime, linked to
    the in-tree libcmlbm.so."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler found for the C ABI test program")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    tmp = C_TEST_BIN + ".tmp"
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), C_TEST_SRC,
           "-L", HERE, "-lcmlbm", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1202_6081_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building the C ABI test program failed")
    os.replace(tmp, C_TEST_BIN)
    return C_TEST_BIN


PROBE_SRC = os.path.join(CSRC, "hbm_probe.hip")
PROBE_BIN = os.path.join(HERE, "hbm_probe")


def build_probe(verbose=False):
    """The HBM rate probe (a standalone HIP program, no part of the library):
    plain read, write and copy streams and the step's memory traffic without
    its arithmetic, the ceilings the step's roofline fraction is read against."""
    tmp = PROBE_BIN + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building hbm_probe")
    os.replace(tmp, PROBE_BIN)
    return PROBE_BIN


HOST_DIR = os.path.join(ROOT, "tests", "host")
HOST_SRC = os.path.join(HOST_DIR, "host_collide.cpp")
HOST_LIB = os.path.join(HOST_DIR, "libhostmath.so")
HOST_SAN_SRC = os.path.join(HOST_DIR, "sanitize_main.cpp")
HOST_SAN_BIN = os.path.join(HOST_DIR, "host_sanitize")
HOST_FLAGS = ["-std=c++17", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-Wno-unused-parameter", "-I", CSRC]


def _cxx():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        raise RuntimeError("no C++ compiler found for the host build of the device math")
    return cxx


def build_host_math(verbose=False):
    """The library's per-node device math (collision, adjoint, initial state)
    compiled for the CPU as a shared library for the CPU tests
    (tests/host/host_collide.cpp includes the same headers the kernels use)."""
    tmp = HOST_LIB + ".tmp"
    cmd = [_cxx(), *HOST_FLAGS, "-O2", "-fPIC", "-shared", HOST_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building the host device math failed")
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def build_host_sanitized(verbose=False):
    """The same host code as an executable with AddressSanitizer and
    UndefinedBehaviorSanitizer, driven by tests/host/sanitize_main.cpp (CPU only)."""
    tmp = HOST_SAN_BIN + ".tmp"
    cmd = [_cxx(), *HOST_FLAGS, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           HOST_SRC, HOST_SAN_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building the sanitized host device math failed")
    os.replace(tmp, HOST_SAN_BIN)
    return HOST_SAN_BIN


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_host_math(verbose=True))
    print(build_c_test(verbose=True))
    print(build_probe(verbose=True))
