"""Builds libcuboid.so (HIP for gfx950) next to this file.

usage: python -m paper_1601_00636_amd.build   (or build() from Python)
       python -m paper_1601_00636_amd.build --host-sanitize
           also builds _build_san/libcuboid.so, whose host C++ runs under
           AddressSanitizer and UBSan (device code as usual); load it with
           CUBOID_LIB=<that path> and gcc's libasan and libubsan in LD_PRELOAD
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcuboid.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = [
    "kernels_tables.hip",
    "kernels_sieve.hip",
    "kernels_roots.hip",
    "kernels_peaks.hip",
    "noalloc.hip",
    "bigint.cpp",
    "graph.cpp",
    "region.cpp",
    "search.cpp",
    "tables_io.cpp",
    "context.cpp",
    "autotune.cpp",
    "server.cpp",
    "api.cpp",
]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", ROCM + "/bin/hipcc")
CXX = os.environ.get("CXX", "g++")
ARCH = "gfx950"
# packed FP32 instructions stay off (no float arithmetic on the hot path anyway)
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + INCLUDE, "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# host C++ instrumentation of the sanitized build (gcc's runtimes)
SANITIZE = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
SAN_DIR = os.path.join(HERE, "_build_san")


def _compile(src, build_dir=BUILD_DIR, sanitize=False):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC] + DEVICE + COMMON + ["-x", "hip", "-c", path, "-o", obj]
    else:
        # host-only C++ (HIP runtime API through its headers)
        extra = SANITIZE if sanitize else []
        cmd = [CXX] + COMMON + extra + ["-D__HIP_PLATFORM_AMD__", "-I" + ROCM + "/include",
                                        "-pthread", "-c", path, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return obj


def build(verbose=False):
    """Compile every HIP/C++ source for gfx950 and link libcuboid.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stdout))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(verbose=False):
    """libcuboid.so with AddressSanitizer and UBSan in its host C++, in _build_san/."""
    os.makedirs(SAN_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda f: _compile(f, SAN_DIR, True), SOURCES))
    runtimes = [subprocess.run([CXX, "-print-file-name=" + n], stdout=subprocess.PIPE,
                               text=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    lib = os.path.join(SAN_DIR, "libcuboid.so")
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", lib] + objs + runtimes + \
        ["-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stdout))
    if verbose:
        print("built", lib, "(preload:", " ".join(runtimes) + ")")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    if "--host-sanitize" in sys.argv[1:]:
        build_host_sanitized(verbose=True)
    sys.exit(0)
