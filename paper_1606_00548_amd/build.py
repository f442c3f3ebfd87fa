"""Build the HIP library libcprmi.so in-tree for gfx950.

Every .hip file under csrc/ is compiled to an object (in parallel) and the
objects are linked into paper_1606_00548_amd/libcprmi.so.  Run as a module
(`python -m paper_1606_00548_amd.build`) or call build().
"""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcprmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"),
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result"]
# roctx ranges around the entry points (seen by rocprofv3 --marker-trace)
ROCTX = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
# The host-sanitized build (build_sanitized): AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only (each flag given to the
# host compilation alone; the GPU code is built as in the product), for the
# C-ABI driver under tests/host_sanitizers.
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
OUT_SAN = os.path.join(PKG, "_build_san")
LIB_SAN = os.path.join(PKG, "libcprmi_san.so")
DRIVER_SRC = os.path.join(ROOT, "tests", "host_sanitizers", "capi_driver.cpp")
DRIVER = os.path.join(ROOT, "tests", "host_sanitizers", "capi_driver")
# assembly evaluates each face flow from both cells: keep their rounding identical
PER_FILE = {"assemble.hip": ["-ffp-contract=off"]}


def _compile(src, out=OUT, extra=()):
    obj = os.path.join(out, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC] + COMMON + PER_FILE.get(os.path.basename(src), []) + list(extra) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{p.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ROCTX
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized(verbose=False):
    """libcprmi_san.so (host code under ASan + UBSan) and the C-ABI driver
    linked against it."""
    os.makedirs(OUT_SAN, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, OUT_SAN, HOST_SAN), srcs))
    steps = [
        [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + HOST_SAN + ["-o", LIB_SAN + ".tmp"] + objs + ROCTX,
        [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include")] + HOST_SAN +
        [DRIVER_SRC, "-o", DRIVER + ".tmp", "-L", PKG, "-lcprmi_san", "-Wl,-rpath," + PKG] + ROCTX,
    ]
    for cmd in steps:
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"sanitized build failed:\n{p.stderr}")
        if cmd is steps[0]:
            os.replace(LIB_SAN + ".tmp", LIB_SAN)
    os.replace(DRIVER + ".tmp", DRIVER)
    if verbose:
        print("built", LIB_SAN, "and", DRIVER)
    return DRIVER


if __name__ == "__main__":
    build(verbose=True)
    if "--sanitized" in sys.argv:
        build_sanitized(verbose=True)
    sys.exit(0)
