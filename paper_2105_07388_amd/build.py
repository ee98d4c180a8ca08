"""Compile the HIP library librankest.so for gfx950 (in-tree).

Every translation unit under csrc/ is compiled by hipcc for gfx950 only, with
packed-FP32 instruction selection disabled, and linked into one shared object
next to this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librankest.so")
ARCH = os.environ.get("RANKEST_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


# Host-code sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer on
# the host side only; the GPU code is compiled as usual) linked with the C
# driver tests/host_sanitizer_driver.cpp into one executable.
SAN_BUILD = os.path.join(BUILD, "hostsan")
SAN_BIN = os.path.join(HERE, "_hostsan", "host_sanitizer_driver")
SAN_DRIVER = os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
SAN_HOST_FLAGS = ["-fno-gpu-sanitize", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]


def _compile_san(src, verbose):
    obj = os.path.join(SAN_BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *SAN_FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build_host_sanitized(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every csrc/ unit with the host-side sanitizers and link the
    driver; returns the executable's path."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    os.makedirs(os.path.dirname(SAN_BIN), exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile_san(s, verbose), sources()))
    drv = os.path.join(SAN_BUILD, "driver.o")
    cmd = ["hipcc", *SAN_HOST_FLAGS, "-std=c++17", "-I", INCLUDE, "-c", SAN_DRIVER, "-o", drv]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp = SAN_BIN + ".tmp"
    cmd = ["hipcc", *SAN_HOST_FLAGS, f"--offload-arch={ARCH}", "-o", tmp, drv, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_BIN)
    return SAN_BIN


if __name__ == "__main__":
    print(build(verbose=True))
