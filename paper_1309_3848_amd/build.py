"""Build libseeds.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libseeds.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# roctx ranges (a profiler's marker trace); the library sits with the ROCm
# runtime libraries
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return any(os.path.getmtime(p) > t for p in deps)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, *sources(), "-o", tmp, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libseeds.so")
    os.replace(tmp, LIB)
    return LIB


# The host-side sanitizer driver (tests/host_sanitizer_driver.cpp): every
# library source compiled together with it into one program whose host code
# carries AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# built as for the library), so the sanitizer runtime is linked in and nothing
# is preloaded.
SAN_DRIVER = os.path.join(PKG, "seeds_host_sanitized")
SAN_SRC = os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp")
SAN_FLAGS = ("-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=all "
             "-Xarch_host -fno-omit-frame-pointer").split()


def build_sanitized_driver(verbose: bool = False) -> str:
    flags = [f for f in FLAGS if f not in ("-shared", "-fPIC", "-O3")]
    tmp = SAN_DRIVER + ".tmp"
    cmd = [HIPCC, *flags, "-O1", "-g", *SAN_FLAGS, "-I", INCLUDE, "-I", CSRC, SAN_SRC,
           *sources(), "-o", tmp, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the host sanitizer driver")
    os.replace(tmp, SAN_DRIVER)
    return SAN_DRIVER


if __name__ == "__main__":
    print(build(force=True, verbose=True))
    print(build_sanitized_driver(verbose=True))
