"""Build step of the HIP library: compiles csrc/*.hip into librcp.so (gfx950).

Flags that matter for the results: -ffp-contract=off (no fused multiply-add
anywhere, so FP32 results follow the written operation order), the default
correctly rounded FP32 division and square root, and packed-FP32 ops disabled.

build_sanitized() makes a second copy of the library whose host code is built
with the address and undefined-behaviour sanitizers (the device code is the
same as in librcp.so), plus the driver tests/sanitize_host_check.cpp linked
against it, both under _asan/.  Nothing in the product loads that copy.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librcp.so")
ASAN_DIR = os.path.join(PKG, "_asan")
ASAN_LIB = os.path.join(ASAN_DIR, "librcp_asan.so")
ASAN_CHECK = os.path.join(ASAN_DIR, "sanitize_host_check")
ASAN_DRIVER = os.path.join(ROOT, "tests", "sanitize_host_check.cpp")
ARCH = os.environ.get("RCP_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# host side only: each -fsanitize= goes right after -Xarch_host
SANITIZE_FLAGS = ["-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def build_sanitized(out_dir: str = ASAN_DIR, verbose: bool = False) -> tuple[str, str]:
    """Compile the library with host-side sanitizers (one process per source
    file) and the host-code driver; returns (library, driver) paths."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, os.path.basename(ASAN_LIB))
    exe = os.path.join(out_dir, os.path.basename(ASAN_CHECK))
    with tempfile.TemporaryDirectory(dir=out_dir) as tmp:
        compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"] + SANITIZE_FLAGS

        def one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [hipcc, *compile_flags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", "-o", obj, src]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode:
                raise RuntimeError(f"{' '.join(cmd)}\n{r.stderr}")
            return obj

        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(one, sources()))
        link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE_FLAGS, "-o", lib + ".tmp", *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(lib + ".tmp", lib)
    drv = [hipcc, f"--offload-arch={ARCH}", "-O1", "-std=c++17", *SANITIZE_FLAGS, f"-I{INCLUDE}",
           "-o", exe + ".tmp", ASAN_DRIVER, f"-L{out_dir}", "-lrcp_asan", "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(drv), flush=True)
    subprocess.check_call(drv)
    os.replace(exe + ".tmp", exe)
    return lib, exe


if __name__ == "__main__":
    print(build(verbose=True))
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose=True))
    sys.exit(0)
