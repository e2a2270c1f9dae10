"""Build libhp.so (all HIP kernels + the C ABI) for gfx950 with hipcc.

Objects go to ``_build/`` beside this file; the shared library is written
in-tree as ``libhp.so`` so that it travels with the source tree.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhp.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unknown-warning-option",
    # atomics here are issued by one lane with a wave-reduced value already
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


# host-side AddressSanitizer + UBSan for the checking build: every flag goes
# to the host pass only (the device code is built as usual)
SAN_FLAGS = [f for x in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                         "-fno-omit-frame-pointer", "-g") for f in ("-Xarch_host", x)]
SAN_OUT = os.path.join(HERE, "libhp_san.so")
SAN_BUILD = os.path.join(HERE, "_build_san")


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(force: bool = True, jobs: int = 8, sanitize: bool = False) -> str:
    """Compile every csrc/*.hip and link libhp.so.  Always recompiles when
    force is true (the default).  sanitize: the host code instrumented with
    AddressSanitizer and UBSan, as libhp_san.so (for host-only checks; the
    process must preload the compiler's ASan runtime, see asan_runtime)."""
    out, bdir = (SAN_OUT, SAN_BUILD) if sanitize else (OUT, BUILD)
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not force and os.path.exists(out):
        newest = max(os.path.getmtime(p) for p in glob.glob(os.path.join(CSRC, "*")))
        if os.path.getmtime(out) >= newest:
            return out
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SAN_FLAGS if sanitize else []), "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"link of {os.path.basename(out)} failed")
    os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """Path of the ASan runtime that libhp_san.so needs preloaded."""
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the compiler's ASan runtime was not found")
    return path


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
