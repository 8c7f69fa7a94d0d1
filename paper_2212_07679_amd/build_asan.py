"""Build a copy of libsnn.so whose host code is instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged), for
the CPU-side ABI tests: ``_build_asan/libsnn_asan.so`` at the repository
root.  The library needs the sanitizer runtime loaded first (LD_PRELOAD of
``asan_runtime()``); nothing in the product path loads it.
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

from paper_2212_07679_amd import build_lib as bl

OUT = os.path.join(bl.ROOT, "_build_asan")
LIB = os.path.join(OUT, "libsnn_asan.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/llvm")
    return found[-1]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [bl.hipcc(), *bl.common_flags(), *bl.FILE_FLAGS.get(os.path.basename(src), []), *HOST_SAN, "-c", src,
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = bl.sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [bl.hipcc(), f"--offload-arch={bl.ARCH}", "-shared", "-fPIC", *HOST_SAN, "-shared-libsan", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print("built", build())
