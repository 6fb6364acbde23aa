"""Build libmffv with AddressSanitizer on its host code only (the argument
checks and plan bookkeeping of the C ABI run on the CPU), for the CPU tests.

The device code is compiled as for the product library; only the host
compilation and the final (host) link use the sanitizer. The library goes to
``_build/asan/libmffv_asan.so`` and is rebuilt when a source is newer.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "_build", "asan")
LIB = os.path.join(OUT, "libmffv_asan.so")
# host-only sanitizer flags: each one bound to the host compilation
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str | None:
    """The shared AddressSanitizer runtime of the ROCm clang (to preload)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build() -> str:
    from paper_2408_03452_amd import build as b
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(b.CSRC, f) for f in b.SOURCES]
    deps = srcs + glob.glob(os.path.join(b.CSRC, "*.hpp")) + [os.path.join(b.INCLUDE, "mffv.h")]
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    procs, objs = [], []
    for src in srcs:
        name = os.path.splitext(os.path.basename(src))[0]
        obj = os.path.join(OUT, name + ".o")
        cmd = [b.hipcc(), *b.COMMON, *b.DEVICE_FLAGS, *b.SOURCE_FLAGS.get(os.path.basename(src), []),
               *HOST_ASAN, "-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"hipcc (host ASan) failed on {src}:\n{out}")
    clang = "/opt/rocm/llvm/bin/clang++"
    link = [clang, "-shared", "-fsanitize=address", "-shared-libasan", "-o", LIB, *objs,
            "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"host ASan link failed:\n{res.stdout}{res.stderr}")
    return LIB


if __name__ == "__main__":
    print(build())
