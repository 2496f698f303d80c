"""Host-only build of libqmc.so with AddressSanitizer and
UndefinedBehaviorSanitizer, for CPU tests of the library's host code:
argument validation, parameter packing, the generators of specialised
kernel source, the lattice-construction helpers and the status paths.

Only the hand-written units are compiled (their device code at -O1, the
host code instrumented); the generated kernel instantiations are left out,
so the kernel registry is empty and every launch path reports that no
kernel exists.  Any sanitizer finding aborts.  The library is loaded by setting
QMC_LIB to its path and preloading clang's shared sanitizer runtime
(runtime_path()).

    python -m paper_1811_11722_amd.build_sanitized OUT.so
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

from .build import ARCH, BUILD, CSRC, HIPCC, INCLUDE, _write_jit_headers

CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
       "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-Wno-unused-value", "-Wno-unused-result",
         f"-I{INCLUDE}", f"-I{CSRC}", f"-I{os.path.join(BUILD, 'gen')}"]


def runtime_path() -> str:
    out = subprocess.run([CLANG, "-print-runtime-dir"], capture_output=True, text=True, check=True).stdout.strip()
    for d in (out, os.path.join(os.path.dirname(out), "linux")):
        p = os.path.join(d, "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
        p = os.path.join(d, "libclang_rt.asan.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("clang's shared AddressSanitizer runtime")


def build(out: str, jobs: int = 0) -> str:
    os.makedirs(os.path.join(BUILD, "gen"), exist_ok=True)
    _write_jit_headers()
    objdir = os.path.join(os.path.dirname(os.path.abspath(out)), "san_obj")
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src)[:-4] + ".o")
        res = subprocess.run([HIPCC, *FLAGS, *SAN, "-c", src, "-o", obj], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"host-only compile failed for {src}:\n{res.stderr[-4000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    link = [CLANG, "-shared", "-fsanitize=address,undefined", "-shared-libsan", "-o", out, *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    return out


if __name__ == "__main__":
    print(build(sys.argv[1]))
