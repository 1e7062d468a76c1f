"""Host-sanitizer build of the library, for the CPU tests only.

    python -m paper_2110_01409_amd.build_sanitized

The host translation units (C ABI, layout builder, sets, server) are compiled
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and linked
with the kernel objects of the ordinary build (``build.build()`` must have run:
they are taken from ``_build/`` unchanged, device code is not instrumented)
into ``_build_san/libdg_san.so``.  A process loads it with the sanitizer
runtime preloaded (``preload()``) and ``DG_LIBRARY`` pointing at it; without a
GPU only the validation and layout paths run, which is what the ABI and
layout tests exercise.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from . import build as _build

HOST_SOURCES = ["dg_api.cpp", "dg_plan.cpp", "dg_set.cpp", "dg_server.cpp"]
OUTDIR = os.path.join(_build.PKG, "_build_san")
LIB = os.path.join(OUTDIR, "libdg_san.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]


def kernel_objects() -> list[str]:
    objdir = os.path.join(_build.PKG, "_build")
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in _build.SOURCES if s.endswith(".hip")]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"kernel objects missing ({', '.join(missing)}): run the ordinary build first")
    return objs


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"g++ failed with status {res.returncode}: {' '.join(cmd)}")


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(_build.CSRC, f) for f in os.listdir(_build.CSRC)] + kernel_objects()
    deps.append(os.path.join(_build.INCLUDE, "dg.h"))
    return any(os.path.getmtime(p) > t for p in deps)


def build() -> str:
    """Compiles the host sources with the sanitizers and links the library
    (only when a source or kernel object is newer than it)."""
    kobjs = kernel_objects()
    if not stale():
        return LIB
    os.makedirs(OUTDIR, exist_ok=True)
    objs = [os.path.join(OUTDIR, os.path.splitext(s)[0] + ".o") for s in HOST_SOURCES]
    cmds = [["g++", "-std=c++17", "-O1", "-g", "-fPIC", *SAN, "-D__HIP_PLATFORM_AMD__",
             "-I", os.path.join(ROCM, "include"), "-I", _build.INCLUDE, "-I", _build.CSRC,
             "-c", os.path.join(_build.CSRC, s), "-o", o] for s, o in zip(HOST_SOURCES, objs)]
    with ThreadPoolExecutor(min(len(cmds), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", *SAN, *objs, *kobjs, "-L", os.path.join(ROCM, "lib"),
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def preload() -> str:
    """The AddressSanitizer runtime g++ links against (to be preloaded)."""
    return subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


def env() -> dict:
    """Environment of a process that runs the library under the sanitizers."""
    e = dict(os.environ)
    e["DG_LIBRARY"] = LIB
    e["LD_PRELOAD"] = preload()
    e["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    e["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return e


if __name__ == "__main__":
    print(build())
