"""Build libmoa.so (HIP, gfx950) in-tree.

    python -m paper_0907_0792_amd.build      # or python paper_0907_0792_amd/build.py
    python -m paper_0907_0792_amd.build --changed   # only units older than their sources

Each ``csrc/*.hip`` file is compiled to an object with hipcc for gfx950 (in
parallel), then linked into ``paper_0907_0792_amd/libmoa.so``. Packed FP32 VALU
instructions are disabled for every kernel.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmoa.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++20", "-Wall", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str, verbose: bool, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    if not force and os.path.exists(obj):
        # Up to date when newer than the source and every shared header.
        deps = [src] + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(INCLUDE, "*.h"))
        if os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
            return obj
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noise and verbose:
        print("\n".join(noise), flush=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None, force: bool = True) -> str:
    """Compile every unit (force) or only those older than their sources
    (force=False), then link."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # --no-undefined: a template instantiated in no unit fails here, not at load.
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    return LIB


# Units with host logic (argument validation, shape algebra, the tile-table
# parser, batch building, the static scratch lookup).
HOST_UNITS = ("moa_abi.hip", "k_batch.hip", "split_static.hip")


def build_host_sanitized(out: str, verbose: bool = False) -> str:
    """A copy of the library whose host code is built with AddressSanitizer
    and UndefinedBehaviorSanitizer (device code as usual), for CPU tests of
    the host logic. The other units' objects come from the regular build;
    the process that loads it must preload clang's ASan runtime."""
    objs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        name = os.path.basename(src)
        obj = os.path.join(BUILD, name.replace(".hip", ".o"))
        if name in HOST_UNITS:
            obj = out + "." + name.replace(".hip", ".o")
            cmd = [HIPCC] + CFLAGS + ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                      "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host",
                                      "-fno-omit-frame-pointer", "-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
        elif not os.path.exists(obj):
            raise FileNotFoundError("%s is not built: run the regular build first" % obj)
        objs.append(obj)
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", out] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, force="--changed" not in sys.argv)
    print("built", LIB)
