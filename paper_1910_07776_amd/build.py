"""Builds libsugg.so (all HIP sources under csrc/) for gfx950 with hipcc.

    python -m paper_1910_07776_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libsugg.so")
OBJDIR = os.path.join(ROOT, "_build", "obj")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(src), _headers_mtime()):
        return obj
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


VERSIONS_SRC = os.path.join(PKG, "profiling", "versions.hip")
VERSIONS_BIN = os.path.join(LIBDIR, "sugg_versions")


def _build_versions() -> str:
    """The profiled-versions program (real Tier 1 data), an executable."""
    tmp = VERSIONS_BIN + ".tmp"
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-fPIC", "-fvisibility=hidden")], VERSIONS_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {VERSIONS_SRC}:\n{r.stderr}")
    os.replace(tmp, VERSIONS_BIN)
    return VERSIONS_BIN


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link the shared library (and the profiled-
    versions program); returns the library's path.  incremental: recompile
    only sources older than their object (or than any header)."""
    os.makedirs(OBJDIR, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(min(int(os.environ.get("MAX_JOBS", "8")), len(srcs) + 1)) as ex:
        vfut = ex.submit(_build_versions) if not (incremental and os.path.exists(VERSIONS_BIN)) else None
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
        if vfut:
            vfut.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
