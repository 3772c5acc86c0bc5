"""Compile the gfx950 library ``libpxd.so`` in-tree with hipcc.

Every source is compiled to its own object in parallel, then the objects are
linked.  Objects are kept under ``_build/`` keyed by a hash of the source, the
headers and the flags; ``force=True`` (what the package's build entry uses)
recompiles everything.

Usage: python -m paper_2412_17617_amd.build [-v] [--force]
"""

from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpxd.so")
OBJ_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("PXD_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-pthread",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    csrc = os.path.join(PKG, "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.cpp")) + glob.glob(os.path.join(csrc, "*.hip")))


def _headers():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h")))


def _key(src):
    h = hashlib.sha256()
    for f in [src] + _headers():
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIP_FLAGS).encode())
    return h.hexdigest()[:16]


def _clean(text):
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def _compile(src, force):
    obj = os.path.join(OBJ_DIR, f"{os.path.basename(src)}.{_key(src)}.o")
    if os.path.exists(obj) and not force:
        return obj, ""
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), "-c", src,
           "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({r.returncode}):\n{_clean(r.stdout + r.stderr)}")
    os.replace(obj + ".tmp", obj)
    return obj, _clean(r.stdout + r.stderr)


def build(verbose: bool = False, force: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, force), srcs))
    if verbose:
        for (obj, out) in results:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", *[o for o, _ in results], "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed ({r.returncode}):\n{_clean(r.stdout + r.stderr)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--force" in sys.argv))
