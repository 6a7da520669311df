"""Build the HIP library in-tree for gfx950 (hipcc; no JIT cache).

    python -m paper_2406_05577_amd.build

Every translation unit is compiled to an object in parallel (the register-path
kernel instantiations are split over several units), then linked into
libfftb.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfftb.so")
OBJ_DIR = os.path.join(PKG, "_build")

# Packed FP32 instructions are disabled for all device code; the host pass
# warns that it does not know the feature, which is harmless.
HIP_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
    return [os.path.join(CSRC, f) for f in names]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _filter(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def _compile(src: str) -> str:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIP_FLAGS + ["-c", src, "-o", obj + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({res.returncode}):\n"
                           f"{_filter(res.stdout + res.stderr)}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [hipcc()] + HIP_FLAGS + ["-shared"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed ({res.returncode}):\n{_filter(res.stdout + res.stderr)}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
