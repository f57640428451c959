"""Build the HIP library (liblbm.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_kernels.hip", "lbm_et.hip", "lbm_sparse.hip", "lbm_closure.hip", "lbm_refine.hip", "lbm_features.hip", "lbm_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str) -> str:
    obj = os.path.join(CSRC, "_obj", os.path.splitext(src)[0] + ".o")
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build() -> str:
    """Compile every source (always) and link liblbm.so; returns its path."""
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    _build_example()
    return LIB


EXAMPLE_SRC = os.path.join(HERE, "examples", "abi_tgv.cpp")
EXAMPLE_BIN = os.path.join(HERE, "examples", "abi_tgv")


def _build_example():
    """The C ABI driven from plain host code (examples/abi_tgv.cpp), linked
    against the library next to it."""
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", EXAMPLE_SRC, "-o", EXAMPLE_BIN + ".tmp",
           "-L" + HERE, "-llbm", "-Wl,-rpath,$ORIGIN/.."]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stderr}")
    os.replace(EXAMPLE_BIN + ".tmp", EXAMPLE_BIN)


if __name__ == "__main__":
    print(build())
