"""Build the HIP library (gfx950) in-tree: paper_2006_16935_amd/libitse.so."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libitse.so")
SOURCES = ["itse_f32.hip", "itse_f64.hip", "itse_runtime.hip", "itse_batch.hip", "itse_server.hip",
           "itse_persist.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # a * b + c is fused where one expression writes it and nowhere else: the
         # rounding of every kernel is fixed by its source, not by what the optimiser
         # sees around it, so a pass's tile gives the same bits in its own kernel and
         # inlined in the persistent batch kernel
         "-ffp-contract=on",
         "-Wno-unused-result"]
# The persistent batch kernel runs every pass's tiles in one loop: machine-level
# hoisting of loop-invariant values out of that loop would keep them live across
# all tiles (and cost occupancy), so it is off for that file.
SOURCE_FLAGS = {"itse_persist.hip": ["-mllvm", "-disable-machine-licm"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
