"""Build liboversketch.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1811_02653_amd.build

Every HIP source is compiled for gfx950 with packed-FP32 instruction
selection disabled and linked into paper_1811_02653_amd/liboversketch.so.
The measured-ceiling kernels the benchmark times beside it (csrc/ceilings.hip)
go into a separate paper_1811_02653_amd/libosk_ceilings.so.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liboversketch.so")
CEIL_OUT = os.path.join(HERE, "libosk_ceilings.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["hash.hip", "sketch.hip", "gemm.hip", "quant.hip", "api.hip", "gram.hip", "noalloc.hip"]
CEIL_SOURCES = ["ceilings.hip"]
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the compiler from forming packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(SRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), res.stderr))
    return obj


def _link(objs, out):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + CEIL_SOURCES
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], OUT)
    _link([objs[s] for s in CEIL_SOURCES], CEIL_OUT)
    if verbose:
        print("built", OUT, "and", CEIL_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
