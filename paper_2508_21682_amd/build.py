"""Build libhf.so (hand-written HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhf.so")
PEAKS_SRC = os.path.join(HERE, "peaks", "peaks.hip")
PEAKS = os.path.join(HERE, "peaks", "hf_peaks")
ARCH = os.environ.get("HF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no v_pk_*_f32 generated from ordinary float code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    if src is None:
        return build_peaks()
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    subprocess.check_call([HIPCC] + FLAGS + ["-c", src, "-o", obj])
    return obj


def build_peaks() -> str:
    """The standalone ceiling probes (copy, random gathers, fp16 MFMA) that
    `bench.py --peaks` runs; not part of libhf."""
    tmp = PEAKS + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC] + [f for f in FLAGS if f != "-fPIC"] + [PEAKS_SRC, "-o", tmp])
    os.replace(tmp, PEAKS)
    return PEAKS


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, sources() + [None]))[:-1]
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
