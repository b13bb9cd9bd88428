"""Build the native libraries in-tree (gfx950 only).

libwh.so         the C-ABI library (include/wh.h): HIP kernels + host runtime
libwhsynth.so    host input generator (gcc)
libwhsynth_dev.so  device input generator (hipcc)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwh.so")

ARCH = "gfx950"
HIP_SOURCES = ["whz_dispatch.hip", "dense_kernels.hip", "serve.hip", "host_stream.hip", "thermal.hip", "whz_var.hip", "wh_api.hip", "noalloc.hip"]
# words per compressed block (rate = 2 * words) with a compiled decoder
WHZ_WORDS = [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16]
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-ffp-contract=fast",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra=(), tag: str = "") -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + tag + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj


def build_libwh(verbose: bool = False) -> str:
    jobs = [(src, (), "") for src in HIP_SOURCES]
    jobs += [("whz_kernels.hip", (f"-DWH_NW={k}",), f"_nw{k}") for k in WHZ_WORDS]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_all(verbose: bool = False) -> None:
    from . import synth
    synth.build_host()
    synth.build_device(hipcc())
    build_libwh(verbose)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_1902_08018_amd import build as b
    b.build_all(verbose=True)
