"""Builds liblbm.so (the HIP library behind include/lbm.h) in-tree for gfx950.

    python -m paper_2506_00907_amd.build [--force]

Every source is compiled with hipcc for gfx950 only; packed FP32 instructions
are disabled for the device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# -ffp-contract=on: multiply-adds fuse within one source expression only, so
# every kernel that inlines the same node or link update rounds it the same
# way (the default fuses across statements, depending on the surrounding code)
CFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-ffp-contract=on",
          f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(os.path.dirname(PKG), "include")]
SOURCES = ["lbm_host.cpp", "lbm_batch.cpp", "lbm_static.hip", "lbm_bandwidth.hip", "lbm_kernels_f64.hip", "lbm_kernels_f32.hip", "lbm_kernels_f16.hip",
           "lbm_kernels_bf16.hip", "nn_host.cpp", "nn_kernels.hip"]
HEADERS = ["lbm_device.hpp", "lbm_internal.hpp", "lbm_ctx.hpp", "nn_internal.hpp"]


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *[f"-D{d}" for d in defines], "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(force: bool = True, jobs: int = 8, out: str = LIB, defines=()) -> str:
    """Compiles every source and links `out` (the in-tree liblbm.so by
    default; another path with extra preprocessor definitions builds a
    variant, loaded through LBM_LIBRARY)."""
    build_dir = BUILD if out == LIB else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    deps.append(os.path.join(os.path.dirname(PKG), "include", "lbm.h"))
    if not force and os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(d) for d in deps):
        return out
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=LIB)
    ap.add_argument("--define", action="append", default=[])
    a = ap.parse_args()
    print(build(force=True, out=os.path.abspath(a.out), defines=a.define))
