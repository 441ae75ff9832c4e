"""Builds the HIP library ``liblbm.so`` for gfx950 in-tree with hipcc.

Every source is compiled on each call (the caller decides when to build);
objects go to ``_build/`` beside this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblbm.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["kernels.hip", "lbm_api.cpp", "builder.cpp", "mlp.hip"]

# Packed-FP32 instructions are disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def device_asm(src: str = "kernels.hip") -> str:
    """gfx950 assembly of one source (device code only), with the build's
    flags; used to check register use and scratch of the kernels."""
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [HIPCC] + [f for f in FLAGS if f != "-fPIC"] + [
            "--cuda-device-only", "-S", "-x", "hip", os.path.join(CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc -S failed for {src}:\n{r.stderr}")
        return open(out).read()


def kernel_resources(asm: str) -> dict:
    """{kernel symbol: {"vgpr": n, "sgpr": n, "scratch": bytes}} from the
    .set directives of an assembly listing."""
    import re
    res = {}
    for name, key, val in re.findall(r"\.set (\S+)\.(num_vgpr|numbered_sgpr|private_seg_size), (\d+)", asm):
        k = {"num_vgpr": "vgpr", "numbered_sgpr": "sgpr", "private_seg_size": "scratch"}[key]
        res.setdefault(name, {})[k] = int(val)
    return res


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
