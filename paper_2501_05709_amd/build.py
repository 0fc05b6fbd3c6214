"""Build libfr.so (HIP kernels for gfx950 + host library + C ABI) in-tree.

    python -m paper_2501_05709_amd.build [--verbose]

Every source is compiled by hipcc for gfx950 only.  Packed FP32 VALU
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfr.so")
# (source, object stem, extra defines): the FR kernel file is compiled in five parts, its
# launchers of one precision and dimension each plus the dispatch, built in parallel
KERNEL_PARTS = 5
SOURCES = ([("fr_kernels.hip", f"fr_kernels_part{k}", [f"-DFR_PART={k}"]) for k in range(KERNEL_PARTS)]
           + [(s, s, []) for s in ("fr_host.cpp", "fr_pool.cpp", "fr_fwh.hip")])
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    # code object v5 loads in both the system HIP runtime and the one bundled with torch
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
            "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


_RESOURCE_KEYS = {"VGPRs": "vgpr", "AGPRs": "agpr", "SGPRs Spill": "sgpr_spill", "VGPRs Spill": "vgpr_spill",
                  "ScratchSize [bytes/lane]": "scratch", "Occupancy [waves/SIMD]": "occupancy",
                  "LDS Size [bytes/block]": "lds"}


def parse_resource_usage(text):
    """Per-kernel resource usage from the compiler's kernel-resource-usage remarks:
    {mangled name: {vgpr, agpr, sgpr_spill, vgpr_spill, scratch, occupancy, lds}}."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z /\[\]]+?):\s+(-?\d+)\s", line + " ")
        if cur is not None and m and m.group(1).strip() in _RESOURCE_KEYS:
            cur[_RESOURCE_KEYS[m.group(1).strip()]] = int(m.group(2))
    return out


def _compile(job, verbose):
    src, stem, defines = job
    os.makedirs(OBJ, exist_ok=True)
    out = os.path.join(OBJ, stem + ".o")
    device = src.endswith(".hip")
    lang = ["-x", "hip"] if device else []
    # device sources also report each kernel's registers, spills, occupancy and LDS
    remarks = ["-Rpass-analysis=kernel-resource-usage"] if device else []
    cmd = [hipcc()] + common_flags() + defines + lang + remarks + ["-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if device:
        with open(os.path.join(OBJ, stem + ".resources.json"), "w") as f:
            json.dump(parse_resource_usage(r.stderr), f, indent=0, sort_keys=True)
    warnings = "\n".join(l for l in r.stderr.splitlines() if "warning:" in l)
    if verbose and warnings:
        print(warnings, flush=True)
    return out


def build(verbose=False):
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    # one resource report for the kernel file: the union of its parts
    merged = {}
    for k in range(KERNEL_PARTS):
        with open(os.path.join(OBJ, f"fr_kernels_part{k}.resources.json")) as f:
            merged.update(json.load(f))
    with open(os.path.join(OBJ, "fr_kernels.hip.resources.json"), "w") as f:
        json.dump(merged, f, indent=0, sort_keys=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
    print(LIB)
