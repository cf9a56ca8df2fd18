"""Builds the native libraries in-tree.

librel.so   - the HIP kernels and the C-ABI of include/rel.h, compiled for
              gfx950 with hipcc (cross-compiles without a GPU).
libreldatagen.so - the seeded input generators (host C, OpenMP).
"""

from __future__ import annotations

import concurrent.futures
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIB_PATH = os.path.join(PKG, "librel.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["api.cpp", "autotune.cpp", "profile.cpp", "server.cpp", "filter.hip", "join.hip", "groupby.hip", "partition.hip",
           "pipeline.hip",
           "pipeline_batch.hip", "records.hip", "stream.hip", "bloom.hip", "late.hip", "strings.hip"]

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # packed fp32 instructions stay off (none of this code needs them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


# The fused pipeline kernels are instantiated per first-dim access mode in
# separate objects (see pipeline.hip, pipeline_batch.hip) so that the variants
# compile in parallel.
UNITS = [(s, s.replace(".hip", "").replace(".cpp", ""), []) for s in SOURCES] + [
    ("pipeline.hip", f"pipeline_d{m}", [f"-DREL_PIPE_D0={m}"]) for m in range(1, 7)] + [
    ("pipeline_batch.hip", f"pipeline_batch_d{m}", [f"-DREL_BATCH_D0={m}"]) for m in (0, 1, 3, 5)]


def _compile(unit) -> str:
    src, name, defs = unit
    obj = os.path.join(BUILD_DIR, name + ".o")
    cmd = [HIPCC, "-x", "hip", *HIP_FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_rel(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = min(len(UNITS), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


def build_all(verbose: bool = False) -> None:
    from . import datagen
    build_rel(verbose)
    datagen.build()
