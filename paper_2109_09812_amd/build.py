"""Builds libmeshrx.so (HIP, gfx950) in-tree.

    python -m paper_2109_09812_amd.build [--jobs N]

Every compilation unit is compiled with hipcc for gfx950; the sort kernels
are compiled once per record width (4..64 bytes) from one source.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmeshrx.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _units():
    units = []
    for k in range(1, 17):
        units.append((os.path.join(CSRC, "sort_inst.hip"), os.path.join(BUILD, f"sort_k{k}.o"),
                      [f"-DMRX_INST_K={k}"]))
    for name in ("meshrx", "gather"):
        units.append((os.path.join(CSRC, name + ".hip"), os.path.join(BUILD, name + ".o"), []))
    return units


def _compile(unit):
    src, obj, extra = unit
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    noise = "is not a recognized feature for this target"
    msgs = [l for l in (r.stderr or "").splitlines() if noise not in l and l.strip()]
    return obj, msgs


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    units = _units()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, units))
    if verbose:
        for obj, msgs in results:
            for m in msgs:
                print(f"[{os.path.basename(obj)}] {m}", file=sys.stderr)
    objs = [obj for obj, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    args = ap.parse_args()
    print(build(args.jobs, verbose=True))


if __name__ == "__main__":
    main()
