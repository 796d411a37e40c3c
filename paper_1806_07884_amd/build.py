"""Builds librbf.so (HIP kernels + C-ABI) for gfx950 in-tree, and its
checked variant librbf_checked.so.

    python -m paper_1806_07884_amd.build [--no-checked]

The checked variant compiles the sources that hold device index checks
(checks.h) with RBF_CHECKED: every checked index that falls outside its
buffer skips its access and is reported by the entry point as RBF_ERR_HIP
with the check's file and line.  The other objects are shared with the normal
build.  Objects go to ``_build/`` (``_build/checked/``) at the repository
root; the shared libraries land next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "librbf.so")
OUT_CHECKED = os.path.join(PKG, "librbf_checked.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

SOURCES = ["sort_scan.hip", "plan_kernels.hip", "assemble_kernels.hip", "cg_kernels.hip",
           "eval_kernels.hip", "mlp_kernels.hip", "poly_kernels.hip", "halo_kernels.hip",
           "stream_kernels.hip", "lsqr_kernels.hip", "tile_kernels.hip",
           "api.hip"]
# sources whose objects differ in the checked build
CHECKED_SOURCES = ["plan_kernels.hip", "assemble_kernels.hip", "eval_kernels.hip",
                   "tile_kernels.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
          # keep the compiler from emitting packed FP32 arithmetic
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(job: tuple[str, bool]) -> str:
    src, checked = job
    out_dir = os.path.join(BUILD_DIR, "checked") if checked else BUILD_DIR
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    flags = CFLAGS + (["-DRBF_CHECKED"] if checked else [])
    cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}{' (checked)' if checked else ''}:\n"
                           f"{res.stderr}")
    return obj


def _link(objs: list[str], out: str) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed for {os.path.basename(out)}:\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, checked: bool = True) -> str:
    """Compiles and links librbf.so (and, with checked, librbf_checked.so);
    returns the path of librbf.so."""
    os.makedirs(os.path.join(BUILD_DIR, "checked"), exist_ok=True)
    jobs = [(s, False) for s in SOURCES]
    if checked:
        jobs += [(s, True) for s in CHECKED_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = dict(zip(jobs, ex.map(_compile, jobs)))
    _link([objs[(s, False)] for s in SOURCES], OUT)
    if verbose:
        print(f"built {OUT}")
    if checked:
        _link([objs[(s, s in CHECKED_SOURCES)] for s in SOURCES], OUT_CHECKED)
        if verbose:
            print(f"built {OUT_CHECKED}")
    return OUT


if __name__ == "__main__":
    build(verbose=True, checked="--no-checked" not in sys.argv[1:])
    sys.exit(0)
