"""Build libdia.so for gfx950 with hipcc (in-tree, next to this file).

Usage: python -m paper_2104_13715_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdia.so")
SOURCES = ["tile_dispatch.cpp", "fit_kernels.hip", "newton_kernels.hip", "bf16x3_kernels.hip", "dia_api.cpp",
           "batched_api.cpp", "newton_host.cpp", "noalloc_api.cpp"]
KERNEL_SIZES = list(range(1, 50, 2))  # one translation unit of tiled kernels per odd kernel size

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("DIA_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 (v_pk_*_f32) is switched off for every device pass
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def _compile(job) -> str:
    src, defines, name = job
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [HIPCC, *FLAGS, *defines, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


# Host-code sanitizers for the CPU checks of the C ABI (argument validation, layouts, autotuner):
# every flag goes to the host pass only; the device code is that of the normal build.
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libdia_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile_san(job) -> str:
    src, defines, name = job
    obj = os.path.join(SAN_DIR, name + ".o")
    cmd = [HIPCC, *FLAGS, *SAN_FLAGS, *defines, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc (sanitized host pass) failed on {src}")
    return obj


def build_sanitized(jobs: int = 8) -> str:
    """libdia_san.so: the C-ABI sources with AddressSanitizer and UndefinedBehaviorSanitizer on their host
    code, linked with the per-size kernel objects of the normal build (build() first).  Load it with the
    clang ASan runtime preloaded (see tests/test_host_sanitizers.py)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    kernels = [os.path.join(OBJDIR, f"tile_inst_m{m:02d}.o") for m in KERNEL_SIZES]
    missing = [k for k in kernels if not os.path.exists(k)]
    if missing:
        raise RuntimeError("the normal build's kernel objects are missing: run build() first")
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile_san, [(s, [], os.path.splitext(s)[0]) for s in SOURCES]))
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_FLAGS[:4], "-shared-libsan", *objs, *kernels,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitized link failed")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def build(jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    work = [("tile_inst.hip", [f"-DDIA_INST_M={m}"], f"tile_inst_m{m:02d}") for m in KERNEL_SIZES]
    work += [(s, [], os.path.splitext(s)[0]) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, work))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(OBJDIR, ignore_errors=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--sanitize", action="store_true", help="also build the host-sanitizer library")
    a = ap.parse_args()
    print(build(a.jobs))
    if a.sanitize:
        print(build_sanitized(a.jobs))
