"""The C ABI's host code (argument checks, workspace layouts, batched tile plans, the no-allocation
entry point's size check) under AddressSanitizer and UndefinedBehaviorSanitizer.  The library is
rebuilt with both sanitizers on its host pass (``paper_2104_13715_amd/build.py --sanitize``; the device
code is the normal build's) and exercised in a child process with the clang ASan runtime preloaded:
the CPU ABI checks of test_abi_cpu.py, then a sweep of workspace queries over kernel sizes, image
shapes, leading dimensions and epoch lists.  Any sanitizer report fails the test.  CPU only."""
import glob
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2104_13715_amd")


def _asan_runtime():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return rt[-1] if rt else None


def _builder():
    spec = importlib.util.spec_from_file_location("_dia_build_san", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def san_lib():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    b = _builder()
    if not all(os.path.exists(os.path.join(b.OBJDIR, f"tile_inst_m{m:02d}.o")) for m in b.KERNEL_SIZES):
        pytest.skip("the normal build's kernel objects are missing (run the build first)")
    srcs = [os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC)] + [os.path.join(ROOT, "include", "dia.h")]
    if not os.path.exists(b.SAN_LIB) or os.path.getmtime(b.SAN_LIB) < max(os.path.getmtime(f) for f in srcs):
        b.build_sanitized(jobs=min(8, os.cpu_count() or 1))
    return b.SAN_LIB, rt


def _run(san, args, timeout=600):
    lib, rt = san
    env = dict(os.environ, DIA_LIBRARY=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_abi_checks_under_sanitizers(san_lib):
    out = _run(san_lib, ["-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi_cpu.py"])
    assert "passed" in out


SWEEP = r'''
import ctypes, random
import paper_2104_13715_amd as dia
assert "libdia_san" in dia.LIB_PATH
lib = dia._lib
n = dia._sz(0)
random.seed(5)
count = 0
for m in range(1, 52):
    for op in range(-1, 7):
        for rows, cols in ((m, m), (m + 1, 3 * m), (97, 61), (480, 512), (2048, 1999), (4096, 4096), (1, 70000)):
            for pad in (0, 1, 77):
                st = lib.dia_workspace_size(op, rows, cols, cols + pad, m, ctypes.byref(n))
                count += 1
                if st == 0 and op in (1, 2, 3, 4):
                    assert n.value > 0
# batched plans: epoch lists of mixed sizes and offsets inside and outside the reference
R = dia._Image(0x100000, 2048, 2048, 2048)
for trial in range(60):
    k = random.randint(1, 40)
    arr = (dia._Epoch * k)()
    for e in range(k):
        side = random.randint(1, 2100)
        arr[e] = dia._Epoch(0x200000 + e * 0x1000, side, side, side + random.randint(0, 3),
                            random.randint(-5, 2048), random.randint(-5, 2048), None, None, None)
    for m in (1, 9, 17, 25, 49, 50):
        for prec in (0, 1, 2):
            for fit in (0, 1):
                lib.dia_batched_workspace_size(R, arr, k, m, prec, fit, ctypes.byref(n))
                count += 1
# the no-allocation entry point rejects a call beyond its scratch before anything is enqueued
obj = dia._Objective(0, 1, 5.0, 1.0, 2.0, 1.0, 1.345, None, None, None, 0.0, 0)
im = dia._Image(0x100000, 2048, 2048, 2048)
assert lib.dia_loss_grad_noalloc(im, im, ctypes.byref(obj), 0x200000, 49, 0x300000, 0x400000, None) == dia.E_SCRATCH
print("sweep calls", count)
'''


def test_workspace_and_plan_sweep_under_sanitizers(san_lib):
    out = _run(san_lib, ["-c", SWEEP])
    assert "sweep calls" in out
