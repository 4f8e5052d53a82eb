"""C-ABI checks that need no GPU: the library loads, exports every function that
include/dia.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dia.h")
LIB = os.path.join(ROOT, "paper_2104_13715_amd", "libdia.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdia.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\*?\s*(dia_\w+)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("dia_model", "dia_loss_grad", "dia_fit", "dia_workspace_size", "dia_status_string"):
        assert f in names


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for f in declared_functions():
        getattr(lib, f)


def test_python_binding_exports_match_header():
    import paper_2104_13715_amd as dia
    assert set(dia.EXPORTS) <= set(declared_functions())


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


def test_status_strings(dia):
    assert dia.status_string(0) == "DIA_OK"
    for s in (1, -1, -2, -3, -4, -5, -6):
        assert dia.status_string(s).startswith("DIA_")
    assert dia.version() >= 10000


@pytest.mark.parametrize("m", [0, 2, 4, -1, 51, 50])
def test_workspace_size_rejects_bad_m(dia, m):
    with pytest.raises(dia.DIAError) as e:
        dia.workspace_size(dia.OP_LOSS_GRAD, 100, 100, 100, m)
    assert e.value.status == dia.E_SIZE


def test_workspace_size_rejects_small_images(dia):
    with pytest.raises(dia.DIAError):
        dia.workspace_size(dia.OP_FIT, 8, 100, 100, 9)
    with pytest.raises(dia.DIAError):
        dia.workspace_size(dia.OP_FIT, 100, 100, 99, 9)
    with pytest.raises(dia.DIAError):
        dia.workspace_size(7, 100, 100, 100, 9)


def test_workspace_sizes_grow_with_op(dia):
    a = dia.workspace_size(dia.OP_LOSS_GRAD, 300, 280, 288, 19)
    b = dia.workspace_size(dia.OP_FIT, 300, 280, 288, 19)
    c = dia.workspace_size(dia.OP_FIT_CLIPPED, 300, 280, 288, 19)
    assert dia.workspace_size(dia.OP_MODEL, 300, 280, 288, 19) == 0
    assert 0 < a < b < c
    assert c - b >= 300 * 288 * 5


def _img(dia, ptr=0x100000, rows=64, cols=64, ld=64):
    return dia._Image(ptr, rows, cols, ld)


def _call_loss_grad(dia, R, I, obj, m=9, theta=0x200000, loss=0x300000, grad=0x400000, ws=0x500000,
                    nbytes=1 << 30):
    return dia._lib.dia_loss_grad(R, I, ctypes.byref(obj) if obj is not None else None, theta, m, loss, grad, ws,
                                  nbytes, None)


def _obj(dia, **kw):
    base = dict(rho=0, var=1, sigma0=5.0, gain=1.0, excess=2.0, var_floor=1.0, c=1.345, weights=None, flat=None,
                mask=None)
    base.update(kw)
    return dia._Objective(**base)


def test_loss_grad_argument_errors_return_before_hip(dia):
    R, I = _img(dia), _img(dia)
    assert _call_loss_grad(dia, R, I, _obj(dia), m=8) == dia.E_SIZE
    assert _call_loss_grad(dia, R, I, _obj(dia), m=65) == dia.E_SIZE
    assert _call_loss_grad(dia, _img(dia, ptr=0), I, _obj(dia)) == dia.E_ARG
    assert _call_loss_grad(dia, R, _img(dia, rows=63), _obj(dia)) == dia.E_SIZE
    assert _call_loss_grad(dia, R, _img(dia, ld=32), _obj(dia)) == dia.E_SIZE
    assert _call_loss_grad(dia, R, I, None) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, rho=3)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, var=5)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, var=0)) == dia.E_ARG            # weights missing
    assert _call_loss_grad(dia, R, I, _obj(dia, gain=0.0)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, rho=1, c=0.0)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, var=3, var_floor=0.0)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, sigma0=0.0, var_floor=0.0)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, lam=-1.0)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, lam=float("nan"))) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, lam=float("inf"))) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, bg_degree=-1)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia, bg_degree=dia.MAX_BG_DEGREE + 1)) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia), theta=0) == dia.E_ARG
    assert _call_loss_grad(dia, R, I, _obj(dia), ws=0) == dia.E_WORKSPACE
    assert _call_loss_grad(dia, R, I, _obj(dia), ws=0x500001) == dia.E_WORKSPACE
    assert _call_loss_grad(dia, R, I, _obj(dia), nbytes=16) == dia.E_WORKSPACE


def test_fit_option_errors_return_before_hip(dia):
    R, I = _img(dia), _img(dia)
    obj = _obj(dia)
    res = dia._FitResult()

    def call(**kw):
        o = dia.fit_options(**kw)
        return dia._lib.dia_fit(R, I, ctypes.byref(obj), 9, ctypes.byref(o), 0x200000, ctypes.byref(res), 0x500000,
                                1 << 30, None)

    assert call(history=0) == dia.E_ARG
    assert call(history=33) == dia.E_ARG
    assert call(lr_K=0.0) == dia.E_ARG
    assert call(beta1=1.0) == dia.E_ARG
    assert call(max_eval=0) == dia.E_ARG
    assert call(init=1, init_phi=0.0) == dia.E_ARG
    assert call(clip_kappa=-1.0) == dia.E_ARG
    assert call(max_lbfgs=-1) == dia.E_ARG
    obj.bg_degree = 1  # the reweight/clip loop keeps the scalar background
    assert call(max_outer=3, clip_kappa=3.0) == dia.E_ARG
    obj.bg_degree = 0
    assert call(poll_every=0) == dia.E_ARG
    o = dia.fit_options(max_outer=3)
    wobj = _obj(dia, var=0, weights=0x700000)
    assert dia._lib.dia_fit(R, I, ctypes.byref(wobj), 9, ctypes.byref(o), 0x200000, ctypes.byref(res), 0x500000,
                            1 << 30, None) == dia.E_ARG
    small = dia.workspace_size(dia.OP_FIT, 64, 64, 64, 9)
    o = dia.fit_options(max_outer=3)
    assert dia._lib.dia_fit(R, I, ctypes.byref(obj), 9, ctypes.byref(o), 0x200000, ctypes.byref(res), 0x500000,
                            small, None) == dia.E_WORKSPACE


def test_model_argument_errors(dia):
    R = _img(dia)
    assert dia._lib.dia_model(R, 0x200000, 9, 0x300000, 10, None) == dia.E_SIZE   # ldM < cols - m + 1
    assert dia._lib.dia_model(R, 0, 9, 0x300000, 56, None) == dia.E_ARG
    assert dia._lib.dia_model(R, 0x200000, 10, 0x300000, 56, None) == dia.E_SIZE


def test_default_options_follow_the_paper(dia):
    o = dia.fit_options()
    assert o.lr_K == 1e-3 and o.lr_B0 == 10.0 and o.tol_switch == 1e-6
    assert o.history == 10 and o.init == dia.INIT["flat"] and o.max_outer == 1


def test_struct_layouts_match_the_header(dia, tmp_path):
    # the ctypes mirrors of the ABI structs have the C compiler's sizes and field offsets
    structs = {"dia_image": dia._Image, "dia_objective": dia._Objective, "dia_epoch": dia._Epoch,
               "dia_fit_opts": dia._FitOpts, "dia_fit_result": dia._FitResult}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "dia.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if (cname == "dia_objective" and fname == "lam") else fname
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_tile_shape_query(dia, monkeypatch):
    # the default shape before any tuning, and every pinned variant's geometry (m = 19: 13 strips of 8
    # columns; the wide default has two forward rows per thread, the two-set shape two sets of one row,
    # the short two-set shape 8 strips, the split-kernel-row shapes 8 and 3)
    assert dia.tile_shape(19, 4096, 4096) == (0, 38, 104)
    for v, ty, tx in ((1, 19, 104), (2, 38, 104), (4, 38, 104), (5, 19, 24), (6, 38, 64), (7, 19, 64), (8, 19, 24)):
        monkeypatch.setenv("DIA_TILE_VARIANT", str(v))
        assert dia.tile_shape(19, 4096, 4096) == (v, ty, tx)
    with pytest.raises(dia.DIAError):
        dia.tile_shape(18, 100, 100)
