"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/icm.h declares, and validates parameters."""
import ctypes
import os
import re

import pytest

import paper_1212_6427_amd.icm as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "icm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(icm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "icm_step" in names and "icm_create" in names
    lib = ctypes.CDLL(I.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(I.icm_replica_params) == 160
    assert ctypes.sizeof(I.icm_diag) == 64
    assert ctypes.sizeof(I.icm_tune_result) == 72


def test_struct_offsets_match_the_c_compiler(tmp_path):
    """Every field of the ctypes mirrors sits at the offset gcc gives the
    header's struct (and the sizes agree)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    structs = [I.icm_replica_params, I.icm_diag, I.icm_tune_result]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "icm.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for fname, _ in st._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, fname, name, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                    text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for fname, _ in st._fields_:
            assert int(got["%s.%s" % (name, fname)]) == getattr(st, fname).offset, (name, fname)


@pytest.mark.parametrize("n,ok", [((32, 32, 32), True), ((48, 36, 24), True), ((6, 12, 18), True),
                                  ((512, 4, 4), True), ((33, 32, 32), False), ((2, 32, 32), False),
                                  ((1024, 4, 4), False), ((20, 32, 32), False), ((14, 32, 32), False)])
def test_grid_size_validation(n, ok):
    p = I.make_params(n)
    if ok:
        assert I.icm_workspace_bytes([p], [3], I.FP64) > 0
    else:
        with pytest.raises(I.ICMError) as e:
            I.icm_workspace_bytes([p], [3], I.FP64)
        assert e.value.status == I.E_INVALID


@pytest.mark.parametrize("field,val", [("kernel", 5), ("h", 0.0), ("rho", -1.0), ("dt", 0.0), ("kT", -1.0),
                                       ("slip", 3), ("thermal_drift", 2), ("advection", 2)])
def test_parameter_validation(field, val):
    p = I.make_params((16, 16, 16))
    setattr(p, field, val)
    with pytest.raises(I.ICMError) as e:
        I.icm_workspace_bytes([p], [1], I.FP64)
    assert e.value.status == I.E_INVALID


@pytest.mark.parametrize("kernel,shift,ok", [(3, 0.0, True), (3, 0.5, True), (3, 1.0, True), (4, 0.0, True),
                                              (4, 0.5, False), (3, 1.5, False), (3, -0.1, False),
                                              (3, float("nan"), False)])
def test_kernel_shift_validation(kernel, shift, ok):
    """The split kernel (Sec. III.A.2) is the three-point kernel's, for
    shifts up to one grid spacing."""
    p = I.make_params((16, 16, 16), kernel=kernel, kernel_shift=shift)
    if ok:
        assert I.icm_workspace_bytes([p], [2], I.FP64) > 0
    else:
        with pytest.raises(I.ICMError) as e:
            I.icm_workspace_bytes([p], [2], I.FP64)
        assert e.value.status == I.E_INVALID


def test_wca_cutoff_must_fit_half_box():
    p = I.make_params((8, 8, 8), wca_eps=1e-2, wca_sigma=4.0)
    with pytest.raises(I.ICMError):
        I.icm_workspace_bytes([p], [2], I.FP64)


def test_workspace_scales_with_precision_and_replicas():
    p = I.make_params((64, 64, 64))
    b64 = I.icm_workspace_bytes([p], [10], I.FP64)
    b32 = I.icm_workspace_bytes([p], [10], I.FP32_GRID)
    assert 0.45 * b64 < b32 < 0.55 * b64
    q = I.make_params((32, 32, 32))
    both = I.icm_workspace_bytes([p, q], [10, 1], I.FP32_GRID)
    assert both > b32
    with pytest.raises(I.ICMError):
        I.icm_workspace_bytes([p], [-1], I.FP64)
    with pytest.raises(I.ICMError):
        I.icm_workspace_bytes([p], [1], 7)


@pytest.mark.parametrize("prec,w", [("FP64", 8), ("FP32_GRID", 4)])
def test_advection_adds_one_face_field_of_workspace(prec, w):
    n = (32, 24, 16)
    off = I.icm_workspace_bytes([I.make_params(n)], [4], getattr(I, prec))
    on = I.icm_workspace_bytes([I.make_params(n, advection=True)], [4], getattr(I, prec))
    field = 3 * 32 * 24 * 16 * w
    assert field <= on - off <= field + 512


def test_solve_noalloc_validates_before_touching_the_device():
    """Bad sizes, coefficients, precision or NULL fields are refused with
    ICM_E_INVALID and a message, before any HIP call (so also without a GPU)."""
    bad = [((16, 16, 15), 1.0, 1.0, 0.0, I.FP64), ((16, 16, 1024), 1.0, 1.0, 0.0, I.FP64),
           ((16, 14, 16), 1.0, 1.0, 0.0, I.FP64), ((16, 16, 16), 0.0, 1.0, 0.0, I.FP64),
           ((16, 16, 16), 1.0, 0.0, 0.0, I.FP64), ((16, 16, 16), 1.0, 1.0, -1.0, I.FP64),
           ((16, 16, 16), 1.0, 1.0, 0.0, 7)]
    for n, h, a, b, prec in bad:
        with pytest.raises(I.ICMError) as e:
            I.icm_solve_noalloc(n, h, a, b, prec, 1 << 20, 1 << 20, 0)
        assert e.value.status == I.E_INVALID, (n, h, a, b, prec)
        assert "icm_solve_noalloc" in str(e.value)
    with pytest.raises(I.ICMError) as e:
        I.icm_solve_noalloc((16, 16, 16), 1.0, 1.0, 0.0, I.FP64, 0, 1 << 20, 0)
    assert e.value.status == I.E_INVALID
