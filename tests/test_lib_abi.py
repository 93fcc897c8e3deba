"""The C-ABI library loads, exports every symbol the header declares, and its
host-side validation returns the documented error codes (no GPU needed:
every call here fails validation before touching the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctpd.h")
LIB = os.path.join(ROOT, "paper_1810_03275_amd", "libctpd.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libctpd.so is not built (run __graft_entry__.build())")
    from paper_1810_03275_amd import _lib
    return _lib.load(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ct_radon_fwd", "ct_radon_adj", "ct_grad", "ct_div", "ct_precond_apply",
                 "ct_pd_step", "ct_reconstruct", "ct_gap", "ct_power_norm"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_declares_every_symbol():
    from paper_1810_03275_amd import _lib
    assert set(_lib.SIGNATURES) == set(_declared())


def test_validation_errors_without_device(lib):
    from paper_1810_03275_amd import _lib
    h = ctypes.c_void_p()
    bad = [
        _lib.CtGeom(0, 10, 10, 1.0, 1.0),      # n < 2
        _lib.CtGeom(8, 0, 10, 1.0, 1.0),       # N < 1
        _lib.CtGeom(8, 10, 1, 1.0, 1.0),       # M < 2
        _lib.CtGeom(8, 10, 10, -1.0, 1.0),     # h <= 0
        _lib.CtGeom(8, 10, 10, 1.0, 0.0),      # ds <= 0
    ]
    for g in bad:
        assert lib.ct_plan_create(ctypes.byref(g), None, ctypes.byref(h)) == -1
        assert b"ct_plan_create" in lib.ct_last_error()
    g = _lib.CtGeom(8, 10, 10, 1.0, 2.0)       # ds/h outside [0.75, 1.4]
    assert lib.ct_plan_create(ctypes.byref(g), None, ctypes.byref(h)) == -2
    g = _lib.CtGeom(16384, 10, 10, 1.0, 1.0)
    assert lib.ct_plan_create(ctypes.byref(g), None, ctypes.byref(h)) == -2
    nan_angles = (ctypes.c_double * 10)(*([0.0] * 9 + [float("nan")]))
    g = _lib.CtGeom(8, 10, 10, 1.0, 1.0)
    assert lib.ct_plan_create(ctypes.byref(g), nan_angles, ctypes.byref(h)) == -1
    assert lib.ct_plan_create(None, None, ctypes.byref(h)) == -1
    assert lib.ct_radon_fwd(None, None, None, None) == -1
    assert lib.ct_radon_adj(None, None, None, None) == -1
    assert lib.ct_grad(0, 1.0, None, None, None) == -1
    assert lib.ct_div(8, 0.0, None, None, None) == -1
    assert lib.ct_tv_project(8, None, 1.0, None, None) == -1
    assert lib.ct_pd_step(None, 1, None) == -1
    assert lib.ct_gap(None, None, None) == -1
    assert lib.ct_solver_create(None, None, None, None, ctypes.byref(h)) == -1
    pc = ctypes.c_void_p()
    assert lib.ct_precond_create(10, 1.0, 0.3, 1.0, 0.3, ctypes.byref(pc)) == -2  # 10 = 2*5
    assert lib.ct_precond_create(64, -1.0, 0.3, 1.0, 0.3, ctypes.byref(pc)) == -1
    assert lib.ct_precond_create(63, 1.0, 0.3, 1.0, 0.3, ctypes.byref(pc)) == -2  # odd
    assert lib.ct_plan_destroy(None) == 0 and lib.ct_solver_destroy(None) == 0
    assert lib.ct_version() >= 10000


def test_params_default(lib):
    from paper_1810_03275_amd import _lib
    p = _lib.CtParams()
    lib.ct_params_default(ctypes.byref(p))
    assert p.sigma == 1.0 and abs(p.tau - 8 ** -0.5) < 1e-15 and p.eps == 0.3
    assert p.c_safety == pytest.approx(1.1) and p.power_iters == 30 and p.c == 0.0


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the C layout (x86-64 SysV)."""
    from paper_1810_03275_amd import _lib
    assert ctypes.sizeof(_lib.CtGeom) == 32
    assert _lib.CtGeom.h.offset == 16 and _lib.CtGeom.ds.offset == 24
    assert ctypes.sizeof(_lib.CtProblem) == 40 and _lib.CtProblem.lambda_.offset == 32
    assert ctypes.sizeof(_lib.CtParams) == 80 and _lib.CtParams.start_norm.offset == 64


def test_package_import_requires_library(monkeypatch, tmp_path):
    """The product path fails loudly without the built library (no fallback)."""
    from paper_1810_03275_amd import _lib
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))


def test_mask_packing():
    import numpy as np
    import paper_1810_03275_amd as ct
    m = np.zeros((3, 70), bool)
    m[0, 0] = m[1, 31] = m[1, 32] = m[2, 69] = True
    pad = np.zeros((3, 96), bool)
    pad[:, :70] = m
    bits = np.packbits(pad, axis=1, bitorder="little").view(np.uint32)
    assert bits[0, 0] == 1 and bits[1, 0] == 1 << 31 and bits[1, 1] == 1 and bits[2, 2] == 1 << 5
    assert callable(ct.pack_mask)
