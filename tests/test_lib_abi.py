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
    assert lib.ct_valu_probe(0, 16, 0, None, None) == -1
    assert lib.ct_valu_probe(1, 16, 5, None, None) == -1
    assert lib.ct_copy_probe(None, None, 16, 1, None) == -1
    assert lib.ct_version() >= 10000


def test_params_default(lib):
    from paper_1810_03275_amd import _lib
    p = _lib.CtParams()
    p.fwd_walk = 7
    lib.ct_params_default(ctypes.byref(p))
    assert p.sigma == 1.0 and abs(p.tau - 8 ** -0.5) < 1e-15 and p.eps == 0.3
    assert p.c_safety == pytest.approx(1.1) and p.power_iters == 30 and p.c == 0.0
    # launch choices: all left to the tuning, no cache file
    assert p.bp_slices == 0 and p.bp_kernel == -1 and p.tv_blocks == 0 and p.options == 0
    assert p.tune_cache is None and p.fwd_walk == 0


def test_plan_options_validation(lib):
    """Plan options are checked on the host: unknown values are invalid, and
    the mirror-pair backprojector needs angles that pair as theta, pi - theta
    (one angle has no partner)."""
    from paper_1810_03275_amd import _lib
    g = _lib.CtGeom(64, 90, 96, 1.0, 1.0)
    steps = ctypes.c_int64()
    for bad in (_lib.CtPlanOpts(5, 0), _lib.CtPlanOpts(-1, 3)):
        assert lib.ct_plan_check_ex(ctypes.byref(g), None, ctypes.byref(bad),
                                    ctypes.byref(steps)) == -1
    ok = _lib.CtPlanOpts(8, 2)
    assert lib.ct_plan_check_ex(ctypes.byref(g), None, ctypes.byref(ok), ctypes.byref(steps)) == 0
    one = _lib.CtGeom(64, 1, 96, 1.0, 1.0)
    pairs = _lib.CtPlanOpts(4, 0)
    assert lib.ct_plan_check_ex(ctypes.byref(one), None, ctypes.byref(pairs),
                                ctypes.byref(steps)) == -2
    assert b"pair" in lib.ct_last_error()
    walk1 = _lib.CtPlanOpts(-1, 1)
    assert lib.ct_plan_check_ex(ctypes.byref(g), None, ctypes.byref(walk1),
                                ctypes.byref(steps)) == 0


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the C layout: a probe built
    from the header by the host C compiler prints every size and offset."""
    import shutil
    import subprocess
    from paper_1810_03275_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"ct_geom": _lib.CtGeom, "ct_problem": _lib.CtProblem,
               "ct_params": _lib.CtParams, "ct_plan_opts": _lib.CtPlanOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ctpd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname   # a Python keyword
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, what, val = line.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), (cname, what, got, val)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())


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
