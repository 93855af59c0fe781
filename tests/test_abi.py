"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function the public header declares, reports status names, refuses to
plan without a device, and its own reference tables agree with the oracle's
independently built ones."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2107_04121_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "fe_execute" in names and len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    from paper_2107_04121_amd import _lib
    assert set(_lib.EXPORTS) <= set(names)


def test_status_strings(L):
    from paper_2107_04121_amd import _lib
    for code, name in _lib.STATUS.items():
        assert L.fe_status_string(code).decode() == name
    assert L.fe_status_string(99).decode() == "FE_ERR_UNKNOWN"


def test_reference_sizes(L):
    import paper_2107_04121_amd as fe
    assert fe.reference_sizes("hex", 2) == (27, 27)
    assert fe.reference_sizes("hex", 3) == (64, 64)
    assert fe.reference_sizes("tet", 2) == (10, 27)
    with pytest.raises(fe.FeError):
        fe.reference_sizes("tet", 3)


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("hex", 3),
                                    ("hex", 4), ("hex", 5), ("tet", 1),
                                    ("tet", 2)])
def test_library_tables_match_oracle(orc, cell, p):
    import paper_2107_04121_amd as fe
    lib_t = fe.reference_tables(cell, p)
    orc_t = orc.tables(cell, p)
    for name, a, b in zip(("w", "pts", "bf", "bfg"), lib_t, orc_t):
        assert np.abs(a - b).max() <= 1e-14 * max(1.0, np.abs(b).max()) * (
            10 if p >= 3 else 1), name


def test_argument_validation_without_device(L):
    from paper_2107_04121_amd import _lib
    h = ctypes.c_void_p()
    opts = _lib.fe_options(0, 0, 0, -1)
    # invalid arguments are rejected before any device query
    assert L.fe_plan_create(7, 1, 0, 0, 0, 0, ctypes.byref(opts),
                            ctypes.byref(h)) == 1
    assert L.fe_plan_create(0, 1, 3, 0, 0, 0, ctypes.byref(opts),
                            ctypes.byref(h)) == 1   # elasticity w/o material
    assert L.fe_plan_create(0, 1, 2, 0, 0, 1, ctypes.byref(opts),
                            ctypes.byref(h)) == 1   # laplace with material
    assert L.fe_plan_create(0, 9, 2, 0, 0, 0, ctypes.byref(opts),
                            ctypes.byref(h)) == 2   # unsupported order
    assert L.fe_plan_create(0, 1, 4, 0, 0, 1, ctypes.byref(opts),
                            ctypes.byref(h)) == 1   # weighted dot w/o TENSOR_QP
    assert L.fe_plan_create(0, 1, 5, 0, 0, 4, ctypes.byref(opts),
                            ctypes.byref(h)) == 1   # convection with material
    assert L.fe_plan_create(0, 1, 6, 0, 0, 0, ctypes.byref(opts),
                            ctypes.byref(h)) == 1   # no such form
    assert L.fe_execute(None, 1, 1, None, None, None, None, None, None, 0,
                        None) == 1
    assert L.fe_plan_destroy(None) == 0


def test_no_device_is_an_error_not_a_fallback(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2107_04121_amd as fe
    with pytest.raises(fe.FeError) as ei:
        fe.Plan("hex", 1, "laplace", "matrix")
    assert ei.value.status == 7
