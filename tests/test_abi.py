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
    opts = _lib.fe_options(0, -1, 0, 0)
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


def _ref_struct(cell, p, w, bf, bfg):
    import paper_2107_04121_amd as fe
    return fe.make_reference(cell, p, w, bf, bfg)


def test_caller_reference_validation_without_device(orc):
    """fe_plan_create_ref checks the caller's tables before any device
    query: sizes the kernels are not compiled for and hexahedral tables that
    do not factor are FE_ERR_UNSUPPORTED, non-positive weights and a basis
    that is not a partition of unity FE_ERR_INVALID_ARG."""
    from paper_2107_04121_amd import _lib
    L = _lib.lib()
    opts = _lib.fe_options(0, -1, 0, 0)
    h = ctypes.c_void_p()
    w, _, bf, bfg = orc.tables("hex", 2)

    def create(w_, bf_, bfg_, cell="hex", p=2):
        ref, keep = _ref_struct(cell, p, w_, bf_, bfg_)
        return L.fe_plan_create_ref(ctypes.byref(ref), 2, 0, 0, 0, ctypes.byref(opts), ctypes.byref(h))

    # the oracle's own tables pass validation and stop at the device query
    assert create(w, bf, bfg) == 7
    # [-1,1]^3 tables (weights x 8, gradients x 1/2) are valid too
    assert create(8 * w, bf, 0.5 * bfg) == 7
    # a rule with one point less: not what the kernels are compiled for
    assert create(w[:-1], bf[:-1], bfg[:-1]) == 2
    # a negative weight
    w2 = w.copy()
    w2[3] = -w2[3]
    assert create(w2, bf, bfg) == 1
    # not a partition of unity
    assert create(w, 1.01 * bf, bfg) == 1
    # permuted points: no longer lexicographic tensor-product tables
    perm = np.random.default_rng(0).permutation(len(w))
    assert create(w[perm], bf[perm], bfg[perm]) == 2
    # P1 tetrahedron with non-constant gradients is refused
    wt, _, bft, bfgt = orc.tables("tet", 1)
    bfgt2 = bfgt.copy()
    bfgt2[1, 0, 0] += 0.1
    bfgt2[1, 0, 1] -= 0.1
    assert create(wt, bft, bfgt2, "tet", 1) == 2
    assert create(wt, bft, bfgt, "tet", 1) == 7


def test_bilinear_validation_without_device():
    from paper_2107_04121_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    W0 = np.eye(3)
    dp = ctypes.POINTER(ctypes.c_double)
    good = _lib.fe_bilinear(1, 1, 1, 1, W0.ctypes.data_as(dp), None, None, 0, 0, 0)
    bad_op = _lib.fe_bilinear(2, 1, 1, 1, W0.ctypes.data_as(dp), None, None, 0, 0, 0)
    bad_comp = _lib.fe_bilinear(1, 2, 1, 1, W0.ctypes.data_as(dp), None, None, 0, 0, 0)
    no_w = _lib.fe_bilinear(1, 1, 1, 1, None, None, None, 0, 0, 0)
    args = (0, 1, 0, 0, 0)
    assert L.fe_plan_create_bilinear(*args, ctypes.byref(bad_op), None, ctypes.byref(h)) == 1
    assert L.fe_plan_create_bilinear(*args, ctypes.byref(bad_comp), None, ctypes.byref(h)) == 1
    assert L.fe_plan_create_bilinear(*args, ctypes.byref(no_w), None, ctypes.byref(h)) == 1
    assert L.fe_plan_create_bilinear(0, 1, 0, 0, 4, ctypes.byref(good), None, ctypes.byref(h)) == 1  # no P
    assert L.fe_plan_create_bilinear(*args, ctypes.byref(good), None, ctypes.byref(h)) == 7
    # the ordinary creator refuses the bilinear form id
    assert L.fe_plan_create(0, 1, 6, 0, 0, 0, None, ctypes.byref(h)) == 1
