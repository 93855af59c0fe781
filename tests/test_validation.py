"""Host-side argument checks of the Python binding and the C ABI that need no
GPU: wrong shapes, dtypes and entry counts raise before anything reaches a
kernel, and the batch builder refuses a group with cells but no nodes."""
import ctypes

import pytest
import torch

import paper_2107_04121_amd as fe


def _mesh_arrays(n_cells=4, nb=8, n_nodes=20):
    X = torch.zeros((n_nodes, 3), dtype=torch.float64)
    C = torch.zeros((n_cells, nb), dtype=torch.int32)
    return X, C


def test_conn_columns_and_dtypes():
    X, C = _mesh_arrays()
    with pytest.raises(ValueError, match="columns"):
        fe.validate_inputs(27, 27, 1, None, torch.float64, X, C)
    with pytest.raises(ValueError, match="coords"):
        fe.validate_inputs(8, 8, 1, None, torch.float64, X.float(), C)
    with pytest.raises(ValueError, match="int32"):
        fe.validate_inputs(8, 8, 1, None, torch.float64, X, C.long())


@pytest.mark.parametrize("kind,per_cell", [("iso_cell", 2), ("iso_qp", 16), ("voigt_qp", 288),
                                           ("tensor_qp", 72)])
def test_material_entry_count(kind, per_cell):
    X, C = _mesh_arrays()
    assert fe.material_entries(kind, 8) == per_cell
    good = torch.zeros(4 * per_cell, dtype=torch.float64)
    bad = torch.zeros(4 * per_cell + 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="material has"):
        fe.validate_inputs(8, 8, 3, kind, torch.float64, X, C, material=bad)
    # the right count passes the shape checks and stops only at the device check
    with pytest.raises(ValueError, match="cuda"):
        fe.validate_inputs(8, 8, 3, kind, torch.float64, X, C, material=good)


def test_iso_cell_array_on_iso_qp_plan():
    X, C = _mesh_arrays()
    with pytest.raises(ValueError, match="material has"):
        fe.validate_inputs(8, 8, 3, "iso_qp", torch.float64, X, C,
                           material=torch.zeros((4, 2), dtype=torch.float64))


def test_dofs_entry_count_and_dtype():
    X, C = _mesh_arrays()
    with pytest.raises(ValueError, match="dofs has"):
        fe.validate_inputs(8, 8, 3, None, torch.float64, X, C, dofs=torch.zeros(20, dtype=torch.float64))
    with pytest.raises(ValueError, match="dofs must be"):
        fe.validate_inputs(8, 8, 3, None, torch.float64, X, C, dofs=torch.zeros(60, dtype=torch.float32))


def test_batch_group_checks_before_the_library():
    X, C = _mesh_arrays()
    lm = torch.ones((4, 2), dtype=torch.float32)
    with pytest.raises(ValueError, match="coords"):
        fe.Batch([dict(cell="hex", order=1, forms=("mass",), coords=X.float(), conn=C)], autotune=False)
    with pytest.raises(ValueError, match="conn"):
        fe.Batch([dict(cell="hex", order=1, forms=("mass",), coords=X, conn=C.long())], autotune=False)
    with pytest.raises(ValueError, match="conn"):
        fe.Batch([dict(cell="hex", order=2, forms=("mass",), coords=X, conn=C)], autotune=False)
    with pytest.raises(ValueError, match="unknown forms"):
        fe.Batch([dict(cell="hex", order=1, forms=("stokes",), coords=X, conn=C)], autotune=False)
    with pytest.raises(ValueError, match="cuda"):
        fe.Batch([dict(cell="hex", order=1, forms=("elasticity",), coords=X, conn=C, material=lm)],
                 autotune=False)


def test_batch_group_with_cells_but_no_nodes():
    from paper_2107_04121_amd import _lib
    L = _lib.lib()
    g = (_lib.fe_group * 1)()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p).value
    g[0] = _lib.fe_group(0, 1, 1 << 0, 0, 5, 0, p, p, None, p, None, None)
    h = ctypes.c_void_p()
    assert L.fe_batch_create(1, g, 1, 0, ctypes.byref(h)) == 1
    assert b"bad group" in L.fe_last_error()
