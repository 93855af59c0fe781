"""The notation front-end drives the library: every form of the table of
example weak forms, given in the paper's notation (with renamed indices),
evaluates through the C ABI to the same output as the library plan of that
form, bit for bit, and within the parity gates of the oracle; a layout with
the cell axis last gives the cell-minor residual."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


CASES = [
    (("0,0", "q", "p"), "mass", None),
    (("k,k", "v", "u"), "vmass", None),
    (("0.j,0.j", "q", "p"), "laplace", None),
    (("ab,a,b", "M", "v", "u"), "wdot", "tensor_qp"),
    (("k,k.l,l", "v", "u", "u"), "convect", None),
    (("IK,s(i:j)->I,s(k:l)->K", "D", "v", "u"), "elasticity", "voigt_qp"),
]


@pytest.mark.parametrize("expr,form,kind", CASES)
def test_front_end_matches_plans(orc, expr, form, kind):
    import torch
    import paper_2107_04121_amd as fe
    from paper_2107_04121_amd.transpile import WeakForm
    mesh = meshgen.hex_mesh((4, 3, 3), 2, alpha=0.15, seed=60, curved=0.04)
    nb, nq = orc.sizes("hex", 2)
    nc = 1 if form in ("mass", "laplace") else 3
    U = meshgen.dofs(mesh.n_nodes, nc, seed=61)
    mat = (meshgen.tensor_qp(mesh.n_cells, nq, seed=62) if kind == "tensor_qp" else
           meshgen.voigt_random_spd((mesh.n_cells, nq), seed=62) if kind == "voigt_qp" else None)
    X, C, Ud = _t(mesh.coords), _t(mesh.conn), _t(U)
    M = None if mat is None else _t(mat)
    wf = WeakForm(expr, "hex", 2)
    assert wf.form == form
    for mode in ("matrix", "residual", "eval"):
        got = wf(X, C, mode=mode, material=M, dofs=Ud)
        wf.check()
        plan = fe.Plan("hex", 2, form, mode, "fp64", material=kind)
        ref = plan(X, C, material=M, dofs=Ud if (mode != "matrix" or form == "convect") else None)
        assert torch.equal(got, ref), mode
    K = wf(X, C, mode="matrix", material=M, dofs=Ud).cpu().numpy()
    ref = orc.matrix(mesh, form, mat, kind, u=U if form == "convect" else None)
    err = float((np.abs(K - ref).reshape(mesh.n_cells, -1).max(1) /
                 np.abs(ref).reshape(mesh.n_cells, -1).max(1)).max())
    assert err < 1e-12


def test_front_end_cell_minor_layout(orc):
    from paper_2107_04121_amd.transpile import WeakForm
    mesh = meshgen.hex_mesh((5, 4, 3), 3, alpha=0.15, seed=63, curved=0.04)
    U = meshgen.dofs(mesh.n_nodes, 1, seed=64)
    wf = WeakForm(("0.i,0.i", "v", "u"), "hex", 3, layout="qgvd0c")
    r = wf(_t(mesh.coords), _t(mesh.conn), mode="residual", dofs=_t(U))
    wf.check()
    assert tuple(r.shape) == (1, 64, mesh.n_cells)
    ref = orc.residual(mesh, "laplace", U)
    got = r.cpu().numpy().transpose(2, 0, 1)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12
