"""Edge cases of the matrix-core, high-order and assembly paths through the
C ABI: an empty mesh (no launch, empty output), a single cell (one persistent
workgroup, ragged tiles) against the oracle, a single cell with an inverted
Jacobian reported as a fault, and a two-cell assembly."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _err(got, ref):
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.maximum(np.abs(r).max(1), 1e-300)).max())


CASES = [
    # (order, form, mode, material kind, expected variant)
    (4, "elasticity", "matrix", "iso_cell", "mfma"),
    (5, "laplace", "matrix", None, "mfma"),
    (5, "vmass", "matrix", None, "mfma"),
    (4, "elasticity", "residual", "iso_qp", "sumfact"),
    (5, "mass", "eval", None, "sumfact"),
    (2, "convect", "matrix", None, "mfma"),
    (3, "wdot", "matrix", "tensor_qp", "mfma"),
]


def _inputs(orc, mesh, form, kind, p):
    nb, nq = orc.sizes("hex", p)
    mat = {"iso_cell": lambda: meshgen.lame_cell(mesh.n_cells, seed=71),
           "iso_qp": lambda: meshgen.lame_qp(mesh.n_cells, nq, seed=71),
           "tensor_qp": lambda: meshgen.tensor_qp(mesh.n_cells, nq, seed=71)}.get(kind, lambda: None)()
    U = meshgen.dofs(mesh.n_nodes, orc.n_comp(form), seed=72)
    return mat, U


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p,form,mode,kind,variant", CASES)
def test_empty_and_single_cell(orc, p, form, mode, kind, variant, prec):
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(1, p, alpha=0.0, seed=70, curved=0.01)
    mat, U = _inputs(orc, mesh, form, kind, p)
    plan = fe.Plan("hex", p, form, mode, prec, material=kind)
    assert plan.variant == variant
    dt = plan.dtype
    X, C = _t(mesh.coords), _t(mesh.conn)
    M = None if mat is None else _t(mat, dt)
    dofs = _t(U, dt) if (mode != "matrix" or form == "convect") else None
    print(f"[edge] Q{p} {form} {mode} {prec} empty + single cell", flush=True)
    empty = plan(X, C[:0], material=None if M is None else M[:0], dofs=dofs)
    plan.check()
    assert empty.shape[0] == 0 or (mode == "eval" and empty.numel() == 0)
    out = plan(X, C, material=M, dofs=dofs)
    plan.check()
    if mode == "matrix":
        ref = orc.matrix(mesh, form, mat, kind, u=U if form == "convect" else None)
    elif mode == "residual":
        ref = orc.residual(mesh, form, U, mat, kind)
    else:
        ref = orc.energy(mesh, form, U, mat, kind)
    assert _err(out.cpu().numpy(), ref) < TOL[prec]
    torch.cuda.synchronize()


@pytest.mark.parametrize("p,form,kind", [(4, "laplace", None), (5, "elasticity", "iso_cell"),
                                         (2, "convect", None), (3, "wdot", "tensor_qp")])
def test_inverted_cell_is_reported(orc, p, form, kind):
    """A cell whose first two vertex layers are swapped has det J < 0 at
    every point: the matrix kernels raise the fault flag, plan.check()
    reports it, and the call does not fault the device."""
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(1, p, alpha=0.0, seed=73)
    n1 = p + 1
    conn = mesh.conn.reshape(1, n1, n1, n1)[:, :, :, ::-1].reshape(1, -1).copy()  # mirror x: det < 0
    mat, U = _inputs(orc, mesh, form, kind, p)
    plan = fe.Plan("hex", p, form, "matrix", "fp64", material=kind)
    plan(_t(mesh.coords), _t(conn), material=None if mat is None else _t(mat),
         dofs=_t(U) if form == "convect" else None)
    with pytest.raises(fe.FeError) as ei:
        plan.check()
    assert ei.value.status == 3  # FE_ERR_NONPOSITIVE_JACOBIAN


def test_assembly_two_cells(orc):
    """Two Q2 cells sharing a face: the assembled matrix equals the oracle's
    (shared rows hold sums from both cells)."""
    import paper_2107_04121_amd as fe
    import scipy.sparse as sp
    mesh = meshgen.hex_mesh((2, 1, 1), 2, alpha=0.1, seed=74)
    C = _t(mesh.conn)
    plan = fe.Plan("hex", 2, "laplace", "matrix", "fp64")
    Ke = plan(_t(mesh.coords), C)
    pat = fe.Pattern(C, mesh.n_nodes)
    inc = fe.Incidence(C, mesh.n_nodes)
    vals = fe.assemble_matrix(pat, inc, C, Ke)
    got = sp.bsr_matrix((vals.cpu().numpy(), pat.cols.cpu().numpy(), pat.row_ptr.cpu().numpy()),
                        shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    ref = orc.assemble_matrix(mesh, orc.matrix(mesh, "laplace"), 1)
    assert abs(got - ref).max() / abs(ref).max() < 1e-12
    assert pat.nnz == ref.nnz
