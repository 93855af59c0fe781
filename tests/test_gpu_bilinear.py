"""The generic bilinear kernel (fe_plan_create_bilinear) driven by the
notation front-end: forms of the table of example weak forms that also have
dedicated kernels, evaluated through the derived coupling tables against the
FP64 oracle, and bilinear forms with no dedicated kernel (the Stokes
couplings, the vector Laplacian, the weighted dot with M transposed, a
gradient-value coupling) against numpy.einsum of the derived expressions
over the oracle's own operands (oracle.einsum_form), in matrix, residual and
eval mode, FP64 and FP32, on meshes that span several workgroups.

Gates: FP64 1e-12, FP32 1e-5 of each cell's max-norm (eval: of the largest
cell value)."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _mesh(cell, p):
    if cell == "hex":
        dims = {1: (5, 4, 3), 2: (4, 3, 3), 3: (3, 2, 2)}[p]
        return meshgen.hex_mesh(dims, p, alpha=0.15, seed=80 + p, curved=0.04 if p > 1 else 0.0)
    return meshgen.tet_mesh((3, 3, 2), p, alpha=0.15, seed=80 + p)


def _err(got, ref):
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.maximum(np.abs(r).max(1), 1e-300)).max())


def _cell_dofs(mesh, U):
    ue = U[mesh.conn]                                    # (c, d, nc)
    return ue[:, :, 0] if U.shape[1] == 1 else np.transpose(ue, (0, 2, 1))


CELLS = [("hex", 1), ("hex", 2), ("hex", 3), ("tet", 1), ("tet", 2)]
DEDICATED = [(("0,0", "v", "u"), "mass", None),
             (("i,i", "v", "u"), "vmass", None),
             (("0.i,0.i", "v", "u"), "laplace", None),
             (("ij,i,j", "M", "v", "u"), "wdot", "tensor_qp"),
             (("IK,s(i:j)->I,s(k:l)->K", "D", "v", "u"), "elasticity", "voigt_qp")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("expr,form,kind", DEDICATED)
@pytest.mark.parametrize("cell,p", CELLS)
def test_generic_kernel_on_the_table_forms(orc, cell, p, expr, form, kind, prec):
    import paper_2107_04121_amd as fe
    from paper_2107_04121_amd.transpile import transpile
    t = transpile(*expr)
    assert t.form == form
    mesh = _mesh(cell, p)
    nb, nq = orc.sizes(cell, p)
    nc = t.n_comp
    U = meshgen.dofs(mesh.n_nodes, nc, seed=82)
    mat = None
    if kind == "tensor_qp":
        mat = meshgen.tensor_qp(mesh.n_cells, nq, seed=83)
    elif kind == "voigt_qp":
        mat = meshgen.voigt_random_spd((mesh.n_cells, nq), seed=83)
    X, C = _t(mesh.coords), _t(mesh.conn)
    refs = {"matrix": orc.matrix(mesh, form, mat, kind),
            "residual": orc.residual(mesh, form, U, mat, kind),
            "eval": orc.energy(mesh, form, U, mat, kind)}
    for mode, ref in refs.items():
        plan = fe.BilinearPlan(t, cell, p, mode, prec)
        print(f"[bilinear] {cell}{p} {form} {mode} {prec} cells={mesh.n_cells}", flush=True)
        dt = plan.dtype
        out = plan(X, C, material=None if mat is None else _t(mat, dt),
                   dofs=None if mode == "matrix" else _t(U, dt))
        plan.check()
        got = out.cpu().numpy()
        err = (float(np.abs(got - ref).max() / np.abs(ref).max()) if mode == "eval"
               else _err(got, ref))
        assert err < TOL[prec], (mode, err)


NEW = [(("i.i,0", "v", "p"), 3, 1, None),           # Stokes coupling
       (("0,i.i", "q", "u"), 1, 3, None),           # transposed Stokes coupling
       (("i.j,i.j", "v", "u"), 3, 3, None),         # vector Laplacian
       (("0.i,i", "q", "u"), 1, 3, None),           # gradient of a scalar against a vector
       (("ji,i,j", "M", "v", "u"), 3, 3, "M")]      # weighted dot with M transposed


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("expr,nct,ncu,mname", NEW)
@pytest.mark.parametrize("cell,p", [("hex", 2), ("hex", 1), ("tet", 2)])
def test_forms_without_a_dedicated_kernel(orc, cell, p, expr, nct, ncu, mname, prec):
    import paper_2107_04121_amd as fe
    from paper_2107_04121_amd.transpile import WeakForm, transpile
    t = transpile(*expr)
    assert t.form is None and t.structure["kernel"] == "bilinear"
    mesh = _mesh(cell, p)
    nb, nq = orc.sizes(cell, p)
    U = meshgen.dofs(mesh.n_nodes, ncu, seed=84)
    arrays = {"dofs": _cell_dofs(mesh, U)}
    M = None
    if mname:
        M = meshgen.tensor_qp(mesh.n_cells, nq, seed=85)
        arrays[mname] = M
    X, C = _t(mesh.coords), _t(mesh.conn)
    wf = WeakForm(expr, cell, p, precision=prec)
    for mode in ("matrix", "residual"):
        ref = oracle_ref = None
        import oracle as orc_mod
        oracle_ref = orc_mod.einsum_form(mesh, t.einsum[mode], arrays)
        ref = oracle_ref.reshape(mesh.n_cells, -1)
        print(f"[bilinear-new] {expr[0]} {cell}{p} {mode} {prec}", flush=True)
        dt = fe.BilinearPlan(t, cell, p, mode, prec).dtype
        got = wf(X, C, mode=mode, material=None if M is None else _t(M, dt),
                 dofs=_t(U, dt) if mode == "residual" else None)
        wf.check()
        got = got.cpu().numpy().reshape(mesh.n_cells, -1)
        if mode == "matrix":
            assert got.shape[1] == nct * nb * ncu * nb
        assert _err(got, ref) < TOL[prec], mode


def test_stokes_pair_is_a_transpose(orc):
    """The transposed Stokes coupling ('0,i.i', q, u) is the transpose of the
    coupling ('i.i,0', v, p) cell by cell (FP64, bit for bit up to the
    order of the sums)."""
    from paper_2107_04121_amd.transpile import WeakForm
    mesh = _mesh("hex", 2)
    X, C = _t(mesh.coords), _t(mesh.conn)
    B = WeakForm(("i.i,0", "v", "p"), "hex", 2)(X, C, mode="matrix").cpu().numpy()
    Bt = WeakForm(("0,i.i", "q", "u"), "hex", 2)(X, C, mode="matrix").cpu().numpy()
    assert B.shape == (mesh.n_cells, 81, 27) and Bt.shape == (mesh.n_cells, 27, 81)
    assert np.abs(B - np.transpose(Bt, (0, 2, 1))).max() < 1e-13 * np.abs(B).max()
