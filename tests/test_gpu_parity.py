"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle,
element by element, on seeded meshes spanning several workgroup tiles and a
ragged tail, curved and straight, for every cell kind, order, form, mode,
precision and material layout.

Gates (relative to each element's max-norm): FP64 1e-12, FP32 1e-5,
BF16X3 1e-4 (derivation in the design notes: FP32 unit roundoff 6e-8 times
the accumulation length and the conditioning of the element contraction).
"""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def _dev():
    import torch
    return torch.device("cuda:0")


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(_dev())
    return t if dtype is None else t.to(dtype)


def elem_rel_err(got, ref):
    """max over elements of max|got - ref| / max|ref| (per element)."""
    n = ref.shape[0]
    g = got.reshape(n, -1).astype(np.float64)
    r = ref.reshape(n, -1)
    scale = np.maximum(np.abs(r).max(1), 1e-300)
    return float((np.abs(g - r).max(1) / scale).max())


def _mesh(cell, p, curved):
    if cell == "hex":
        dims = {1: (7, 5, 3), 2: (5, 3, 3), 3: (3, 3, 2)}[p]
        return meshgen.hex_mesh(dims, p, alpha=0.15, seed=p,
                                curved=0.04 if curved else 0.0)
    return meshgen.tet_mesh((4, 3, 2), p, alpha=0.15, seed=p)


def _material(kind, mesh, nq):
    if kind is None:
        return None
    if kind == "iso_cell":
        return meshgen.lame_cell(mesh.n_cells, seed=3)
    if kind == "iso_qp":
        return meshgen.lame_qp(mesh.n_cells, nq, seed=3)
    return meshgen.voigt_random_spd((mesh.n_cells, nq), seed=3)


CELLS = [("hex", 1, False), ("hex", 2, True), ("hex", 3, True),
         ("tet", 1, False), ("tet", 2, False)]
FORMS = [("mass", None), ("vmass", None), ("laplace", None),
         ("elasticity", "iso_cell"), ("elasticity", "iso_qp"),
         ("elasticity", "voigt_qp")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", FORMS)
@pytest.mark.parametrize("cell,p,curved", CELLS)
def test_matrix_parity(orc, cell, p, curved, form, kind, prec):
    import paper_2107_04121_amd as fe
    mesh = _mesh(cell, p, curved)
    nb, nq = orc.sizes(cell, p)
    mat = _material(kind, mesh, nq)
    ref = orc.matrix(mesh, form, mat, kind)
    plan = fe.Plan(cell, p, form, "matrix", prec, material=kind)
    print(f"[parity] matrix {cell}{p} {form}/{kind} {prec} "
          f"variant={plan.variant} cells={mesh.n_cells}", flush=True)
    dt = plan.dtype
    out = plan(_t(mesh.coords), _t(mesh.conn),
               material=None if mat is None else _t(mat, dt))
    plan.check()
    err = elem_rel_err(out.cpu().numpy(), ref)
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", FORMS)
@pytest.mark.parametrize("cell,p,curved", CELLS)
def test_residual_and_eval_parity(orc, cell, p, curved, form, kind, prec):
    import paper_2107_04121_amd as fe
    mesh = _mesh(cell, p, curved)
    nb, nq = orc.sizes(cell, p)
    nc = orc.n_comp(form)
    mat = _material(kind, mesh, nq)
    U = meshgen.dofs(mesh.n_nodes, nc, seed=5)
    ref_r = orc.residual(mesh, form, U, mat, kind)
    ref_e = orc.energy(mesh, form, U, mat, kind)
    for mode, ref in (("residual", ref_r), ("eval", ref_e)):
        plan = fe.Plan(cell, p, form, mode, prec, material=kind)
        print(f"[parity] {mode} {cell}{p} {form}/{kind} {prec} "
              f"variant={plan.variant}", flush=True)
        dt = plan.dtype
        out = plan(_t(mesh.coords), _t(mesh.conn),
                   material=None if mat is None else _t(mat, dt),
                   dofs=_t(U, dt))
        plan.check()
        got = out.cpu().numpy()
        if mode == "eval":
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
        else:
            err = elem_rel_err(got, ref)
        assert err < TOL[prec], (mode, err)


def test_empty_and_single_cell(orc):
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(1, 2, alpha=0.0)
    plan = fe.Plan("hex", 2, "laplace", "matrix", "fp64")
    X, C = _t(mesh.coords), _t(mesh.conn)
    out = plan(X, C[:0])
    assert out.shape == (0, 27, 27)
    K = plan(X, C)
    plan.check()
    assert elem_rel_err(K.cpu().numpy(), orc.matrix(mesh, "laplace")) < 1e-12
    torch.cuda.synchronize()


def test_faults_are_reported(orc):
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh((3, 2, 2), 1, alpha=0.1)
    conn = mesh.conn.copy()
    conn[5, [0, 1]] = conn[5, [1, 0]]                  # inverted cell
    plan = fe.Plan("hex", 1, "laplace", "matrix", "fp64")
    plan(_t(mesh.coords), _t(conn))
    with pytest.raises(fe.FeError) as ei:
        plan.check()
    assert ei.value.status == 3
    plan.check()                                       # bits were cleared
    conn = mesh.conn.copy()
    conn[7, 3] = mesh.n_nodes + 5                      # out of range
    plan(_t(mesh.coords), _t(conn))
    with pytest.raises(fe.FeError) as ei:
        plan.check()
    assert ei.value.status == 4


def test_repeatable_bitwise(orc):
    import torch
    import paper_2107_04121_amd as fe
    mesh = _mesh("hex", 2, True)
    lm = meshgen.lame_cell(mesh.n_cells, seed=1)
    plan = fe.Plan("hex", 2, "elasticity", "matrix", "fp64",
                   material="iso_cell")
    a = plan(_t(mesh.coords), _t(mesh.conn), material=_t(lm))
    b = plan(_t(mesh.coords), _t(mesh.conn), material=_t(lm))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["auto", "generic"])
def test_elasticity_q2_variants(orc, prec, variant):
    """Q2 elasticity matrices with per-cell coefficients: the matrix-core
    kernel (auto) and the generic kernel, every precision, on a curved mesh
    whose cell count leaves a ragged tail across the 8 XCD ranges."""
    import paper_2107_04121_amd as fe
    if variant == "generic" and prec == "bf16x3":
        pytest.skip("bf16x3 exists only on the matrix-core path")
    mesh = meshgen.hex_mesh((7, 5, 3), 2, alpha=0.15, seed=11, curved=0.04)
    lm = meshgen.lame_cell(mesh.n_cells, seed=12)
    ref = orc.matrix(mesh, "elasticity", lm, "iso_cell")
    plan = fe.Plan("hex", 2, "elasticity", "matrix", prec,
                   material="iso_cell", variant=variant)
    assert plan.variant == ("mfma" if variant == "auto" else "generic")
    print(f"[parity] q2 elasticity {prec} {plan.variant}", flush=True)
    out = plan(_t(mesh.coords), _t(mesh.conn), material=_t(lm, plan.dtype))
    plan.check()
    err = elem_rel_err(out.cpu().numpy(), ref)
    print(f"[parity] max rel err {err:.3e}", flush=True)
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", [("mass", None), ("vmass", None),
                                       ("laplace", None),
                                       ("elasticity", "iso_cell"),
                                       ("elasticity", "iso_qp"),
                                       ("elasticity", "voigt_qp")])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_variants(orc, p, form, kind, prec):
    """Sum-factorized (auto for hexahedra), generic and matrix-first
    residuals, cell-major and cell-minor outputs, against the oracle."""
    import paper_2107_04121_amd as fe
    mesh = _mesh("hex", p, True)
    nb, nq = orc.sizes("hex", p)
    nc = orc.n_comp(form)
    mat = _material(kind, mesh, nq)
    U = meshgen.dofs(mesh.n_nodes, nc, seed=6)
    ref = orc.residual(mesh, form, U, mat, kind)
    X, C = _t(mesh.coords), _t(mesh.conn)
    for variant, layout, chunk in (("auto", "cell_major", 0),
                                   ("auto", "cell_minor", 0),
                                   ("generic", "cell_major", 0),
                                   ("matrix_first", "cell_major", 7)):
        plan = fe.Plan("hex", p, form, "residual", prec, material=kind,
                       variant=variant, layout=layout, chunk=chunk)
        if variant == "auto":
            assert plan.variant == "sumfact"
        dt = plan.dtype
        out = plan(X, C, material=None if mat is None else _t(mat, dt),
                   dofs=_t(U, dt))
        plan.check()
        got = out.cpu().numpy()
        if layout == "cell_minor":
            got = np.moveaxis(got, -1, 0)
        err = elem_rel_err(got, ref)
        print(f"[parity] residual Q{p} {form}/{kind} {prec} {plan.variant} "
              f"{layout} {err:.2e}", flush=True)
        assert err < TOL[prec], (variant, layout, err)


LOW = [("hex", 1), ("tet", 1), ("tet", 2)]
LOW_FORMS = [("mass", None), ("vmass", None), ("laplace", None),
             ("elasticity", "iso_cell"), ("elasticity", "iso_qp")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", LOW_FORMS)
@pytest.mark.parametrize("cell,p", LOW)
def test_lowo_matrix_cellwise(orc, cell, p, form, kind, prec):
    """Cell-per-lane kernels (the automatic choice for Q1/P1/P2 matrices)
    and the generic kernel, both against the oracle, on meshes of several
    64-cell workgroups with a ragged last one."""
    import paper_2107_04121_amd as fe
    mesh = (meshgen.hex_mesh((9, 8, 7), 1, alpha=0.2, seed=11) if cell == "hex"
            else meshgen.tet_mesh((5, 4, 4), p, alpha=0.15, seed=11))
    nb, nq = orc.sizes(cell, p)
    mat = _material(kind, mesh, nq)
    ref = orc.matrix(mesh, form, mat, kind)
    assert mesh.n_cells % 64 != 0
    for variant in ("auto", "generic"):
        plan = fe.Plan(cell, p, form, "matrix", prec, material=kind,
                       variant=variant)
        assert plan.variant == ("cellwise" if variant == "auto"
                                else "generic")
        print(f"[parity] lowo {cell}{p} {form}/{kind} {prec} "
              f"{plan.variant} cells={mesh.n_cells}", flush=True)
        dt = plan.dtype
        out = plan(_t(mesh.coords), _t(mesh.conn),
                   material=None if mat is None else _t(mat, dt))
        plan.check()
        err = elem_rel_err(out.cpu().numpy(), ref)
        assert err < TOL[prec], (variant, err)
