"""Orders 4 and 5 on hexahedra (the highest orders of the paper's table of
cell and DOF counts) through the C ABI against the FP64 oracle: residual
and eval by sum factorization in both output layouts, the adjoint of the
elastic energy, and the forms without a kernel at these orders refused at
plan creation.  Meshes span several workgroups with a ragged tail (Q4: two
cells per wave, eight per workgroup; Q5: one per wave, four per workgroup);
the curvature noise is scaled down with the order so that every Jacobian
stays positive."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}
HIGH = [(4, (4, 3, 2), 0.02), (5, (3, 2, 2), 0.01)]


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _mesh(p, dims, curved, seed=40):
    return meshgen.hex_mesh(dims, p, alpha=0.15, seed=seed + p, curved=curved)


def _material(kind, mesh, nq):
    if kind == "iso_cell":
        return meshgen.lame_cell(mesh.n_cells, seed=41)
    if kind == "iso_qp":
        return meshgen.lame_qp(mesh.n_cells, nq, seed=41)
    return None


def elem_rel_err(got, ref):
    n = ref.shape[0]
    g = got.reshape(n, -1).astype(np.float64)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.maximum(np.abs(r).max(1), 1e-300)).max())


FORMS = [("mass", None), ("vmass", None), ("laplace", None),
         ("elasticity", "iso_cell"), ("elasticity", "iso_qp")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", FORMS)
@pytest.mark.parametrize("p,dims,curved", HIGH)
def test_residual_and_eval(orc, p, dims, curved, form, kind, prec):
    import paper_2107_04121_amd as fe
    mesh = _mesh(p, dims, curved)
    nb, nq = orc.sizes("hex", p)
    nc = orc.n_comp(form)
    mat = _material(kind, mesh, nq)
    U = meshgen.dofs(mesh.n_nodes, nc, seed=42)
    ref_r = orc.residual(mesh, form, U, mat, kind)
    ref_e = orc.energy(mesh, form, U, mat, kind)
    X, C = _t(mesh.coords), _t(mesh.conn)
    for mode, layout in (("residual", "cell_major"), ("residual", "cell_minor"), ("eval", "cell_major")):
        plan = fe.Plan("hex", p, form, mode, prec, material=kind, layout=layout)
        print(f"[high] {mode} Q{p} {form}/{kind} {prec} {layout} variant={plan.variant} "
              f"cells={mesh.n_cells}", flush=True)
        assert plan.variant == "sumfact"
        dt = plan.dtype
        out = plan(X, C, material=None if mat is None else _t(mat, dt), dofs=_t(U, dt))
        plan.check()
        got = out.cpu().numpy()
        if mode == "eval":
            err = float(np.abs(got - ref_e).max() / np.abs(ref_e).max())
        else:
            if layout == "cell_minor":
                got = np.moveaxis(got, -1, 0)
            err = elem_rel_err(got, ref_r)
        assert err < TOL[prec], (mode, layout, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p,dims,curved", HIGH)
def test_energy_grad(orc, p, dims, curved, prec):
    import paper_2107_04121_amd as fe
    from paper_2107_04121_amd import _energy_grad
    mesh = _mesh(p, dims, curved, seed=43)
    nb, nq = orc.sizes("hex", p)
    c = meshgen.lame_qp(mesh.n_cells, nq, seed=44)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=45)
    gm_ref, gx_ref = orc.energy_grad(mesh, c, U)
    plan = fe.Plan("hex", p, "elasticity", "eval", prec, material="iso_qp")
    X, C = _t(mesh.coords), _t(mesh.conn)
    inc = fe.Incidence(C, mesh.n_nodes)
    print(f"[high] adjoint Q{p} {prec} cells={mesh.n_cells}", flush=True)
    gm, gx = _energy_grad(plan, inc, X, C, _t(c, plan.dtype), _t(U, plan.dtype), 1.0)
    gm, gx = gm.cpu().numpy(), gx.cpu().numpy()
    em = float(np.abs(gm - gm_ref).max() / np.abs(gm_ref).max())
    ex = float(np.abs(gx - gx_ref).max() / np.abs(gx_ref).max())
    assert em < TOL[prec] and ex < TOL[prec], (em, ex)


@pytest.mark.parametrize("form,kind,mode", [("elasticity", "voigt_qp", "residual"),
                                            ("wdot", "tensor_qp", "residual"),
                                            ("convect", None, "residual")])
def test_forms_without_kernel_refused(form, kind, mode):
    import paper_2107_04121_amd as fe
    for p in (4, 5):
        with pytest.raises(fe.FeError) as ei:
            fe.Plan("hex", p, form, mode, "fp64", material=kind)
        assert ei.value.status == 2  # FE_ERR_UNSUPPORTED
