"""GPU parity at the benchmark sizes, in the launch configurations the
benchmark times: outputs on sampled cells (first, last, cells at the XCD
range boundaries of the persistent kernels, and seeded random ones) against
the FP64 oracle computed cell by cell, plus properties that hold for every
cell of the full output (symmetry, zero Laplace row sums, rigid translations
in the elasticity kernel).

Gates as in the other parity tests: FP64 1e-12, FP32 1e-5, BF16X3 1e-4 of
each cell's max-norm.
"""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _sample(n_cells, k=40, seed=7):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(n_cells, size=min(k, n_cells), replace=False).tolist())
    # first / last cells and the boundaries of eight contiguous ranges
    for x in range(9):
        c = min(n_cells - 1, (x * ((n_cells + 7) // 8)))
        idx.update({c, max(0, c - 1)})
    idx.update({0, n_cells - 1})
    return np.array(sorted(idx))


def _sub(mesh, idx):
    return meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[idx], cell=mesh.cell, order=mesh.order, h=mesh.h)


def _err(got, ref):
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.abs(r).max(1)).max())


def test_q1_laplace_16cube_full(orc):
    """Q1 Laplace matrices and residuals on all 4,096 cells (16^3, +-0.2h)."""
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(16, 1, alpha=0.2, seed=0)
    U = meshgen.dofs(mesh.n_nodes, 1, seed=0)
    pm = fe.Plan("hex", 1, "laplace", "matrix", "fp64")
    pr = fe.Plan("hex", 1, "laplace", "residual", "fp64")
    print(f"[fullsize] q1 16^3 {pm.variant}/{pr.variant}", flush=True)
    K = pm(_t(mesh.coords), _t(mesh.conn))
    r = pr(_t(mesh.coords), _t(mesh.conn), dofs=_t(U))
    pm.check()
    pr.check()
    assert _err(K.cpu().numpy(), orc.matrix(mesh, "laplace")) < TOL["fp64"]
    assert _err(r.cpu().numpy(), orc.residual(mesh, "laplace", U)) < TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_q2_elasticity_48cube(orc, prec):
    """Q2 elasticity matrices on 48^3 = 110,592 cells: sampled cells against
    the oracle; every cell symmetric and free of rigid translations."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(48, 2, alpha=0.15, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0)
    plan = fe.Plan("hex", 2, "elasticity", "matrix", prec, material="iso_cell")
    print(f"[fullsize] q2 48^3 {prec} {plan.variant}", flush=True)
    K = plan(_t(mesh.coords), _t(mesh.conn), material=_t(lm, plan.dtype))
    plan.check()
    idx = _sample(mesh.n_cells)
    ref = orc.matrix(_sub(mesh, idx), "elasticity", lm[idx], "iso_cell")
    err = _err(K[_t(idx)].cpu().numpy(), ref)
    print(f"[fullsize] q2 48^3 {prec} sampled err {err:.2e}", flush=True)
    assert err < TOL[prec]
    # whole output: K = K^T and K t = 0 for the three translations t
    scale = K.abs().amax(dim=(1, 2))
    asym = (K - K.transpose(1, 2)).abs().amax(dim=(1, 2)) / scale
    assert float(asym.max()) < 4 * TOL[prec]
    for c in range(3):
        t = torch.zeros(81, dtype=K.dtype, device=K.device)
        t[c * 27:(c + 1) * 27] = 1
        row = (K @ t).abs().amax(dim=1) / scale
        assert float(row.max()) < 50 * TOL[prec], (c, float(row.max()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_q1_laplace_128cube_rowsums(orc, prec):
    """Q1 Laplace matrices on 128^3 cells (the largest point of the c1 sweep):
    every row sums to zero, every matrix is symmetric, and sampled cells
    match the oracle."""
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(128, 1, alpha=0.2, seed=0)
    plan = fe.Plan("hex", 1, "laplace", "matrix", prec)
    K = plan(_t(mesh.coords), _t(mesh.conn))
    plan.check()
    scale = K.abs().amax(dim=(1, 2))
    rows = float((K.sum(dim=2).abs().amax(dim=1) / scale).max())
    assert rows < (1e-13 if prec == "fp64" else 1e-5), rows
    assert float(((K - K.transpose(1, 2)).abs().amax(dim=(1, 2)) / scale).max()) == 0.0
    idx = _sample(mesh.n_cells, 16)
    err = _err(K[_t(idx)].cpu().numpy(), orc.matrix(_sub(mesh, idx), "laplace"))
    print(f"[fullsize] q1 128^3 laplace {prec} sampled err {err:.2e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("form", ["laplace", "elasticity"])
def test_q3_residual_96cube(orc, form):
    """Q3 residuals on 96^3 = 884,736 cells, FP32 with FP64 geometry, both
    output layouts: sampled cells against the oracle."""
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(96, 3, alpha=0.15, seed=0)
    nc = 3 if form == "elasticity" else 1
    U = meshgen.dofs(mesh.n_nodes, nc, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0) if nc == 3 else None
    kind = "iso_cell" if nc == 3 else None
    idx = _sample(mesh.n_cells, 24)
    ref = orc.residual(_sub(mesh, idx), form, U, None if lm is None else lm[idx], kind)
    X, C = _t(mesh.coords), _t(mesh.conn)
    for layout in ("cell_major", "cell_minor"):
        plan = fe.Plan("hex", 3, form, "residual", "fp32", material=kind, layout=layout)
        print(f"[fullsize] q3 96^3 {form} {layout} {plan.variant}", flush=True)
        out = plan(X, C, material=None if lm is None else _t(lm, plan.dtype), dofs=_t(U, plan.dtype))
        plan.check()
        it = _t(idx)
        got = out[it] if layout == "cell_major" else out.movedim(-1, 0)[it]
        err = _err(got.cpu().numpy(), ref)
        print(f"[fullsize] q3 96^3 {form} {layout} sampled err {err:.2e}", flush=True)
        assert err < TOL["fp32"]
        del out


def test_batch_uneven_full_groups(orc):
    """The batched uneven mesh at its full sizes (300k P1, 120k P2 tets, 200k
    Q1, 40k Q2 hex, three forms each, FP32, tuned tiles): sampled cells of
    every group and form against the oracle."""
    import paper_2107_04121_amd as fe
    specs = [("tet", 1, (50, 40, 25)), ("tet", 2, (40, 25, 20)), ("hex", 1, (100, 50, 40)),
             ("hex", 2, (40, 40, 25))]
    ss = np.random.SeedSequence(0).spawn(4)
    meshes, groups = [], []
    for (cell, p, dims), s in zip(specs, ss):
        seed = int(s.generate_state(1)[0])
        m = (meshgen.tet_mesh(dims, p, alpha=0.15, seed=seed) if cell == "tet"
             else meshgen.hex_mesh(dims, p, alpha=0.15, seed=seed))
        lm = meshgen.lame_cell(m.n_cells, seed=seed)
        meshes.append((m, lm))
        groups.append(dict(cell=cell, order=p, coords=_t(m.coords), conn=_t(m.conn),
                           material=_t(lm).float(), forms=("mass", "laplace", "elasticity")))
    b = fe.Batch(groups, precision="fp32", autotune=True)
    print(f"[fullsize] batch tiles {b.tiles}", flush=True)
    b.run()
    b.check()
    for (m, lm), o in zip(meshes, b.outputs):
        idx = _sample(m.n_cells, 16)
        sub = _sub(m, idx)
        it = _t(idx)
        for form, ref in (("mass", orc.matrix(sub, "mass")), ("laplace", orc.matrix(sub, "laplace")),
                          ("elasticity", orc.matrix(sub, "elasticity", lm[idx], "iso_cell"))):
            err = _err(o[form][it].cpu().numpy(), ref)
            print(f"[fullsize] batch {m.cell}{m.order} {form} err {err:.2e}", flush=True)
            assert err < TOL["fp32"], (m.cell, m.order, form, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c5_adjoint_32cube_full(orc, prec):
    """The adjoint workload at its full size: Q2 elasticity energy
    J = sum_e u_e^T K_e u_e on 32^3 cells (vertices +-0.15h, seed 0) with
    per-point (lambda, mu) lognormal(0, 0.5) and u ~ N(0, 1), through the
    autograd wrapper the benchmark times.  J against the oracle's energy, and
    EVERY entry of dJ/dc, dJ/dx and dJ/du against the oracle's gradient and
    twice its assembled residual."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(32, 2, alpha=0.15, seed=0)
    c = meshgen.lame_qp(mesh.n_cells, 27, seed=0)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=0)
    ep = fe.ElasticEnergyPlan("hex", 2, _t(mesh.conn), mesh.n_nodes, prec)
    dt = ep.eval.dtype
    ct = _t(c, dt).requires_grad_(True)
    xt = _t(mesh.coords).requires_grad_(True)
    ut = _t(U, dt).requires_grad_(True)
    print(f"[fullsize] c5 32^3 adjoint {prec} eval={ep.eval.variant}", flush=True)
    J = fe.ElasticEnergy(ct, xt, ut, ep)
    J.backward()
    torch.cuda.synchronize()
    J_ref = orc.energy(mesh, "elasticity", U, c, "iso_qp").sum()
    gm_ref, gx_ref = orc.energy_grad(mesh, c, U)
    r = orc.residual(mesh, "elasticity", U, c, "iso_qp")
    gu_ref = np.zeros_like(U)
    for k in range(3):
        np.add.at(gu_ref[:, k], mesh.conn.ravel(), r[:, k, :].ravel())
    gu_ref *= 2.0

    def rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    errs = dict(J=abs(float(J.detach()) - J_ref) / abs(J_ref),
                dJdc=rel(ct.grad.cpu().numpy(), gm_ref),
                dJdx=rel(xt.grad.cpu().numpy(), gx_ref),
                dJdu=rel(ut.grad.cpu().numpy(), gu_ref))
    print(f"[fullsize] c5 {prec} errors {errs}", flush=True)
    assert max(errs.values()) < TOL[prec], errs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["wdot", "convect"])
def test_q2_forms_f2_32cube(orc, form, prec):
    """Weighted dot and convection matrices of Q2 hexahedra on 32^3 =
    32,768 cells (the matrix-core kernel, persistent over XCD ranges):
    sampled cells against the oracle; for every cell, the weighted dot's
    blocks symmetric, and the convection matrix times the state twice the
    residual of the sum-factorized kernel."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(32, 2, alpha=0.15, seed=0)
    nq = 27
    kind = "tensor_qp" if form == "wdot" else None
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=1) if kind else None
    U = meshgen.dofs(mesh.n_nodes, 3, seed=2)
    plan = fe.Plan("hex", 2, form, "matrix", prec, material=kind)
    print(f"[fullsize] q2 32^3 {form} {prec} {plan.variant}", flush=True)
    assert plan.variant == "mfma"
    dt = plan.dtype
    X, C, Ud = _t(mesh.coords), _t(mesh.conn), _t(U, dt)
    Md = None if M is None else _t(M, dt)
    K = plan(X, C, material=Md, dofs=Ud)
    plan.check()
    idx = _sample(mesh.n_cells)
    ref = orc.matrix(_sub(mesh, idx), form, None if M is None else M[idx], kind, u=U)
    err = _err(K[_t(idx)].cpu().numpy(), ref)
    print(f"[fullsize] q2 32^3 {form} {prec} sampled err {err:.2e}", flush=True)
    assert err < TOL[prec]
    scale = K.abs().amax(dim=(1, 2))
    if form == "wdot":
        Kb = K.reshape(-1, 3, 27, 3, 27)
        asym = (Kb - Kb.transpose(2, 4)).abs().amax(dim=(1, 2, 3, 4)) / scale
        assert float(asym.max()) < 4 * TOL[prec]
    else:
        r = fe.Plan("hex", 2, "convect", "residual", prec)(X, C, dofs=Ud)
        ue = Ud[C.long()].transpose(1, 2).reshape(mesh.n_cells, -1).contiguous()
        Ku = torch.bmm(K, ue.unsqueeze(2)).squeeze(2)
        rr = r.reshape(mesh.n_cells, -1)
        rel = (Ku - 2 * rr).abs().amax(1) / (K.abs().amax(dim=(1, 2)) * ue.abs().amax(1))
        assert float(rel.max()) < 50 * TOL[prec], float(rel.max())
