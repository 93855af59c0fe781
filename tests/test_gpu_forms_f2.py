"""GPU parity of the weighted vector dot product ('ij,i,j', M, v, u) and the
Navier-Stokes convection ('i,i.j,j', v, u, u) against the FP64 oracle, in
matrix, residual and eval modes, through the C ABI, for every cell kind and
order the generic kernels cover, on meshes that span several workgroups and
end in a ragged tail.  The convection matrix is the derivative at the DOFs
passed (eq. fe4).

Gates: FP64 1e-12, FP32 1e-5 of each element's max-norm (eval: of the
largest element value).
"""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
CELLS = [("hex", 1, False), ("hex", 2, True), ("hex", 3, True), ("tet", 1, False), ("tet", 2, False)]


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _mesh(cell, p, curved):
    if cell == "hex":
        dims = {1: (7, 5, 3), 2: (5, 3, 3), 3: (3, 3, 2)}[p]
        return meshgen.hex_mesh(dims, p, alpha=0.15, seed=40 + p, curved=0.04 if curved else 0.0)
    return meshgen.tet_mesh((4, 3, 2), p, alpha=0.15, seed=40 + p)


def _err(got, ref):
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.maximum(np.abs(r).max(1), 1e-300)).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["wdot", "convect"])
@pytest.mark.parametrize("cell,p,curved", CELLS)
def test_forms_f2_parity(orc, cell, p, curved, form, prec):
    import paper_2107_04121_amd as fe
    mesh = _mesh(cell, p, curved)
    nb, nq = orc.sizes(cell, p)
    kind = "tensor_qp" if form == "wdot" else None
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=41) if kind else None
    U = meshgen.dofs(mesh.n_nodes, 3, seed=42)
    X, C = _t(mesh.coords), _t(mesh.conn)
    refs = {"matrix": orc.matrix(mesh, form, M, kind, u=U),
            "residual": orc.residual(mesh, form, U, M, kind),
            "eval": orc.energy(mesh, form, U, M, kind)}
    for mode, ref in refs.items():
        plan = fe.Plan(cell, p, form, mode, prec, material=kind)
        print(f"[f2] {cell}{p} {form} {mode} {prec} variant={plan.variant} cells={mesh.n_cells}", flush=True)
        dt = plan.dtype
        out = plan(X, C, material=None if M is None else _t(M, dt), dofs=_t(U, dt))
        plan.check()
        got = out.cpu().numpy()
        if mode == "eval":
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
        else:
            err = _err(got, ref)
        assert err < TOL[prec], (mode, err)


def test_convect_matrix_times_state_is_twice_residual():
    """K(u) u = 2 r(u) between the GPU matrix and residual kernels (FP64)."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = _mesh("hex", 2, True)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=43)
    X, C, Ud = _t(mesh.coords), _t(mesh.conn), _t(U)
    K = fe.Plan("hex", 2, "convect", "matrix", "fp64")(X, C, dofs=Ud)
    r = fe.Plan("hex", 2, "convect", "residual", "fp64")(X, C, dofs=Ud)
    ue = Ud[C.long()].transpose(1, 2).reshape(mesh.n_cells, -1)
    Ku = torch.bmm(K, ue.unsqueeze(2)).squeeze(2)
    rr = r.reshape(mesh.n_cells, -1)
    assert float(((Ku - 2 * rr).abs().amax(1) / rr.abs().amax(1)).max()) < 1e-12


def test_f2_argument_rules():
    import paper_2107_04121_amd as fe
    with pytest.raises(fe.FeError):
        fe.Plan("hex", 1, "convect", "residual", "fp64", variant="matrix_first")
    with pytest.raises(fe.FeError):
        fe.Plan("hex", 1, "wdot", "matrix", "fp64")              # no TENSOR_QP
    mesh = _mesh("hex", 1, False)
    plan = fe.Plan("hex", 1, "convect", "matrix", "fp64")
    with pytest.raises(fe.FeError):
        plan(_t(mesh.coords), _t(mesh.conn))                     # no state u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["wdot", "convect"])
@pytest.mark.parametrize("p", [2, 3])
def test_forms_f2_matrix_cores_many_cells(orc, p, form, prec):
    """Q2/Q3 matrices of the two forms on the matrix cores, on more cells
    than the persistent grid has workgroups: sampled cells against the
    oracle, every cell against the generic kernel."""
    import torch
    import paper_2107_04121_amd as fe
    dims = {2: (11, 10, 10), 3: (9, 8, 8)}[p]
    mesh = meshgen.hex_mesh(dims, p, alpha=0.15, seed=44 + p, curved=0.04)
    nb, nq = orc.sizes("hex", p)
    kind = "tensor_qp" if form == "wdot" else None
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=45) if kind else None
    U = meshgen.dofs(mesh.n_nodes, 3, seed=46)
    plan = fe.Plan("hex", p, form, "matrix", prec, material=kind)
    print(f"[f2] many cells Q{p} {form} {prec} variant={plan.variant} cells={mesh.n_cells}", flush=True)
    assert plan.variant == "mfma"
    dt = plan.dtype
    X, C, Ud = _t(mesh.coords), _t(mesh.conn), _t(U, dt)
    Md = None if M is None else _t(M, dt)
    K = plan(X, C, material=Md, dofs=Ud)
    plan.check()
    gen = fe.Plan("hex", p, form, "matrix", prec, material=kind, variant="generic")
    Kg = gen(X, C, material=Md, dofs=Ud)
    gen.check()
    assert _err(K.cpu().numpy(), Kg.double().cpu().numpy()) < TOL[prec]
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.choice(mesh.n_cells, 20, replace=False), [0, mesh.n_cells - 1]]))
    sub = meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[idx], cell="hex", order=p, h=mesh.h)
    ref = orc.matrix(sub, form, None if M is None else M[idx], kind, u=U)
    assert _err(K[torch.as_tensor(idx, device=K.device)].cpu().numpy(), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["wdot", "convect"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_forms_f2_residual_sumfact_vs_generic(orc, p, form, prec):
    """Hex residuals and evals of the two forms: the sum-factorized kernel
    (cell-major and cell-minor output) against the generic kernel and the
    oracle."""
    import paper_2107_04121_amd as fe
    mesh = _mesh("hex", p, True)
    nb, nq = orc.sizes("hex", p)
    kind = "tensor_qp" if form == "wdot" else None
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=51) if kind else None
    U = meshgen.dofs(mesh.n_nodes, 3, seed=52)
    X, C = _t(mesh.coords), _t(mesh.conn)
    ref = orc.residual(mesh, form, U, M, kind)
    outs = {}
    for variant, layout in (("auto", "cell_major"), ("auto", "cell_minor"), ("generic", "cell_major")):
        plan = fe.Plan("hex", p, form, "residual", prec, material=kind, variant=variant, layout=layout)
        assert plan.variant == ("sumfact" if variant == "auto" else "generic")
        out = plan(X, C, material=None if M is None else _t(M, plan.dtype), dofs=_t(U, plan.dtype))
        plan.check()
        got = out.cpu().numpy()
        if layout == "cell_minor":
            got = np.moveaxis(got, -1, 0)
        outs[(variant, layout)] = got
        assert _err(got, ref) < TOL[prec], (variant, layout)
    assert np.array_equal(outs[("auto", "cell_major")], outs[("auto", "cell_minor")])
    ev = fe.Plan("hex", p, form, "eval", prec, material=kind)
    assert ev.variant == "sumfact"
    e = ev(X, C, material=None if M is None else _t(M, ev.dtype), dofs=_t(U, ev.dtype)).cpu().numpy()
    ref_e = orc.energy(mesh, form, U, M, kind)
    assert float(np.abs(e - ref_e).max() / np.abs(ref_e).max()) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cell,p,curved", [("hex", 2, True), ("hex", 1, False), ("tet", 2, False)])
def test_wdot_matrix_first_chunked(orc, cell, p, curved, prec):
    """Matrix-first weighted-dot residual in chunks of 7 cells: every chunk
    must read its own per-point 3 x 3 matrices (9 n_qp entries per cell)."""
    import paper_2107_04121_amd as fe
    mesh = _mesh(cell, p, curved)
    nb, nq = orc.sizes(cell, p)
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=43)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=44)
    X, C = _t(mesh.coords), _t(mesh.conn)
    ref = orc.residual(mesh, "wdot", U, M, "tensor_qp")
    plan = fe.Plan(cell, p, "wdot", "residual", prec, material="tensor_qp", variant="matrix_first", chunk=7)
    print(f"[f2 matrix-first] {cell}{p} wdot {prec} cells={mesh.n_cells} chunk=7", flush=True)
    assert mesh.n_cells > 3 * 7
    dt = plan.dtype
    out = plan(X, C, material=_t(M, dt), dofs=_t(U, dt), workspace=plan.workspace(mesh.n_cells, X.device))
    plan.check()
    assert _err(out.cpu().numpy(), ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["wdot", "convect"])
def test_forms_f2_q2_matrix_output_offsets(orc, form, prec):
    """Q2 matrices of the two forms written through an LDS staging area in
    16-byte vectors: an output that starts at any element offset from a
    16-byte boundary (and cells whose matrices start at either parity) gets
    the same values as an aligned one, bit for bit, with nothing written
    outside the matrices."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh((3, 3, 3), 2, alpha=0.15, seed=48, curved=0.04)
    nb, nq = orc.sizes("hex", 2)
    kind = "tensor_qp" if form == "wdot" else None
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=49) if kind else None
    U = meshgen.dofs(mesh.n_nodes, 3, seed=50)
    plan = fe.Plan("hex", 2, form, "matrix", prec, material=kind)
    assert plan.variant == "mfma"
    dt = plan.dtype
    X, C, Ud = _t(mesh.coords), _t(mesh.conn), _t(U, dt)
    Md = None if M is None else _t(M, dt)
    K0 = plan(X, C, material=Md, dofs=Ud)
    plan.check()
    n = K0.numel()
    for off in ((1,) if prec == "fp64" else (1, 2, 3)):
        print(f"[f2] output offset {off} Q2 {form} {prec}", flush=True)
        buf = torch.full((n + off + 4,), 7.0, dtype=dt, device="cuda:0")
        out = buf[off:off + n].view(K0.shape)
        plan(X, C, material=Md, dofs=Ud, out=out)
        plan.check()
        assert torch.equal(out, K0)
        assert bool((buf[:off] == 7.0).all()) and bool((buf[off + n:] == 7.0).all())
