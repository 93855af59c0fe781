"""The notation front-end: parsing and form matching (the table of example
weak forms, with renamed indices and the unsupported rows), the einsum
expressions it emits against the ones the paper prints, and those
expressions evaluated with numpy.einsum (operands from the oracle's
reference tables with numpy's det/inv) against the oracle in every mode.
No GPU: the library's plans are exercised by test_gpu_transpile.py."""
import numpy as np
import pytest

import meshgen
from paper_2107_04121_amd.transpile import WeakForm, apply_layout, layout_support, transpile


@pytest.mark.parametrize("expr,args,form", [
    ("0,0", ("q", "p"), "mass"),
    ("i,i", ("v", "u"), "vmass"),
    ("k,k", ("v", "u"), "vmass"),
    ("0.i,0.i", ("q", "p"), "laplace"),
    ("0.j,0.j", ("q", "p"), "laplace"),
    ("ij,i,j", ("M", "v", "u"), "wdot"),
    ("ab,a,b", ("M", "v", "u"), "wdot"),
    ("i,i.j,j", ("v", "u", "u"), "convect"),
    ("k,k.l,l", ("v", "u", "u"), "convect"),
    ("IK,s(i:j)->I,s(k:l)->K", ("D", "v", "u"), "elasticity"),
    ("AB,s(a:b)->A,s(c:d)->B", ("D", "v", "u"), "elasticity"),
])
def test_forms_recognised(expr, args, form):
    """The dedicated kernel is chosen from the derived structure (operators,
    component counts, the coupling left by the identity and extractor
    operands), whatever the index letters."""
    t = transpile(expr, *args)
    assert t.form == form
    assert t.structure["kernel"] == form
    assert t.test == args[1 if t.material else 0]


@pytest.mark.parametrize("expr,args,test_op,trial_op", [
    ("i.i,0", ("v", "p"), "div", "value"),      # Stokes coupling
    ("0,i.i", ("q", "u"), "value", "div"),      # transposed Stokes coupling
    ("ji,i,j", ("M", "v", "u"), "value", "value"),  # M transposed: v_i M_ji u_j
    ("i.j,i.j", ("v", "u"), "grad", "grad"),    # vector Laplacian
    ("0.i,i", ("q", "u"), "grad", "value"),
])
def test_other_bilinear_forms_go_to_the_generic_kernel(expr, args, test_op, trial_op):
    t = transpile(expr, *args)
    assert t.form is None and t.structure["kernel"] == "bilinear"
    assert (t.structure["test_op"], t.structure["trial_op"]) == (test_op, trial_op)


def test_stokes_coupling_expressions_and_coupling():
    t = transpile("i.i,0", "v", "p")
    assert t.einsum["matrix"][0][0] == "cq,cqid,ir,qe->crde"
    assert t.einsum["residual"][0][0] == "cq,cqid,ir,qe,ce->crd"
    W0 = t.structure["W0"]                      # rows (r, j), the divergence picks r == j
    assert W0.shape == (9, 1)
    np.testing.assert_array_equal(W0[:, 0], np.eye(3).ravel())


@pytest.mark.parametrize("expr,args", [
    ("i.i", ("v",)),                  # divergence operator: a linear form, no unknown
    ("i,j.i,j", ("v", "u", "u")),    # trilinear, but not the convection
])
def test_forms_without_a_kernel_give_a_reason(expr, args):
    t = transpile(expr, *args)
    assert t.structure.get("kernel") is None and t.reason
    with pytest.raises(NotImplementedError):
        WeakForm((expr,) + args, "hex", 1)


def test_more_than_one_unknown_raises():
    with pytest.raises(NotImplementedError):
        transpile("i,i.j,j", "v", "u", "w")     # advection by another field


def test_malformed_expressions_raise():
    with pytest.raises(ValueError):
        transpile("0.i,0.i", "v")
    with pytest.raises(ValueError):
        transpile("0.i,0.ii", "v", "u")
    with pytest.raises(ValueError):
        transpile("i,i", "u", "u")
    with pytest.raises(ValueError):
        transpile("i,j", "v", "u")              # free indices: not a scalar integrand
    with pytest.raises(ValueError):
        WeakForm(("i,i", "v", "u"), "hex", 1, layout="cqgvd")
    with pytest.raises(ValueError):
        WeakForm(("0.i,0.i", "v", "u"), "hex", 1, material_kind="iso_cell")


def test_emitted_strings_are_the_papers():
    """The matrix-mode expressions the paper prints for the weak Laplacian,
    the vector dot product and linear elasticity."""
    assert transpile("0.i,0.i", "v", "u").einsum["matrix"][0][0] == "cq,cqjd,cqje->cde"
    assert transpile("i,i", "v", "u").einsum["matrix"][0][0] == "cq,qd,ir,qe,is->crdse"
    assert transpile("IK,s(i:j)->I,s(k:l)->K", "D", "v", "u").einsum["matrix"][0][0] == \
        "cq,cqje,rjI,cqIK,cqlf,slK->cresf"
    # and the residual of the vector dot product
    assert transpile("i,i", "v", "u").einsum["residual"][0][0] == "cq,qd,ir,qe,cie->crd"
    # the convection matrix is a sum of two expressions (eq. fe4)
    assert len(transpile("i,i.j,j", "v", "u", "u").einsum["matrix"]) == 2


def test_layout_permutes_data_operands():
    t = transpile("IK,s(i:j)->I,s(k:l)->K", "D", "v", "u")
    (e,), where = apply_layout(t, "matrix", "qcgvd0")
    assert e == "qc,qcje,rjI,qcIK,qclf,slK->cresf" and where == "first"
    (e,), where = apply_layout(t, "residual", "qgvd0c")
    assert e.endswith("->rec") and where == "last"
    assert e.split(",")[1] == "qjec"              # bfg: q, g, d, then c


def test_layout_support_rules():
    t = transpile("ij,i,j", "M", "v", "u")
    assert layout_support(t, "matrix", "cqgvd0")[0]
    assert layout_support(t, "residual", "qgvd0c")[0] is False      # material would be read q-first
    t = transpile("0.i,0.i", "v", "u")
    assert layout_support(t, "residual", "qgvd0c")[0]
    assert layout_support(t, "matrix", "qgvd0c")[0] is False
    assert layout_support(t, "residual", "qcgvd0")[0] is False      # cells neither first nor last
    # every one of the 720 permutations is either run or refused with a reason
    import itertools
    for p in itertools.permutations("cqgvd0"):
        ok, why = layout_support(t, "residual", "".join(p))
        assert ok or why


def test_paths_rank_gradient_first_below_matrix_first():
    """The cheapest path of the residual contracts the DOFs with the
    gradients first (the gradient-first order of the sum-factorized and
    generic kernels); forming the element matrix first costs more."""
    from paper_2107_04121_amd.contraction import path_flops
    t = transpile("0.i,0.i", "v", "u")
    sizes = dict(c=1, q=27, j=3, d=27, e=27)
    (best,) = t.paths_for("residual", sizes)
    expr = t.einsum["residual"][0][0]
    # matrix first: det with both gradients, then the DOFs
    mf = path_flops(expr, sizes, [(0, 1), (0, 1), (0, 1)])
    assert best.flops < mf.flops
    first = best.steps[0]
    assert "ce" in first[:2] and "cqje" in first[:2]


def _psg():
    P = np.zeros((3, 3, 6))
    for I, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        P[i, j, I] = 1.0
        P[j, i, I] = 1.0
    return P


def _operands(orc, mesh, U, mats):
    w, _, bf, bfg_ref = orc.tables(mesh.cell, mesh.order)
    X = mesh.coords[mesh.conn]
    J = np.einsum("cdi,qjd->cqij", X, bfg_ref)
    det = np.linalg.det(J) * w[None, :]
    Ji = np.linalg.inv(J)
    bfg = np.einsum("qjd,cqji->cqid", bfg_ref, Ji)
    ops = dict(det=det, bf=bf, bfg=bfg, I=np.eye(3), Psg=_psg(), **mats)
    return ops


def _evaluate(t, mode, ops):
    total = 0.0
    for expr, names in t.einsum[mode]:
        total = total + np.einsum(expr, *[ops[n] for n in names], optimize=True)
    return total


CASES = [
    ("0,0", ("v", "u"), None),
    ("i,i", ("v", "u"), None),
    ("0.i,0.i", ("v", "u"), None),
    ("ij,i,j", ("M", "v", "u"), "tensor_qp"),
    ("i,i.j,j", ("v", "u", "u"), None),
    ("IK,s(i:j)->I,s(k:l)->K", ("D", "v", "u"), "voigt_qp"),
]


@pytest.mark.parametrize("expr,args,kind", CASES)
@pytest.mark.parametrize("mode", ["matrix", "residual", "eval"])
def test_emitted_einsum_matches_oracle(orc, expr, args, kind, mode):
    t = transpile(expr, *args)
    mesh = meshgen.hex_mesh(2, 2, alpha=0.15, seed=50, curved=0.04)
    nb, nq = orc.sizes("hex", 2)
    nc = t.n_comp
    U = meshgen.dofs(mesh.n_nodes, nc, seed=51)
    mats = {}
    if kind == "tensor_qp":
        mats["M"] = meshgen.tensor_qp(mesh.n_cells, nq, seed=52)
    elif kind == "voigt_qp":
        mats["D"] = meshgen.voigt_random_spd((mesh.n_cells, nq), seed=52)
    ops = _operands(orc, mesh, U, mats)
    ue = U[mesh.conn]                              # (c, d, nc)
    ops["dofs"] = ue[:, :, 0] if nc == 1 else np.transpose(ue, (0, 2, 1))
    mat = mats.get("M", mats.get("D"))
    got = _evaluate(t, mode, ops)
    if mode == "matrix":
        ref = orc.matrix(mesh, t.form, mat, kind, u=U if t.form == "convect" else None)
    elif mode == "residual":
        ref = orc.residual(mesh, t.form, U, mat, kind)
    else:
        ref = orc.energy(mesh, t.form, U, mat, kind)
    got = np.asarray(got).reshape(ref.shape)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12


def test_component_counts_agree():
    """The package's n_comp and the front-end's component count agree for
    every form (mass and Laplace scalar, the rest vector)."""
    import paper_2107_04121_amd as fe
    for expr, args, _ in CASES:
        t = transpile(expr, *args)
        assert fe.n_comp(t.form) == t.n_comp, t.form
