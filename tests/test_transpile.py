"""The notation front-end: parsing and form matching (the table of example
weak forms, with renamed indices and the unsupported rows), the einsum
expressions it emits against the ones the paper prints, and those
expressions evaluated with numpy.einsum (operands from the oracle's
reference tables with numpy's det/inv) against the oracle in every mode.
No GPU: the library's plans are exercised by test_gpu_transpile.py."""
import numpy as np
import pytest

import meshgen
from paper_2107_04121_amd.transpile import STATE_EINSUM, WeakForm, transpile


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
    t = transpile(expr, *args)
    assert t.form == form
    assert t.test == args[1 if t.material else 0]


@pytest.mark.parametrize("expr,args", [
    ("i.i,0", ("v", "p")),            # Stokes coupling: no kernel
    ("i.i", ("v",)),                  # divergence operator
    ("ji,i,j", ("M", "v", "u")),      # M transposed: v_i M_ji u_j
    ("i,j", ("v", "u")),              # not a dot product
    ("i,i.j,j", ("v", "u", "w")),     # advection by another field
])
def test_unsupported_forms_raise(expr, args):
    with pytest.raises(NotImplementedError):
        transpile(expr, *args)


def test_malformed_expressions_raise():
    with pytest.raises(ValueError):
        transpile("0.i,0.i", "v")
    with pytest.raises(ValueError):
        transpile("0.i,0.ii", "v", "u")
    with pytest.raises(ValueError):
        transpile("i,i", "u", "u")
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
    # the convection matrix is a sum of two expressions (eq. fe4)
    assert len(transpile("i,i.j,j", "v", "u", "u").einsum["matrix"]) == 2


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
    if t.form == "convect":
        for name, (ex, names) in STATE_EINSUM.items():
            ops[name] = np.einsum(ex, *[ops[n] for n in names])
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
    from paper_2107_04121_amd.transpile import _N_COMP
    for form, nc in _N_COMP.items():
        assert fe.n_comp(form) == nc, form
