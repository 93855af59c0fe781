"""Pins of the oracle's element matrices and residuals (CPU only).

Each check compares the oracle against something it does not compute itself:
closed forms from exact rational 1-D integrals, affine-map identities, numpy
einsum of the contraction strings the paper prints, and invariants the
mathematics fixes (symmetry, zero row sums, volume, rigid-body modes,
translation/rotation/scaling behaviour, path equivalence).
"""
import os

import numpy as np
import pytest

import meshgen
from _exact import (box_grad_products, elasticity_from_S, laplace_from_S,
                    mapped_grad_products, tet_reference)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _single(cell, p, nodes):
    n = nodes.shape[0]
    return meshgen.Mesh(coords=np.ascontiguousarray(nodes, float),
                        conn=np.arange(n, dtype=np.int32)[None, :],
                        cell=cell, order=p, h=np.ones(3))


def _hex_ref_nodes(p):
    n = p + 1
    t = np.arange(n) / p
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    return np.stack([t[i.ravel()], t[j.ravel()], t[k.ravel()]], axis=1)


def _tet_ref_nodes(p):
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    if p == 1:
        return V
    E = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
    return np.concatenate([V, [(V[a] + V[b]) / 2 for a, b in E]])


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------------------ closed forms --

def test_q1_unit_cube_closed_form(orc):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "q1_unit_cube.txt"))
            if ln.strip() and not ln.startswith("#")]
    from fractions import Fraction
    lap = {int(r[0]): float(Fraction(r[1])) for r in rows}
    mas = {int(r[0]): float(Fraction(r[2])) for r in rows}
    for h in (1.0, 0.25):
        m = meshgen.hex_mesh(1, 1, box=(h, h, h))
        K = orc.matrix(m, "laplace")[0]
        M = orc.matrix(m, "mass")[0]
        for a in range(8):
            for b in range(8):
                k = bin(a ^ b).count("1")
                assert abs(K[a, b] - lap[k] * h) < 1e-15
                assert abs(M[a, b] - mas[k] * h ** 3) < 1e-16


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_box_tensor_product(orc, p):
    h = (0.7, 1.3, 0.4)
    m = meshgen.hex_mesh(1, p, box=h)
    S, mass = box_grad_products(p, h)
    assert _rel(orc.matrix(m, "laplace")[0], laplace_from_S(S)) < 1e-13
    assert _rel(orc.matrix(m, "mass")[0], mass) < 1e-13
    lm = np.array([[1.7, 0.6]])
    Kel = orc.matrix(m, "elasticity", lm, "iso_cell")[0]
    assert _rel(Kel, elasticity_from_S(S, 1.7, 0.6)) < 1e-13
    Mv = orc.matrix(m, "vmass")[0]
    assert _rel(Mv, np.kron(np.eye(3), mass)) < 1e-13


def _rand_affine(seed):
    rng = np.random.default_rng(seed)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    return A, rng.standard_normal(3)


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("hex", 3),
                                    ("hex", 4), ("hex", 5), ("tet", 1),
                                    ("tet", 2)])
def test_affine_element(orc, cell, p):
    """x = A xi + b: matrices follow from the exact reference integrals."""
    A, b = _rand_affine(7 + p)
    if cell == "hex":
        S_ref, mass_ref = box_grad_products(p)
        nodes = _hex_ref_nodes(p)
    else:
        S_ref, mass_ref = tet_reference(p)
        nodes = _tet_ref_nodes(p)
    m = _single(cell, p, nodes @ A.T + b)
    S = mapped_grad_products(S_ref, A)
    dA = np.linalg.det(A)
    assert _rel(orc.matrix(m, "laplace")[0], laplace_from_S(S)) < 1e-12
    assert _rel(orc.matrix(m, "mass")[0], dA * mass_ref) < 1e-12
    lm = np.array([[0.8, 1.9]])
    assert _rel(orc.matrix(m, "elasticity", lm, "iso_cell")[0],
                elasticity_from_S(S, 0.8, 1.9)) < 1e-12


# ------------------------------------------------ paper contraction strings --

def _operands(orc, mesh):
    """det (c,q) and bfg (c,q,3,d) built with numpy's det/inv from the
    oracle's reference tables."""
    w, _, bf, bfg_ref = orc.tables(mesh.cell, mesh.order)
    X = mesh.coords[mesh.conn]                     # (c, d, 3)
    J = np.einsum("cdi,qjd->cqij", X, bfg_ref)     # dx_i/dxi_j
    det = np.linalg.det(J) * w[None, :]
    Ji = np.linalg.inv(J)                          # (c,q,j,i) = dxi_j/dx_i
    bfg = np.einsum("qjd,cqji->cqid", bfg_ref, Ji)
    return det, bf, bfg


def _psg():
    P = np.zeros((3, 3, 6))
    for I, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2),
                                (1, 2)]):
        P[i, j, I] = 1.0
        P[j, i, I] = 1.0
    return P


@pytest.mark.parametrize("p", [1, 2])
def test_paper_einsum_strings(orc, p):
    mesh = meshgen.hex_mesh(2, p, alpha=0.2, seed=3, curved=0.05)
    det, bf, bfg = _operands(orc, mesh)
    c, nb = mesh.n_cells, mesh.n_basis
    # weak Laplacian, matrix mode
    K = np.einsum("cq,cqjd,cqje->cde", det, bfg, bfg)
    assert _rel(orc.matrix(mesh, "laplace"), K) < 1e-12
    # vector dot product, matrix and residual modes
    I3 = np.eye(3)
    Mv = np.einsum("cq,qd,ir,qe,is->crdse", det, bf, I3, bf, I3)
    assert _rel(orc.matrix(mesh, "vmass"), Mv.reshape(c, 3 * nb, 3 * nb)) \
        < 1e-12
    U = meshgen.dofs(mesh.n_nodes, 3, seed=1)
    dofs = np.transpose(U[mesh.conn], (0, 2, 1))   # (c, i, e)
    rv = np.einsum("cq,qd,ir,qe,cie->crd", det, bf, I3, bf, dofs)
    assert _rel(orc.residual(mesh, "vmass", U), rv) < 1e-12
    # linear elasticity with a general per-qp Voigt D, matrix mode
    D = meshgen.voigt_random_spd((c, det.shape[1]), seed=5)
    Psg = _psg()
    Ke = np.einsum("cq,cqje,rjI,cqIK,cqlf,slK->cresf", det, bfg, Psg, D,
                   bfg, Psg, optimize=True)
    got = orc.matrix(mesh, "elasticity", D, "voigt_qp")
    assert _rel(got, Ke.reshape(c, 3 * nb, 3 * nb)) < 1e-12


def test_isotropic_voigt_equivalence(orc):
    mesh = meshgen.hex_mesh(2, 2, alpha=0.15, seed=1, curved=0.05)
    nq = orc.sizes("hex", 2)[1]
    lm = meshgen.lame_cell(mesh.n_cells, seed=2)
    lmq = np.repeat(lm[:, None, :], nq, axis=1)
    Kc = orc.matrix(mesh, "elasticity", lm, "iso_cell")
    Kq = orc.matrix(mesh, "elasticity", lmq, "iso_qp")
    Kv = orc.matrix(mesh, "elasticity", meshgen.voigt_iso(lmq), "voigt_qp")
    assert _rel(Kq, Kc) < 1e-14
    assert _rel(Kv, Kc) < 1e-13


# -------------------------------------------------------------- invariants --

CURVED = [("hex", 1, dict(alpha=0.2)), ("hex", 2, dict(alpha=0.15,
                                                       curved=0.05)),
          ("hex", 3, dict(alpha=0.15, curved=0.05)),
          ("hex", 3, dict(alpha=0.15)), ("tet", 1, dict(alpha=0.15)), ("tet", 2, dict(alpha=0.15))]


def _mesh(cell, p, n, kw, seed=0):
    if cell == "hex":
        return meshgen.hex_mesh(n, p, seed=seed, **kw)
    return meshgen.tet_mesh(n, p, seed=seed, **kw)


def _rigid_modes(X):
    """(6, 3, nb) component-major rigid-body displacement fields at nodes."""
    nb = X.shape[0]
    modes = []
    for r in range(3):
        u = np.zeros((3, nb))
        u[r] = 1.0
        modes.append(u)
    for w in np.eye(3):
        modes.append(np.cross(w, X).T)
    return np.array(modes)


@pytest.mark.parametrize("cell,p,kw", CURVED)
def test_invariants(orc, cell, p, kw):
    mesh = _mesh(cell, p, 3 if p < 3 else 2, kw)
    K = orc.matrix(mesh, "laplace")
    M = orc.matrix(mesh, "mass")
    lm = meshgen.lame_cell(mesh.n_cells, seed=4)
    E = orc.matrix(mesh, "elasticity", lm, "iso_cell")
    for A in (K, M, E):
        assert _rel(A, np.swapaxes(A, 1, 2)) < 1e-13
    # Laplace annihilates constants
    assert np.abs(K.sum(2)).max() < 1e-12 * np.abs(K).max()
    # total mass = volume of the unit cube (exact whenever the rule integrates
    # det J exactly: trilinear/affine geometry, Q2 with 3-point Gauss)
    # (a curved Q3 map has det J of degree 8 per variable, beyond the 4-point
    # rule, so only the quadrature error bound applies there)
    curved_q3 = (cell, p) == ("hex", 3) and kw.get("curved", 0) > 0
    assert abs(M.sum() - 1.0) < (1e-3 if curved_q3 else 1e-13)
    assert np.all(M.sum((1, 2)) > 0)
    # rigid-body modes in the elasticity null space; PSD with rank 3nb-6
    nb = mesh.n_basis
    for e in range(0, mesh.n_cells, max(1, mesh.n_cells // 5)):
        X = mesh.coords[mesh.conn[e]]
        R = _rigid_modes(X).reshape(6, 3 * nb)
        assert np.abs(E[e] @ R.T).max() < 1e-11 * np.abs(E[e]).max()
        ev = np.linalg.eigvalsh(E[e])
        assert ev[0] > -1e-12 * ev[-1]
        assert np.sum(ev > 1e-9 * ev[-1]) == 3 * nb - 6
        evl = np.linalg.eigvalsh(K[e])
        assert np.sum(evl > 1e-9 * evl[-1]) == nb - 1


@pytest.mark.parametrize("cell,p,kw", CURVED[:4])
def test_rigid_motions_and_scaling(orc, cell, p, kw):
    mesh = _mesh(cell, p, 2, kw, seed=5)
    lm = meshgen.lame_cell(mesh.n_cells, seed=6)
    K = orc.matrix(mesh, "laplace")
    M = orc.matrix(mesh, "mass")
    E = orc.matrix(mesh, "elasticity", lm, "iso_cell")
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    s = 1.7
    moved = meshgen.Mesh(coords=s * mesh.coords @ Q.T + np.array([3., -1, 2]),
                         conn=mesh.conn, cell=cell, order=p, h=mesh.h)
    K2 = orc.matrix(moved, "laplace")
    M2 = orc.matrix(moved, "mass")
    E2 = orc.matrix(moved, "elasticity", lm, "iso_cell")
    assert _rel(K2, s * K) < 1e-12
    assert _rel(M2, s ** 3 * M) < 1e-12
    nb = mesh.n_basis
    R = np.kron(Q, np.eye(nb))           # component-major rotation
    assert _rel(E2, s * np.einsum("ij,cjk,lk->cil", R, E, R)) < 1e-12


@pytest.mark.parametrize("form", ["mass", "vmass", "laplace", "elasticity"])
@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("hex", 3),
                                    ("tet", 2)])
def test_residual_paths_and_energy(orc, form, cell, p):
    kw = dict(alpha=0.15, curved=0.04) if cell == "hex" else dict(alpha=0.15)
    mesh = _mesh(cell, p, 2, kw, seed=8)
    nc = orc.n_comp(form)
    U = meshgen.dofs(mesh.n_nodes, nc, seed=9)
    mat, kind = None, None
    if form == "elasticity":
        mat, kind = meshgen.lame_cell(mesh.n_cells, seed=10), "iso_cell"
    r_gf = orc.residual(mesh, form, U, mat, kind)
    r_mf = orc.residual(mesh, form, U, mat, kind, path="matrix_first")
    K = orc.matrix(mesh, form, mat, kind)
    ue = np.transpose(U[mesh.conn], (0, 2, 1)).reshape(mesh.n_cells, -1)
    r_k = np.einsum("cij,cj->ci", K, ue).reshape(r_gf.shape)
    assert _rel(r_gf, r_k) < 1e-13
    assert _rel(r_mf, r_k) < 1e-14
    E = orc.energy(mesh, form, U, mat, kind)
    assert _rel(E, np.einsum("ci,ci->c", ue, r_k.reshape(ue.shape))) < 1e-13


def test_patch_test_linear_field(orc):
    """Assembled Laplace residual of a linear field vanishes at interior
    nodes (trilinear geometry, exact 2-point rule)."""
    mesh = meshgen.hex_mesh(4, 1, alpha=0.2, seed=2)
    U = mesh.coords @ np.array([0.3, -1.2, 2.0]) + 0.5
    r = orc.residual(mesh, "laplace", U)[:, 0, :]
    g = np.zeros(mesh.n_nodes)
    np.add.at(g, mesh.conn.ravel(), r.ravel())
    X = mesh.coords
    inner = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert inner.sum() == 27
    assert np.abs(g[inner]).max() < 1e-13


def test_error_paths(orc):
    m = meshgen.hex_mesh(2, 1)
    bad = meshgen.Mesh(coords=m.coords, conn=m.conn.copy(), cell="hex",
                       order=1, h=m.h)
    bad.conn[3, [0, 1]] = bad.conn[3, [1, 0]]     # mirrored cell
    with pytest.raises(orc.OracleError) as ei:
        orc.matrix(bad, "laplace")
    assert ei.value.code == -2
    bad2 = meshgen.Mesh(coords=m.coords, conn=m.conn.copy(), cell="hex",
                        order=1, h=m.h)
    bad2.conn[1, 2] = m.n_nodes
    with pytest.raises(orc.OracleError) as ei:
        orc.matrix(bad2, "mass")
    assert ei.value.code == -3
    with pytest.raises(orc.OracleError):
        orc.matrix(m, "elasticity")              # no material
