"""Pins of the oracle's weighted vector dot product ('ij,i,j', M, v, u) and
Navier-Stokes convection ('i,i.j,j', v, u, u) forms (table of example weak
forms; eqs. fe2-fe4), against facts fixed by the mathematics rather than by
the oracle's own loops:

* closed-form integrals on the unit cube (the Gauss rule is exact for them);
* the weighted dot with a constant M is M (x) the scalar mass matrix, whose
  entries are pinned elsewhere (volumes, reference-cube closed forms);
* u = A x lies in the isoparametric space, so (u.grad)u = A A x and the
  convection residual equals the vector mass matrix times the nodal values of
  A A x, for straight and curved cells;
* the convection residual is quadratic in u, so its central difference in any
  direction equals the matrix (its derivative, eq. fe4) times that direction
  exactly, for any step; K(u) u = 2 r(u);
* a constant field has no convection.
"""
import numpy as np
import pytest

import meshgen
import oracle as orc

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _unit_cube():
    m = meshgen.hex_mesh(1, 1, alpha=0.0, seed=0)
    assert np.allclose(m.coords.min(0), 0) and np.allclose(m.coords.max(0), 1)
    return m


def _field(mesh, fn):
    """(n_nodes, 3) nodal values of a vector field given as fn(x, y, z)."""
    x, y, z = mesh.coords.T
    return np.stack(fn(x, y, z), axis=1)


@pytest.mark.parametrize("fn,val", [
    (lambda x, y, z: (x, 0 * x, 0 * x), 1.0 / 3.0),        # int x^2
    (lambda x, y, z: (x, y, 0 * x), 2.0 / 3.0),            # int x^2 + y^2
    (lambda x, y, z: (y, x, 0 * x), 0.5),                  # int 2xy
    (lambda x, y, z: (0 * x + 1, 0 * x, 0 * x), 0.0),      # constant field
    (lambda x, y, z: (y, 0 * x, 0 * x), 0.0),              # u_j d_j u_0 = 0
])
def test_convect_eval_closed_forms(fn, val):
    m = _unit_cube()
    U = _field(m, fn)
    e = orc.energy(m, "convect", U)
    assert abs(e.sum() - val) < 1e-14


def test_wdot_constant_field_closed_form():
    """u = c constant, M constant: int c^T M c = vol c^T M c (vol = 1)."""
    m = _unit_cube()
    nb, nq = orc.sizes("hex", 1)
    M3 = np.array([[2.0, 0.5, -0.3], [0.1, 1.0, 0.4], [0.7, -0.2, 3.0]])
    M = np.broadcast_to(M3, (m.n_cells, nq, 3, 3)).copy()
    c = np.array([0.3, -1.2, 0.8])
    U = np.broadcast_to(c, (m.n_nodes, 3)).copy()
    e = orc.energy(m, "wdot", U, M, "tensor_qp")
    assert abs(e.sum() - c @ M3 @ c) < 1e-14
    # a linear field: u = (x, 0, 0), M = e0 e0^T: int x^2 = 1/3
    M[...] = 0.0
    M[..., 0, 0] = 1.0
    U = _field(m, lambda x, y, z: (x, 0 * x, 0 * x))
    assert abs(orc.energy(m, "wdot", U, M, "tensor_qp").sum() - 1 / 3) < 1e-14


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("tet", 2)])
def test_wdot_constant_M_is_kronecker_of_mass(cell, p):
    mesh = (meshgen.hex_mesh((2, 2, 1), p, alpha=0.15, seed=3, curved=0.04) if cell == "hex"
            else meshgen.tet_mesh((2, 1, 1), p, alpha=0.1, seed=3))
    nb, nq = orc.sizes(cell, p)
    rng = np.random.default_rng(4)
    M3 = rng.standard_normal((mesh.n_cells, 3, 3)) + 2 * np.eye(3)
    M = np.repeat(M3[:, None], nq, axis=1)
    K = orc.matrix(mesh, "wdot", M, "tensor_qp")
    Ms = orc.matrix(mesh, "mass")
    ref = np.stack([np.kron(M3[e], Ms[e]) for e in range(mesh.n_cells)])
    assert np.abs(K - ref).max() / np.abs(ref).max() < 1e-14
    # identity M gives the vector mass matrix
    I = np.broadcast_to(np.eye(3), (mesh.n_cells, nq, 3, 3)).copy()
    assert np.array_equal(orc.matrix(mesh, "wdot", I, "tensor_qp"), orc.matrix(mesh, "vmass"))


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 3), ("tet", 1)])
def test_wdot_residual_energy_consistent_with_matrix(cell, p):
    """Per-point M (not symmetric): r = K u and energy = u . K u, the
    gradient-first loop against the matrix loop."""
    mesh = (meshgen.hex_mesh((2, 1, 1), p, alpha=0.15, seed=5, curved=0.04) if cell == "hex"
            else meshgen.tet_mesh((2, 1, 1), p, alpha=0.1, seed=5))
    nb, nq = orc.sizes(cell, p)
    M = meshgen.tensor_qp(mesh.n_cells, nq, seed=6)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=7)
    K = orc.matrix(mesh, "wdot", M, "tensor_qp")
    ue = U[mesh.conn].transpose(0, 2, 1).reshape(mesh.n_cells, -1)
    r = orc.residual(mesh, "wdot", U, M, "tensor_qp").reshape(mesh.n_cells, -1)
    ref = np.einsum("eij,ej->ei", K, ue)
    assert np.abs(r - ref).max() / np.abs(ref).max() < 1e-13
    e = orc.energy(mesh, "wdot", U, M, "tensor_qp")
    assert np.abs(e - np.einsum("ei,ei->e", ue, ref)).max() / np.abs(e).max() < 1e-13


@pytest.mark.parametrize("cell,p,curved", [("hex", 1, 0.0), ("hex", 2, 0.05), ("hex", 3, 0.04),
                                           ("tet", 1, 0.0), ("tet", 2, 0.0)])
def test_convect_linear_field_identity(cell, p, curved):
    """u = A x: r_(i,a) = sum_b Mscalar_ab (A A x_b)_i."""
    mesh = (meshgen.hex_mesh((2, 2, 1), p, alpha=0.15, seed=8, curved=curved) if cell == "hex"
            else meshgen.tet_mesh((2, 1, 1), p, alpha=0.1, seed=8))
    A = np.array([[0.3, -1.1, 0.4], [0.8, 0.2, -0.5], [-0.6, 0.9, 0.1]])
    U = mesh.coords @ A.T
    W = mesh.coords @ (A @ A).T               # nodal values of A A x
    r = orc.residual(mesh, "convect", U)       # (n_cells, 3, nb)
    Ms = orc.matrix(mesh, "mass")
    ref = np.einsum("eab,ebi->eia", Ms, W[mesh.conn])
    assert np.abs(r - ref).max() / np.abs(ref).max() < 1e-12


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("tet", 2)])
def test_convect_matrix_is_exact_derivative(cell, p):
    mesh = (meshgen.hex_mesh((2, 1, 1), p, alpha=0.15, seed=9, curved=0.04) if cell == "hex"
            else meshgen.tet_mesh((2, 1, 1), p, alpha=0.1, seed=9))
    U = meshgen.dofs(mesh.n_nodes, 3, seed=10)
    D = meshgen.dofs(mesh.n_nodes, 3, seed=11)
    K = orc.matrix(mesh, "convect", u=U)
    de = D[mesh.conn].transpose(0, 2, 1).reshape(mesh.n_cells, -1)
    ue = U[mesh.conn].transpose(0, 2, 1).reshape(mesh.n_cells, -1)
    Kd = np.einsum("eij,ej->ei", K, de)
    for h in (1.0, 0.25):
        rp = orc.residual(mesh, "convect", U + h * D).reshape(mesh.n_cells, -1)
        rm = orc.residual(mesh, "convect", U - h * D).reshape(mesh.n_cells, -1)
        fd = (rp - rm) / (2 * h)
        assert np.abs(fd - Kd).max() / np.abs(Kd).max() < 1e-12, h
    # homogeneity of degree 2: K(u) u = 2 r(u); eval = u . r
    r = orc.residual(mesh, "convect", U).reshape(mesh.n_cells, -1)
    Ku = np.einsum("eij,ej->ei", K, ue)
    assert np.abs(Ku - 2 * r).max() / np.abs(r).max() < 1e-12
    e = orc.energy(mesh, "convect", U)
    assert np.abs(e - np.einsum("ei,ei->e", ue, r)).max() / np.abs(e).max() < 1e-12


def test_convect_constant_field_has_no_residual():
    mesh = meshgen.hex_mesh((2, 2, 2), 2, alpha=0.15, seed=12, curved=0.04)
    U = np.broadcast_to(np.array([0.4, -1.3, 0.7]), (mesh.n_nodes, 3)).copy()
    r = orc.residual(mesh, "convect", U)
    assert np.abs(r).max() < 1e-13
    assert np.abs(orc.energy(mesh, "convect", U)).max() < 1e-13
