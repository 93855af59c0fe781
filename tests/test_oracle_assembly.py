"""Pins of the oracle's global matrix assembly against facts of the
assembled operators: the assembled mass matrix of a mesh of the unit cube
sums to its volume 1 and is symmetric positive definite; assembled Laplace
rows sum to zero; the assembled matrix applied to a global DOF vector equals
the element residuals added node by node (np.add.at); the vector mass is
I_3 (x) the scalar one in the (node, component) numbering."""
import numpy as np
import pytest

import meshgen


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("tet", 1), ("tet", 2)])
def test_assembled_mass_and_laplace(orc, cell, p):
    mesh = (meshgen.hex_mesh((3, 2, 2), p, alpha=0.15, seed=70) if cell == "hex"
            else meshgen.tet_mesh((2, 2, 1), p, alpha=0.1, seed=70))
    M = orc.assemble_matrix(mesh, orc.matrix(mesh, "mass"), 1)
    assert abs(M.sum() - 1.0) < 1e-13                    # volume of the unit cube
    assert abs(M - M.T).max() < 1e-15
    assert np.linalg.eigvalsh(M.toarray()).min() > 0
    L = orc.assemble_matrix(mesh, orc.matrix(mesh, "laplace"), 1)
    assert np.abs(L @ np.ones(mesh.n_nodes)).max() < 1e-12
    assert abs(L - L.T).max() < 1e-14


@pytest.mark.parametrize("form,kind", [("laplace", None), ("elasticity", "iso_cell"), ("vmass", None)])
def test_assembled_matrix_times_dofs_is_assembled_residual(orc, form, kind):
    mesh = meshgen.hex_mesh((3, 2, 2), 2, alpha=0.15, seed=71, curved=0.04)
    nc = orc.n_comp(form)
    lm = meshgen.lame_cell(mesh.n_cells, seed=72) if kind else None
    U = meshgen.dofs(mesh.n_nodes, nc, seed=73)
    A = orc.assemble_matrix(mesh, orc.matrix(mesh, form, lm, kind), nc)
    r = orc.residual(mesh, form, U, lm, kind)               # (n_cells, nc, nb)
    R = np.zeros((mesh.n_nodes, nc))
    np.add.at(R, mesh.conn, np.transpose(r, (0, 2, 1)))
    got = A @ U.ravel()
    assert np.abs(got - R.ravel()).max() / np.abs(R).max() < 1e-12


def test_assembled_vector_mass_is_kronecker(orc):
    mesh = meshgen.hex_mesh((2, 2, 2), 1, alpha=0.15, seed=74)
    Ms = orc.assemble_matrix(mesh, orc.matrix(mesh, "mass"), 1).toarray()
    Mv = orc.assemble_matrix(mesh, orc.matrix(mesh, "vmass"), 3).toarray()
    assert np.abs(Mv - np.kron(Ms, np.eye(3))).max() < 1e-15
