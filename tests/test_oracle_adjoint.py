"""Pins of the oracle's eval-mode value and its gradients (CPU only).

J(c, x) = sum_e u_e^T K_e(c, x) u_e for linear elasticity with per-quadrature
point coefficients c = (lambda, mu).  Checked against: homogeneity (J is
linear in c and of degree 1 under scaling of x), translation invariance,
central finite differences in FP64 along seeded directions, and element-local
per-entry finite differences.
"""
import numpy as np
import pytest

import meshgen


def _setup(orc, n=2, p=2, seed=0):
    mesh = meshgen.hex_mesh(n, p, alpha=0.15, seed=seed, curved=0.04)
    nq = orc.sizes("hex", p)[1]
    c = meshgen.lame_qp(mesh.n_cells, nq, seed=seed)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=seed)
    return mesh, c, U


def _J(orc, mesh, c, U):
    return orc.energy(mesh, "elasticity", U, c, "iso_qp").sum()


def _moved(mesh, coords):
    return meshgen.Mesh(coords=coords, conn=mesh.conn, cell=mesh.cell,
                        order=mesh.order, h=mesh.h)


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("tet", 2)])
def test_homogeneity_and_translation(orc, cell, p):
    if cell == "hex":
        mesh = meshgen.hex_mesh(2, p, alpha=0.15, seed=1, curved=0.04)
    else:
        mesh = meshgen.tet_mesh(2, p, alpha=0.15, seed=1)
    nq = orc.sizes(cell, p)[1]
    c = meshgen.lame_qp(mesh.n_cells, nq, seed=1)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=1)
    J = _J(orc, mesh, c, U)
    gc, gx = orc.energy_grad(mesh, c, U)
    assert abs((gc * c).sum() - J) < 1e-13 * abs(J)          # linear in c
    assert abs((gx * mesh.coords).sum() - J) < 1e-12 * abs(J)  # degree 1 in x
    assert np.abs(gx.sum(0)).max() < 1e-12 * np.abs(gx).max()  # translation


def test_energy_matches_quadratic_form(orc):
    mesh, c, U = _setup(orc)
    K = orc.matrix(mesh, "elasticity", c, "iso_qp")
    ue = np.transpose(U[mesh.conn], (0, 2, 1)).reshape(mesh.n_cells, -1)
    E = orc.energy(mesh, "elasticity", U, c, "iso_qp")
    np.testing.assert_allclose(E, np.einsum("ci,cij,cj->c", ue, K, ue),
                               rtol=1e-13)


def test_dJ_dc_finite_difference(orc):
    mesh, c, U = _setup(orc, seed=2)
    gc, _ = orc.energy_grad(mesh, c, U, want_coords=False)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(c.shape)
        fd = (_J(orc, mesh, c + h * d, U) - _J(orc, mesh, c - h * d, U)) / (
            2 * h)
        assert abs(fd - (gc * d).sum()) < 1e-8 * abs(fd)


def test_dJ_dx_directional_fd(orc):
    mesh, c, U = _setup(orc, seed=4)
    _, gx = orc.energy_grad(mesh, c, U, want_mat=False)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(mesh.coords.shape) * mesh.h.min()
        Jp = _J(orc, _moved(mesh, mesh.coords + h * d), c, U)
        Jm = _J(orc, _moved(mesh, mesh.coords - h * d), c, U)
        fd = (Jp - Jm) / (2 * h)
        an = (gx * d).sum()
        assert abs(fd - an) < 1e-7 * (abs(an) + np.abs(gx * d).sum() * 1e-3)


def test_dJ_dx_elementwise_fd(orc):
    """Per-entry FD of a single element's energy (a global per-entry FD would
    lose digits to cancellation across the sum)."""
    mesh, c, U = _setup(orc, seed=6)
    e = 3
    one = meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[e:e + 1].copy(),
                       cell="hex", order=2, h=mesh.h)
    ce = c[e:e + 1]
    _, gx = orc.energy_grad(one, ce, U, want_mat=False)
    h = 1e-6
    rng = np.random.default_rng(7)
    for a in rng.choice(27, size=6, replace=False):
        n = one.conn[0, a]
        for k in range(3):
            X = mesh.coords.copy()
            X[n, k] += h
            Jp = _J(orc, _moved(one, X), ce, U)
            X[n, k] -= 2 * h
            Jm = _J(orc, _moved(one, X), ce, U)
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - gx[n, k]) < 1e-7 * max(1.0, np.abs(gx).max())


def test_dJ_du_is_twice_assembled_residual(orc):
    mesh, c, U = _setup(orc, seed=8)
    r = orc.residual(mesh, "elasticity", U, c, "iso_qp")     # (c, 3, nb)
    g = np.zeros_like(U)
    for comp in range(3):
        np.add.at(g[:, comp], mesh.conn.ravel(), r[:, comp, :].ravel())
    d = np.random.default_rng(9).standard_normal(U.shape)
    h = 1e-6
    fd = (_J(orc, mesh, c, U + h * d) - _J(orc, mesh, c, U - h * d)) / (2 * h)
    assert abs(fd - 2.0 * (g * d).sum()) < 1e-8 * abs(fd)
