"""Pins of the oracle's quadrature rules and basis tables (CPU only).

Quadrature: exactness on monomials up to the rule's degree and failure one
degree above (so the degree is exact, not just a lower bound).  Basis:
reproduction of every polynomial of the element's space at the quadrature
points, values and gradients, which fixes the Lagrange basis of the stated
nodes uniquely.
"""
import itertools
from math import factorial

import numpy as np
import pytest


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("alpha", [0, 1, 2])
def test_gauss_jacobi_degree(orc, n, alpha):
    s, w = orc.gauss_jacobi01(n, alpha)
    assert np.all((s > 0) & (s < 1)) and np.all(w > 0)

    def exact(k):  # int_0^1 s^k (1-s)^alpha = k! alpha! / (k+alpha+1)!
        return factorial(k) * factorial(alpha) / factorial(k + alpha + 1)

    for k in range(2 * n):
        assert abs(np.dot(w, s ** k) - exact(k)) < 1e-14
    assert abs(np.dot(w, s ** (2 * n)) - exact(2 * n)) > 1e-10


def test_gauss_legendre_textbook_values(orc):
    # 2- and 3-point Gauss-Legendre on [-1,1]: +-1/sqrt(3) (w=1);
    # 0, +-sqrt(3/5) (w = 8/9, 5/9), mapped to [0,1]
    s, w = orc.gauss_jacobi01(2, 0)
    np.testing.assert_allclose(s, 0.5 + 0.5 * np.array([-1, 1]) / np.sqrt(3),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    s, w = orc.gauss_jacobi01(3, 0)
    np.testing.assert_allclose(
        s, 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0, np.sqrt(0.6)]), atol=1e-15)
    np.testing.assert_allclose(w, np.array([5, 8, 5]) / 18.0, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_hex_rule_exactness(orc, p):
    w, pts, _, _ = orc.tables("hex", p)
    n = p + 1
    assert w.shape == (n ** 3,)
    for a, b, c in itertools.product(range(2 * n), repeat=3):
        val = np.dot(w, pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        assert abs(val - 1.0 / ((a + 1) * (b + 1) * (c + 1))) < 1e-14
    # degree 2n in one variable is not integrated exactly
    assert abs(np.dot(w, pts[:, 0] ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-10


@pytest.mark.parametrize("p", [1, 2])
def test_tet_rule_exactness(orc, p):
    w, pts, _, _ = orc.tables("tet", p)
    deg = 2 * p + 1
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    x, y, z = pts.T
    assert np.all(x >= 0) and np.all(y >= 0) and np.all(z >= 0)
    assert np.all(x + y + z <= 1.0)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                ex = factorial(a) * factorial(b) * factorial(c) / factorial(
                    a + b + c + 3)
                assert abs(np.dot(w, x ** a * y ** b * z ** c) - ex) < 1e-15
    # one degree above is not exact for some monomial
    errs = []
    for a in range(deg + 2):
        for b in range(deg + 2 - a):
            c = deg + 1 - a - b
            ex = factorial(a) * factorial(b) * factorial(c) / factorial(
                deg + 4)
            errs.append(abs(np.dot(w, x ** a * y ** b * z ** c) - ex))
    assert max(errs) > 1e-12


def _hex_nodes(p):
    n = p + 1
    t = np.arange(n) / p
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    return np.stack([t[i.ravel()], t[j.ravel()], t[k.ravel()]], axis=1)


def _tet_nodes(p):
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    if p == 1:
        return V
    E = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
    return np.concatenate([V, [(V[a] + V[b]) / 2 for a, b in E]])


@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("hex", 3),
                                    ("hex", 4), ("hex", 5), ("tet", 1),
                                    ("tet", 2)])
def test_basis_reproduces_polynomial_space(orc, cell, p):
    w, pts, bf, bfg = orc.tables(cell, p)
    nodes = _hex_nodes(p) if cell == "hex" else _tet_nodes(p)
    if cell == "hex":
        exps = list(itertools.product(range(p + 1), repeat=3))
    else:
        exps = [e for e in itertools.product(range(p + 1), repeat=3)
                if sum(e) <= p]
    assert len(exps) == bf.shape[1]
    for e in exps:
        f_nodes = np.prod(nodes ** np.array(e), axis=1)
        f_q = np.prod(pts ** np.array(e), axis=1)
        np.testing.assert_allclose(bf @ f_nodes, f_q, atol=1e-13)
        for j in range(3):
            ej = list(e)
            if ej[j] == 0:
                d_q = np.zeros(len(pts))
            else:
                ej[j] -= 1
                d_q = e[j] * np.prod(pts ** np.array(ej), axis=1)
            np.testing.assert_allclose(bfg[:, j, :] @ f_nodes, d_q,
                                       atol=1e-12)
    # partition of unity and zero gradient sum
    np.testing.assert_allclose(bf.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose(bfg.sum(2), 0.0, atol=1e-12)
