"""Exact rational reference integrals (pure Python Fractions).

Used by the tests to pin the oracle: 1-D Lagrange mass/stiffness/mixed
matrices on [0,1], their tensor products for boxes, and the P1/P2 tetrahedron
reference integrals from the monomial formula
    int_T x^a y^b z^c = a! b! c! / (a+b+c+3)!
None of this shares code with the oracle or the GPU library.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from math import factorial

import numpy as np

# ---------------------------------------------------------------- 1-D -----


def _pmul(a, b):
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pder(a):
    return [i * a[i] for i in range(1, len(a))] or [Fr(0)]


def _pint01(a):
    return sum(c / (i + 1) for i, c in enumerate(a))


def lagrange_poly(p: int, k: int):
    """Coefficients (low -> high) of the equispaced Lagrange polynomial k."""
    nodes = [Fr(m, p) for m in range(p + 1)]
    poly = [Fr(1)]
    for m in range(p + 1):
        if m == k:
            continue
        d = nodes[k] - nodes[m]
        poly = _pmul(poly, [-nodes[m] / d, Fr(1) / d])
    return poly


def mats_1d(p: int):
    """Exact 1-D matrices on [0,1]: M[k,l] = int phi_k phi_l,
    K[k,l] = int phi_k' phi_l', N[k,l] = int phi_k' phi_l."""
    P = [lagrange_poly(p, k) for k in range(p + 1)]
    D = [_pder(x) for x in P]
    n = p + 1
    M = [[_pint01(_pmul(P[k], P[l])) for l in range(n)] for k in range(n)]
    K = [[_pint01(_pmul(D[k], D[l])) for l in range(n)] for k in range(n)]
    N = [[_pint01(_pmul(D[k], P[l])) for l in range(n)] for k in range(n)]
    return M, K, N


def box_grad_products(p: int, h=(1.0, 1.0, 1.0)):
    """S[r][s][a,b] = int_box d phi_a/dx_r  d phi_b/dx_s for the axis-aligned
    box of sides h, Q_p lexicographic numbering (x fastest), as float arrays
    built from exact 1-D matrices by Kronecker products (kron order z,y,x).
    Also returns the mass matrix."""
    M, K, N = (np.array([[float(v) for v in row] for row in A])
               for A in mats_1d(p))
    Nt = N.T  # int phi_k phi_l'

    def axis_mat(d, r, s):
        da, db = (d == r), (d == s)
        if da and db:
            return K / h[d]
        if da:
            return N.copy()
        if db:
            return Nt.copy()
        return M * h[d]

    S = [[None] * 3 for _ in range(3)]
    for r in range(3):
        for s in range(3):
            S[r][s] = np.kron(axis_mat(2, r, s),
                              np.kron(axis_mat(1, r, s), axis_mat(0, r, s)))
    mass = np.kron(M * h[2], np.kron(M * h[1], M * h[0]))
    return S, mass


# ---------------------------------------------------------------- tet -----

def _poly3_mul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = (ka[0] + kb[0], ka[1] + kb[1], ka[2] + kb[2])
            out[k] = out.get(k, Fr(0)) + va * vb
    return out


def _poly3_der(a, j):
    out = {}
    for k, v in a.items():
        if k[j] == 0:
            continue
        kk = list(k)
        kk[j] -= 1
        out[tuple(kk)] = out.get(tuple(kk), Fr(0)) + v * k[j]
    return out


def _poly3_int_tet(a):
    s = Fr(0)
    for (i, j, k), v in a.items():
        s += v * Fr(factorial(i) * factorial(j) * factorial(k),
                    factorial(i + j + k + 3))
    return s


def tet_basis_polys(p: int):
    L = [{(0, 0, 0): Fr(1), (1, 0, 0): Fr(-1), (0, 1, 0): Fr(-1),
          (0, 0, 1): Fr(-1)},
         {(1, 0, 0): Fr(1)}, {(0, 1, 0): Fr(1)}, {(0, 0, 1): Fr(1)}]
    if p == 1:
        return L
    out = []
    for a in range(4):
        two_l_minus_1 = {k: 2 * v for k, v in L[a].items()}
        two_l_minus_1[(0, 0, 0)] = two_l_minus_1.get((0, 0, 0), Fr(0)) - 1
        out.append(_poly3_mul(L[a], two_l_minus_1))
    for i, k in [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]:
        prod = _poly3_mul(L[i], L[k])
        out.append({kk: 4 * v for kk, v in prod.items()})
    return out


def tet_reference(p: int):
    """Exact reference-tet mass matrix and gradient products
    S[j][k][a,b] = int dphi_a/dxi_j dphi_b/dxi_k."""
    P = tet_basis_polys(p)
    n = len(P)
    Dp = [[_poly3_der(P[a], j) for j in range(3)] for a in range(n)]
    mass = np.array([[float(_poly3_int_tet(_poly3_mul(P[a], P[b])))
                      for b in range(n)] for a in range(n)])
    S = [[np.array([[float(_poly3_int_tet(_poly3_mul(Dp[a][j], Dp[b][k])))
                     for b in range(n)] for a in range(n)])
          for k in range(3)] for j in range(3)]
    return S, mass


def hex_reference(p: int):
    """Exact reference-cube mass and gradient products (unit sides)."""
    return box_grad_products(p)[::-1]


def mapped_grad_products(S_ref, A):
    """For the affine map x = A xi + b: int_T dphi_a/dx_r dphi_b/dx_s
    = det(A) sum_jk Ainv[j,r] Ainv[k,s] S_ref[j][k]."""
    Ai = np.linalg.inv(A)
    dA = np.linalg.det(A)
    nb = S_ref[0][0].shape[0]
    S = [[np.zeros((nb, nb)) for _ in range(3)] for _ in range(3)]
    for r in range(3):
        for s in range(3):
            acc = np.zeros((nb, nb))
            for j in range(3):
                for k in range(3):
                    acc += Ai[j, r] * Ai[k, s] * S_ref[j][k]
            S[r][s] = dA * acc
    return S


def laplace_from_S(S):
    return S[0][0] + S[1][1] + S[2][2]


def elasticity_from_S(S, lam, mu):
    """K[(r,a),(s,b)] = lam S[r][s] + mu S[s][r] + delta_rs mu sum_j S[j][j]
    (from e(v):C:e(u) with C isotropic), component-major (3nb x 3nb)."""
    nb = S[0][0].shape[0]
    L = laplace_from_S(S)
    K = np.zeros((3 * nb, 3 * nb))
    for r in range(3):
        for s in range(3):
            blk = lam * S[r][s] + mu * S[s][r]
            if r == s:
                blk = blk + mu * L
            K[r * nb:(r + 1) * nb, s * nb:(s + 1) * nb] = blk
    return K
