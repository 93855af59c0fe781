"""Seeded synthetic inputs: meshes, material coefficients and DOF vectors.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It holds none of the finite element arithmetic (no basis
functions, no quadrature, no Jacobians): it only lays out node lattices,
perturbs them with seeded noise, numbers nodes and cells, and draws
coefficients and DOF values.

Conventions (they define the *input format* both implementations read):

* Hexahedra of order p: nodes form a lattice of m = p*n + 1 points per axis,
  node id = I + m_x*(J + m_y*K).  Cell id = ex + n_x*(ey + n_y*ez).  The
  local node index is lexicographic, a = i + (p+1)*(j + (p+1)*k), x fastest.
* Tetrahedra: every hex cell of a vertex lattice is split into 6 tetrahedra
  along its main diagonal (Kuhn/Freudenthal split).  Local vertex order is
  chosen so that every tetrahedron is positively oriented.  Quadratic
  tetrahedra add edge nodes in the order (0,1), (1,2), (0,2), (0,3), (1,3),
  (2,3); each edge node sits at the midpoint of its edge, shared between
  neighbours.
* Random streams: SeedSequence(seed).spawn(3) -> (geometry, material, dofs).
* Vertex perturbation: U(-alpha*h, alpha*h) drawn for *all* vertices in id
  order, applied to interior vertices only (so the box volume is kept).
  High-order nodes are placed at the trilinear image of their reference
  lattice position inside their cell (the element stays straight-sided in
  the trilinear sense).  `curved` additionally moves every interior lattice
  node (vertices and high-order nodes) by U(-curved*h, curved*h), which makes
  the geometry genuinely isoparametric of order p.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "streams", "hex_mesh", "tet_mesh", "lame_cell", "lame_qp",
    "voigt_iso", "voigt_random_spd", "dofs",
]


@dataclass
class Mesh:
    """A mesh of one cell kind and order.

    coords: (n_nodes, 3) float64, node positions.
    conn:   (n_cells, n_basis) int32, local-to-global node map.
    cell:   "hex" or "tet";  order: polynomial order p.
    h:      (3,) nominal cell size per axis.
    """
    coords: np.ndarray
    conn: np.ndarray
    cell: str
    order: int
    h: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_basis(self) -> int:
        return int(self.conn.shape[1])


def streams(seed: int):
    """(geometry, material, dofs) generators spawned from one seed."""
    ss = np.random.SeedSequence(seed)
    return tuple(np.random.default_rng(s) for s in ss.spawn(3))


def _as3(n):
    if np.isscalar(n):
        return (int(n),) * 3
    return tuple(int(v) for v in n)


def _vertex_lattice(n3, box, alpha, rng):
    """Vertex positions (nx+1, ny+1, nz+1, 3) [index order k, j, i] with
    interior vertices perturbed by U(-alpha*h, alpha*h)."""
    nx, ny, nz = n3
    h = np.asarray(box, dtype=np.float64) / np.asarray(n3, dtype=np.float64)
    gx = np.linspace(0.0, box[0], nx + 1)
    gy = np.linspace(0.0, box[1], ny + 1)
    gz = np.linspace(0.0, box[2], nz + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    V = np.stack([X, Y, Z], axis=-1)  # (nz+1, ny+1, nx+1, 3)
    nv = V.shape[0] * V.shape[1] * V.shape[2]
    noise = rng.uniform(-1.0, 1.0, size=(nv, 3)) * (alpha * h)
    noise = noise.reshape(V.shape)
    interior = np.zeros(V.shape[:3], dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    V = V + noise * interior[..., None]
    return V, h


def hex_mesh(n, order: int, alpha: float = 0.0, seed: int = 0,
             box=(1.0, 1.0, 1.0), curved: float = 0.0) -> Mesh:
    """Structured mesh of n^3 (or nx*ny*nz) hexahedra of Lagrange order p.

    alpha: interior vertex perturbation as a fraction of h.
    curved: extra perturbation of all interior lattice nodes (fraction of h).
    """
    p = int(order)
    if p < 1:
        raise ValueError("order must be >= 1")
    n3 = _as3(n)
    nx, ny, nz = n3
    g_rng, _, _ = streams(seed)
    V, h = _vertex_lattice(n3, box, alpha, g_rng)

    # lattice of m = p*n + 1 nodes per axis; each lattice line index I lies in
    # cell c = min(I // p, n - 1) at local fraction t = (I - p*c) / p.
    def split(nc):
        I = np.arange(p * nc + 1)
        c = np.minimum(I // p, nc - 1)
        t = (I - p * c) / p
        return c, t

    cx, tx = split(nx)
    cy, ty = split(ny)
    cz, tz = split(nz)
    CZ, CY, CX = np.meshgrid(cz, cy, cx, indexing="ij")
    TZ, TY, TX = np.meshgrid(tz, ty, tx, indexing="ij")
    P = np.zeros(CX.shape + (3,))
    # trilinear image of (tx, ty, tz) in cell (cx, cy, cz): placement rule of
    # the generator, a weighted average of the 8 cell vertices
    for dz in (0, 1):
        wz = TZ if dz else 1.0 - TZ
        for dy in (0, 1):
            wy = TY if dy else 1.0 - TY
            for dx in (0, 1):
                wx = TX if dx else 1.0 - TX
                P += (wx * wy * wz)[..., None] * V[CZ + dz, CY + dy, CX + dx]
    mx, my, mz = p * nx + 1, p * ny + 1, p * nz + 1
    coords = P.reshape(-1, 3)
    if curved > 0.0:
        noise = g_rng.uniform(-1.0, 1.0, size=coords.shape) * (curved * h)
        K, J, I = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx),
                              indexing="ij")
        inner = ((I > 0) & (I < mx - 1) & (J > 0) & (J < my - 1)
                 & (K > 0) & (K < mz - 1)).reshape(-1)
        coords = coords + noise * inner[:, None]
    coords = np.ascontiguousarray(coords, dtype=np.float64)

    # connectivity, local a = i + (p+1)*(j + (p+1)*k)
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)
    lk, lj, li = np.meshgrid(np.arange(p + 1), np.arange(p + 1),
                             np.arange(p + 1), indexing="ij")
    li, lj, lk = li.reshape(-1), lj.reshape(-1), lk.reshape(-1)
    gi = p * ex[:, None] + li[None, :]
    gj = p * ey[:, None] + lj[None, :]
    gk = p * ez[:, None] + lk[None, :]
    conn = (gi + mx * (gj + my * gk)).astype(np.int64)
    if conn.max() >= 2**31:
        raise ValueError("mesh too large for int32 connectivity")
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    return Mesh(coords=coords, conn=conn, cell="hex", order=p, h=h,
                info=dict(n=n3, alpha=alpha, seed=seed, curved=curved,
                          box=tuple(box)))


# Kuhn split of the unit cube (corner c = dx + 2*dy + 4*dz) into 6
# tetrahedra sharing the diagonal 0-7; each path 0 -> 7 flips one axis at a
# time.  Orientation is fixed below by swapping two vertices where needed.
_KUHN_PATHS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1),
               (2, 1, 0)]


def _kuhn_tets():
    tets = []
    for perm in _KUHN_PATHS:
        c = 0
        verts = [0]
        for ax in perm:
            c |= 1 << ax
            verts.append(c)
        # orientation from the corner offsets (combinatorial sign only)
        off = [np.array([(v >> 0) & 1, (v >> 1) & 1, (v >> 2) & 1], float)
               for v in verts]
        vol6 = np.linalg.det(np.stack([off[1] - off[0], off[2] - off[0],
                                       off[3] - off[0]]))
        if vol6 < 0:
            verts[1], verts[2] = verts[2], verts[1]
        tets.append(verts)
    return np.array(tets, dtype=np.int64)


_TET_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


def tet_mesh(n, order: int, alpha: float = 0.0, seed: int = 0,
             box=(1.0, 1.0, 1.0)) -> Mesh:
    """6*nx*ny*nz tetrahedra (order 1 or 2) from a perturbed vertex lattice."""
    p = int(order)
    if p not in (1, 2):
        raise ValueError("tetrahedra of order 1 or 2 only")
    n3 = _as3(n)
    nx, ny, nz = n3
    g_rng, _, _ = streams(seed)
    V, h = _vertex_lattice(n3, box, alpha, g_rng)
    vcoords = V.reshape(-1, 3)
    mx, my = nx + 1, ny + 1
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)
    corner = np.empty((ex.size, 8), dtype=np.int64)
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corner[:, c] = (ex + dx) + mx * ((ey + dy) + my * (ez + dz))
    kt = _kuhn_tets()
    conn1 = corner[:, kt].reshape(-1, 4)  # (6*ncells, 4), cell-major
    if p == 1:
        return Mesh(coords=np.ascontiguousarray(vcoords), conn=conn1.astype(
            np.int32), cell="tet", order=1, h=h,
            info=dict(n=n3, alpha=alpha, seed=seed, box=tuple(box)))
    # quadratic: unique edges -> midpoint nodes appended after the vertices
    ev = np.stack([np.stack([conn1[:, a], conn1[:, b]], axis=1)
                   for a, b in _TET_EDGES], axis=1)  # (nt, 6, 2)
    key = np.sort(ev, axis=2).reshape(-1, 2)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    mid = 0.5 * (vcoords[uniq[:, 0]] + vcoords[uniq[:, 1]])
    coords = np.concatenate([vcoords, mid], axis=0)
    edge_ids = vcoords.shape[0] + inv.reshape(-1, 6)
    conn = np.concatenate([conn1, edge_ids], axis=1)
    if conn.max() >= 2**31:
        raise ValueError("mesh too large for int32 connectivity")
    return Mesh(coords=np.ascontiguousarray(coords), conn=conn.astype(
        np.int32), cell="tet", order=2, h=h,
        info=dict(n=n3, alpha=alpha, seed=seed, box=tuple(box)))


def lame_cell(n_cells: int, seed: int = 0) -> np.ndarray:
    """(n_cells, 2) float64 [lambda, mu], each lognormal(0, 0.5)."""
    _, m_rng, _ = streams(seed)
    return np.ascontiguousarray(m_rng.lognormal(0.0, 0.5, size=(n_cells, 2)))


def lame_qp(n_cells: int, n_qp: int, seed: int = 0) -> np.ndarray:
    """(n_cells, n_qp, 2) float64 [lambda, mu] per quadrature point."""
    _, m_rng, _ = streams(seed)
    return np.ascontiguousarray(
        m_rng.lognormal(0.0, 0.5, size=(n_cells, n_qp, 2)))


def voigt_iso(lam_mu: np.ndarray) -> np.ndarray:
    """Isotropic 6x6 Voigt stiffness (order 11,22,33,12,13,23, engineering
    shear) for every leading index of lam_mu[..., 2]; a coefficient layout
    conversion only."""
    lam = lam_mu[..., 0][..., None, None]
    mu = lam_mu[..., 1][..., None, None]
    m = np.array([1, 1, 1, 0, 0, 0], dtype=np.float64)
    d = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    return np.ascontiguousarray(lam * np.outer(m, m) + mu * d)


def voigt_random_spd(shape, seed: int = 0) -> np.ndarray:
    """Random symmetric positive definite 6x6 matrices, shape + (6, 6)."""
    _, m_rng, _ = streams(seed)
    A = m_rng.standard_normal(tuple(shape) + (6, 6))
    D = A @ np.swapaxes(A, -1, -2) / 6.0 + np.eye(6)
    return np.ascontiguousarray(D)


def tensor_qp(n_cells: int, n_qp: int, seed: int = 0) -> np.ndarray:
    """(n_cells, n_qp, 3, 3) float64 coefficients M of the weighted vector dot
    product: I + 0.3 N with N ~ N(0, 1) entrywise (not symmetric)."""
    _, m_rng, _ = streams(seed)
    A = m_rng.standard_normal((n_cells, n_qp, 3, 3))
    return np.ascontiguousarray(np.eye(3) + 0.3 * A)


def dofs(n_nodes: int, n_comp: int, seed: int = 0) -> np.ndarray:
    """(n_nodes, n_comp) float64 DOF values ~ N(0, 1)."""
    _, _, d_rng = streams(seed)
    return np.ascontiguousarray(d_rng.standard_normal((n_nodes, n_comp)))
