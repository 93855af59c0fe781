"""FP64 CPU oracle for per-element weak-form evaluation (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it, and it shares no code with
the GPU path: the C source `fe_oracle.c` builds its own quadrature rules and
basis tables and evaluates every form with plain nested loops over cells and
quadrature points (the paper's element loops, Algorithms "feloopv" and
"feloopm"), in FP64.

Every function is pinned by the tests against facts the mathematics fixes
(closed-form reference-cube matrices, 1-D tensor-product reductions, row sums,
volumes, rigid-body modes, quadrature exactness, finite differences,
numpy.einsum of the paper's printed contraction strings).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "liborc_fe.so")

CELLS = {"hex": 0, "tet": 1}
FORMS = {"mass": 0, "vmass": 1, "laplace": 2, "elasticity": 3, "wdot": 4,
         "convect": 5}
MATS = {None: 0, "none": 0, "iso_cell": 1, "iso_qp": 2, "voigt_qp": 3,
        "tensor_qp": 4}
_ERR = {-1: "bad argument", -2: "non-positive Jacobian determinant",
        -3: "node index out of range"}


class OracleError(RuntimeError):
    def __init__(self, code):
        self.code = code
        super().__init__(f"oracle status {code}: {_ERR.get(code, '?')}")


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, i32, dp, ip = (ctypes.c_int64, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_int32))
        L.orc_sizes.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
        L.orc_gauss_jacobi01.argtypes = [i32, i32, dp, dp]
        L.orc_tables.argtypes = [i32, i32, dp, dp, dp, dp]
        L.orc_matrix.argtypes = [i32, i32, i32, i64, i64, dp, ip, i32, dp, dp]
        L.orc_matrix_u.argtypes = [i32, i32, i32, i64, i64, dp, ip, i32, dp,
                                   dp, dp]
        L.orc_residual.argtypes = [i32, i32, i32, i64, i64, dp, ip, i32, dp,
                                   dp, i32, dp]
        L.orc_energy.argtypes = [i32, i32, i32, i64, i64, dp, ip, i32, dp, dp,
                                 dp]
        L.orc_energy_grad.argtypes = [i32, i32, i64, i64, dp, ip, dp, dp, dp,
                                      dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(code):
    if code != 0:
        raise OracleError(code)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def sizes(cell: str, order: int):
    nb, nq = ctypes.c_int(), ctypes.c_int()
    _check(lib().orc_sizes(CELLS[cell], order, ctypes.byref(nb),
                           ctypes.byref(nq)))
    return nb.value, nq.value


def n_comp(form: str) -> int:
    return 1 if form in ("mass", "laplace") else 3


def gauss_jacobi01(n: int, alpha: int = 0):
    """n-point Gauss rule on [0,1] for the weight (1-s)^alpha."""
    s, w = np.zeros(n), np.zeros(n)
    _check(lib().orc_gauss_jacobi01(n, alpha, _dp(s), _dp(w)))
    return s, w


def tables(cell: str, order: int):
    """(w[nq], pts[nq,3], bf[nq,nb], bfg[nq,3,nb]) of the reference element."""
    nb, nq = sizes(cell, order)
    w, pts = np.zeros(nq), np.zeros((nq, 3))
    bf, bfg = np.zeros((nq, nb)), np.zeros((nq, 3, nb))
    _check(lib().orc_tables(CELLS[cell], order, _dp(w), _dp(pts), _dp(bf),
                            _dp(bfg)))
    return w, pts, bf, bfg


def _mesh_args(mesh):
    coords = _f64(mesh.coords)
    conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
    return coords, conn


def matrix(mesh, form: str, material=None, mat_kind: str | None = None,
           u=None):
    """Element matrices (n_cells, nc*nb, nc*nb), FP64.  For "convect" the
    matrix is the derivative of the residual at the state u (n_nodes, 3)."""
    coords, conn = _mesh_args(mesh)
    nb = mesh.n_basis
    nd = n_comp(form) * nb
    out = np.empty((mesh.n_cells, nd, nd))
    mat = _f64(material)
    U = None if u is None else _f64(np.asarray(u).reshape(mesh.n_nodes, 3))
    _check(lib().orc_matrix_u(CELLS[mesh.cell], mesh.order, FORMS[form],
                              mesh.n_cells, mesh.n_nodes, _dp(coords),
                              _ip(conn), MATS[mat_kind], _dp(mat), _dp(U),
                              _dp(out)))
    return out


def residual(mesh, form: str, u, material=None, mat_kind: str | None = None,
             path: str = "gradient_first"):
    """Per-element residual (action) (n_cells, nc, nb), FP64, unassembled."""
    coords, conn = _mesh_args(mesh)
    nc = n_comp(form)
    U = _f64(np.asarray(u).reshape(mesh.n_nodes, nc))
    out = np.empty((mesh.n_cells, nc, mesh.n_basis))
    mat = _f64(material)
    _check(lib().orc_residual(CELLS[mesh.cell], mesh.order, FORMS[form],
                              mesh.n_cells, mesh.n_nodes, _dp(coords),
                              _ip(conn), MATS[mat_kind], _dp(mat), _dp(U),
                              {"gradient_first": 0, "matrix_first": 1}[path],
                              _dp(out)))
    return out


def energy(mesh, form: str, u, material=None, mat_kind: str | None = None):
    """Per-element integral value u_e^T K_e u_e (n_cells,), FP64."""
    coords, conn = _mesh_args(mesh)
    nc = n_comp(form)
    U = _f64(np.asarray(u).reshape(mesh.n_nodes, nc))
    out = np.empty(mesh.n_cells)
    mat = _f64(material)
    _check(lib().orc_energy(CELLS[mesh.cell], mesh.order, FORMS[form],
                            mesh.n_cells, mesh.n_nodes, _dp(coords),
                            _ip(conn), MATS[mat_kind], _dp(mat), _dp(U),
                            _dp(out)))
    return out


def energy_grad(mesh, lam_mu_qp, u, want_mat=True, want_coords=True):
    """Gradient of J = sum_e u_e^T K_e u_e (elasticity, per-qp lambda, mu)
    w.r.t. the coefficients (n_cells, nq, 2) and the node coordinates
    (n_nodes, 3)."""
    coords, conn = _mesh_args(mesh)
    nb, nq = sizes(mesh.cell, mesh.order)
    c = _f64(lam_mu_qp)
    U = _f64(np.asarray(u).reshape(mesh.n_nodes, 3))
    gm = np.empty((mesh.n_cells, nq, 2)) if want_mat else None
    gx = np.empty((mesh.n_nodes, 3)) if want_coords else None
    _check(lib().orc_energy_grad(CELLS[mesh.cell], mesh.order, mesh.n_cells,
                                 mesh.n_nodes, _dp(coords), _ip(conn), _dp(c),
                                 _dp(U), _dp(gm), _dp(gx)))
    return gm, gx


def einsum_operands(mesh):
    """The materialised operands of the paper's expression examples (the
    symbols table of section "Expression Examples") for every cell of a
    mesh, from this oracle's own reference tables: det (c, q) = w_q det J,
    bf (q, d), physical gradients bfg (c, q, j, d), the identity I and the
    symmetric-gradient extractor Psg (3, 3, 6) in the Voigt order
    11, 22, 33, 12, 13, 23 with ones for both shear entries."""
    w, _, bf, bfg_ref = tables(mesh.cell, mesh.order)
    X = np.asarray(mesh.coords)[np.asarray(mesh.conn)]   # (c, d, 3)
    J = np.einsum("cdi,qjd->cqij", X, bfg_ref)           # dx_i / dxi_j
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise OracleError(-2)
    Ji = np.linalg.inv(J)                                # (c, q, j, i) = dxi_j / dx_i
    bfg = np.einsum("qjd,cqji->cqid", bfg_ref, Ji)
    Psg = np.zeros((3, 3, 6))
    for K, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        Psg[i, j, K] = Psg[j, i, K] = 1.0
    return dict(det=det * w[None, :], bf=bf, bfg=bfg, I=np.eye(3), Psg=Psg)


def einsum_form(mesh, expressions, arrays):
    """Sum over (expression, operand names) pairs of numpy.einsum of the
    expression -- the plain definition of a transpiled weak form, evaluated
    the way the paper's numpy backend evaluates it.  arrays supplies the
    materials and 'dofs' (cell DOFs, (c, d) or (c, component, d)); the
    geometric operands come from einsum_operands."""
    ops = einsum_operands(mesh)
    ops.update(arrays)
    total = 0.0
    for expr, names in expressions:
        total = total + np.einsum(expr, *[ops[n] for n in names], optimize=True)
    return np.asarray(total)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following calls (1 = the paper's single-thread
    mode); the results do not depend on it."""
    lib().orc_set_num_threads(int(n))


def assemble_matrix(mesh, cell_mats, n_comp: int):
    """Global matrix (scipy CSR, FP64) of element matrices (n_cells, nc*nb,
    nc*nb): every entry K_e[(c,a),(d,b)] added at global row
    conn[e][a]*nc + c, column conn[e][b]*nc + d (the assembly that follows
    the element loops; duplicates summed by scipy's COO-to-CSR
    conversion)."""
    import scipy.sparse as sp
    nb, nc = mesh.n_basis, n_comp
    K = np.asarray(cell_mats, dtype=np.float64).reshape(mesh.n_cells, nc, nb,
                                                        nc, nb)
    conn = np.asarray(mesh.conn, dtype=np.int64)
    rows = (conn[:, None, :, None, None] * nc
            + np.arange(nc)[None, :, None, None, None])
    cols = (conn[:, None, None, None, :] * nc
            + np.arange(nc)[None, None, None, :, None])
    rows = np.broadcast_to(rows, K.shape).ravel()
    cols = np.broadcast_to(cols, K.shape).ravel()
    n = mesh.n_nodes * nc
    return sp.coo_matrix((K.ravel(), (rows, cols)), shape=(n, n)).tocsr()
