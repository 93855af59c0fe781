"""MI355X (gfx950) per-element finite element weak-form evaluation.

Python face of libfe_forms.so: plans for (cell, order, form, mode, precision,
material kind) and their execution on device tensors.  PyTorch provides the
device memory and the stream; the evaluation itself (gather, FP64 geometry,
contraction, output) runs in the library's HIP kernels.

    plan = Plan("hex", 2, "elasticity", "matrix", "fp64", material="iso_cell")
    K = plan(coords, conn, material=lam_mu)     # (n_cells, 81, 81) on cuda
    plan.check()                                # raises on det J <= 0 etc.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FeError

__all__ = ["Plan", "FeError", "Incidence", "assemble", "Pattern",
           "assemble_matrix", "reference_sizes", "reference_tables",
           "n_comp", "ElasticEnergy", "Batch", "BilinearPlan", "eval_sum",
           "make_reference"]

_TORCH_DT = {"fp64": "float64", "fp32": "float32", "bf16x3": "float32"}


def n_comp(form: str) -> int:
    """Vector components of a form's variables: 1 for mass and Laplace, 3
    for the vector forms."""
    return 1 if form in ("mass", "laplace") else 3


def reference_sizes(cell: str, order: int):
    nb, nq = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.lib().fe_reference_sizes(_lib.CELLS[cell], order,
                                             ctypes.byref(nb),
                                             ctypes.byref(nq)),
               "fe_reference_sizes")
    return nb.value, nq.value


def reference_tables(cell: str, order: int):
    """The library's own (w[nq], pts[nq,3], bf[nq,nb], bfg[nq,3,nb])."""
    nb, nq = reference_sizes(cell, order)
    w, pts = np.zeros(nq), np.zeros((nq, 3))
    bf, bfg = np.zeros((nq, nb)), np.zeros((nq, 3, nb))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(_lib.lib().fe_reference_tables(
        _lib.CELLS[cell], order, w.ctypes.data_as(dp),
        pts.ctypes.data_as(dp), bf.ctypes.data_as(dp),
        bfg.ctypes.data_as(dp)), "fe_reference_tables")
    return w, pts, bf, bfg


def make_reference(cell: str, order: int, weights, bf, bfg):
    """An fe_reference over host FP64 copies of the caller's tables; returns
    (struct, arrays kept alive for it)."""
    w = np.ascontiguousarray(weights, dtype=np.float64)
    b = np.ascontiguousarray(bf, dtype=np.float64)
    g = np.ascontiguousarray(bfg, dtype=np.float64)
    nq = w.shape[0]
    if b.ndim != 2 or b.shape[0] != nq or g.shape != (nq, 3, b.shape[1]):
        raise ValueError("reference tables must be weights[nq], bf[nq, nb], "
                         "bfg[nq, 3, nb]")
    dp = ctypes.POINTER(ctypes.c_double)
    ref = _lib.fe_reference(_lib.CELLS[cell], int(order), b.shape[1], nq,
                            w.ctypes.data_as(dp), b.ctypes.data_as(dp),
                            g.ctypes.data_as(dp))
    return ref, (w, b, g)


def material_entries(kind, n_qp: int) -> int:
    """Material entries per cell of a material kind (the layouts of
    fe_material_kind): iso_cell 2, iso_qp 2 n_qp, voigt_qp 36 n_qp,
    tensor_qp 9 n_qp, none 0."""
    return {"iso_cell": 2, "iso_qp": 2 * n_qp, "voigt_qp": 36 * n_qp,
            "tensor_qp": 9 * n_qp}.get(kind, 0)


def validate_inputs(n_basis, n_qp, n_comp_, material_kind, dtype, coords,
                    conn, material=None, dofs=None):
    """Host-side checks of the arrays passed to a plan (shapes, dtypes,
    entry counts per material kind, then device and contiguity); raises
    ValueError before anything reaches the library."""
    import torch
    if conn.dim() != 2 or conn.shape[1] != n_basis:
        raise ValueError(f"conn must have {n_basis} columns")
    n_cells = conn.shape[0]
    if coords.dtype != torch.float64 or coords.dim() != 2 or \
            coords.shape[1] != 3:
        raise ValueError("coords must be (n_nodes, 3) float64")
    if conn.dtype != torch.int32:
        raise ValueError("conn must be int32")
    if material is not None and material.dtype != dtype:
        raise ValueError(f"material must be {dtype}")
    if dofs is not None and dofs.dtype != dtype:
        raise ValueError(f"dofs must be {dtype}")
    per_cell = material_entries(material_kind, n_qp)
    if per_cell and material is not None and \
            material.numel() != n_cells * per_cell:
        raise ValueError(f"material has {material.numel()} entries, a "
                         f"{material_kind} material of {n_cells} cells "
                         f"needs {n_cells * per_cell}")
    if dofs is not None and dofs.numel() != coords.shape[0] * n_comp_:
        raise ValueError(f"dofs has {dofs.numel()} entries, "
                         f"{coords.shape[0]} nodes x {n_comp_} components "
                         "expected")
    for name, t in (("coords", coords), ("conn", conn),
                    ("material", material), ("dofs", dofs)):
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous cuda tensor")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """One compiled evaluation: cell kind/order, form, mode, precision and
    material layout.  Calls are asynchronous on the current torch stream."""

    def __init__(self, cell: str, order: int, form: str, mode: str = "matrix",
                 precision: str = "fp64", material: str | None = None,
                 variant: str = "auto", xcd_remap: bool = True,
                 layout: str = "cell_major", chunk: int = 0,
                 reference=None):
        """reference: optional (weights[nq], bf[nq, nb], bfg[nq, 3, nb])
        host arrays of the caller's reference element (fe_plan_create_ref);
        by default the library builds its own."""
        self.cell, self.order, self.form = cell, int(order), form
        self.mode, self.precision, self.material = mode, precision, material
        self.layout = layout
        opts = _lib.fe_options(_lib.VARIANTS[variant], 1 if xcd_remap else 0,
                               _lib.LAYOUTS[layout], int(chunk))
        h = ctypes.c_void_p()
        L = _lib.lib()
        if reference is None:
            _lib.check(L.fe_plan_create(_lib.CELLS[cell], self.order,
                                        _lib.FORMS[form], _lib.MODES[mode],
                                        _lib.PRECS[precision],
                                        _lib.MATS[material],
                                        ctypes.byref(opts), ctypes.byref(h)),
                       "fe_plan_create")
        else:
            ref, self._ref_keep = make_reference(cell, self.order, *reference)
            _lib.check(L.fe_plan_create_ref(ctypes.byref(ref),
                                            _lib.FORMS[form], _lib.MODES[mode],
                                            _lib.PRECS[precision],
                                            _lib.MATS[material],
                                            ctypes.byref(opts),
                                            ctypes.byref(h)),
                       "fe_plan_create_ref")
        self._h = h
        ints = [ctypes.c_int() for _ in range(5)]
        _lib.check(L.fe_plan_info(h, *[ctypes.byref(i) for i in ints]),
                   "fe_plan_info")
        self.n_basis, self.n_qp, self.n_comp, v, self.n_dof = (
            i.value for i in ints)
        self.variant = _lib.VARIANT_NAMES[v]
        self._ws = None

    def __del__(self):
        # the library handle is looked up defensively: at interpreter exit
        # module globals may already be gone
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.fe_plan_destroy(h)
            self._h = None

    @property
    def dtype(self):
        import torch
        return getattr(torch, _TORCH_DT[self.precision])

    def workspace_bytes(self, n_cells: int) -> int:
        b = ctypes.c_size_t()
        _lib.check(_lib.lib().fe_plan_workspace_size(self._h, n_cells,
                                                     ctypes.byref(b)),
                   "fe_plan_workspace_size")
        return b.value

    def workspace(self, n_cells: int, device=None):
        """A zero-filled device workspace large enough for n_cells (reused
        between calls of this plan)."""
        import torch
        need = self.workspace_bytes(n_cells)
        if self._ws is None or self._ws.numel() < need or (
                device is not None and self._ws.device != device):
            self._ws = torch.zeros(need, dtype=torch.uint8,
                                   device=device or "cuda")
        return self._ws

    def out_shape(self, n_cells: int):
        if self.mode == "matrix":
            return (n_cells, self.n_dof, self.n_dof)
        if self.mode == "residual":
            if self.layout == "cell_minor":
                return (self.n_comp, self.n_basis, n_cells)
            return (n_cells, self.n_comp, self.n_basis)
        return (n_cells,)

    def __call__(self, coords, conn, material=None, dofs=None, out=None,
                 workspace=None, stream=None):
        import torch
        validate_inputs(self.n_basis, self.n_qp, self.n_comp, self.material,
                        self.dtype, coords, conn, material, dofs)
        n_cells = conn.shape[0]
        dt = self.dtype
        if out is None:
            out = torch.empty(self.out_shape(n_cells), dtype=dt,
                              device=coords.device)
        elif (tuple(out.shape) != self.out_shape(n_cells) or out.dtype != dt
              or not out.is_contiguous()):
            raise ValueError("out has the wrong shape/dtype/layout")
        ws = workspace if workspace is not None else self.workspace(
            n_cells, coords.device)
        _lib.check(_lib.lib().fe_execute(
            self._h, n_cells, coords.shape[0], _ptr(coords), _ptr(conn),
            _ptr(material), _ptr(dofs), _ptr(out), _ptr(ws), ws.numel(),
            _stream_handle(stream)), "fe_execute")
        return out

    def execute_noalloc(self, coords, conn, material=None, dofs=None,
                        out=None, fault=None, stream=None):
        """fe_execute_noalloc: the same evaluation without a workspace (the
        library's static device scratch holds the fault bits and any
        matrix-first chunk).  out must be given (nothing is allocated);
        fault, a one-element int32 cuda tensor or None, receives the call's
        fault bits."""
        validate_inputs(self.n_basis, self.n_qp, self.n_comp, self.material,
                        self.dtype, coords, conn, material, dofs)
        n_cells = conn.shape[0]
        if out is None or tuple(out.shape) != self.out_shape(n_cells) or \
                out.dtype != self.dtype or not out.is_contiguous():
            raise ValueError("out must be a preallocated contiguous tensor "
                             f"of shape {self.out_shape(n_cells)}")
        _lib.check(_lib.lib().fe_execute_noalloc(
            self._h, n_cells, coords.shape[0], _ptr(coords), _ptr(conn),
            _ptr(material), _ptr(dofs), _ptr(out), _ptr(fault),
            _stream_handle(stream)), "fe_execute_noalloc")
        return out

    def check(self, workspace=None, stream=None):
        """Synchronise and raise FeError if a kernel saw det J <= 0 or an
        out-of-range node number since the last check."""
        ws = workspace if workspace is not None else self._ws
        if ws is None:
            return
        _lib.check(_lib.lib().fe_plan_check(self._h, _ptr(ws),
                                            _stream_handle(stream)),
                   "fe_plan_check")


class Incidence:
    """Node-to-(cell, local node) incidence of a connectivity (CSR, built on
    the device, sorted so every gather over it has a fixed order)."""

    def __init__(self, conn, n_nodes: int, stream=None):
        if conn.dtype.__str__() != "torch.int32" or not conn.is_cuda or \
                not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 cuda tensor")
        self.n_cells, self.n_basis = conn.shape
        self.n_nodes = int(n_nodes)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().fe_incidence_create(
            self.n_cells, self.n_nodes, self.n_basis, _ptr(conn),
            _stream_handle(stream), ctypes.byref(h)), "fe_incidence_create")
        self._h = h

    def __del__(self):
        # the library handle is looked up defensively: at interpreter exit
        # module globals may already be gone
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.fe_incidence_destroy(h)
            self._h = None


def assemble(inc: Incidence, cell_vec, scale: float = 1.0, out=None,
             stream=None):
    """Sum per-cell vectors (n_cells, n_comp, n_basis) into nodal ones
    (n_nodes, n_comp) through the incidence."""
    import torch
    n_cells, nc, nb = cell_vec.shape
    if (n_cells, nb) != (inc.n_cells, inc.n_basis):
        raise ValueError("cell_vec does not match the incidence")
    if not cell_vec.is_contiguous():
        raise ValueError("cell_vec must be contiguous")
    prec = {torch.float64: 0, torch.float32: 1}[cell_vec.dtype]
    if out is None:
        out = torch.empty((inc.n_nodes, nc), dtype=cell_vec.dtype,
                          device=cell_vec.device)
    _lib.check(_lib.lib().fe_assemble(inc._h, nc, prec, _ptr(cell_vec),
                                      float(scale), _ptr(out),
                                      _stream_handle(stream)), "fe_assemble")
    return out


class Pattern:
    """Sparsity pattern of the global matrix of a connectivity: CSR over
    nodes (row node n couples to every node sharing a cell with n), built on
    the device; row_ptr (n_nodes + 1) and cols (nnz) as int32 cuda
    tensors."""

    def __init__(self, conn, n_nodes: int, stream=None):
        import torch
        if conn.dtype != torch.int32 or not conn.is_cuda or \
                not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 cuda tensor")
        self.n_cells, self.n_basis = conn.shape
        self.n_nodes = int(n_nodes)
        h = ctypes.c_void_p()
        L = _lib.lib()
        _lib.check(L.fe_pattern_create(
            self.n_cells, self.n_nodes, self.n_basis, _ptr(conn),
            _stream_handle(stream), ctypes.byref(h)), "fe_pattern_create")
        self._h = h
        nn, nnz = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(L.fe_pattern_info(h, ctypes.byref(nn), ctypes.byref(nnz)),
                   "fe_pattern_info")
        self.nnz = nnz.value
        self.row_ptr = torch.empty(self.n_nodes + 1, dtype=torch.int32,
                                   device=conn.device)
        self.cols = torch.empty(max(self.nnz, 1), dtype=torch.int32,
                                device=conn.device)[:self.nnz]
        _lib.check(L.fe_pattern_copy(h, _ptr(self.row_ptr), _ptr(self.cols),
                                     _stream_handle(stream)),
                   "fe_pattern_copy")

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.fe_pattern_destroy(h)
            self._h = None


def assemble_matrix(pattern: Pattern, inc: Incidence, conn, cell_mats,
                    scale: float = 1.0, out=None, stream=None):
    """Sum element matrices (n_cells, n_comp n_basis, n_comp n_basis) into
    the block-CSR global matrix of the pattern: values (nnz, n_comp,
    n_comp), block k of row node n holding the coupling to node cols[k]."""
    import torch
    n_cells, nd, nd2 = cell_mats.shape
    nc = nd // pattern.n_basis
    if nd != nd2 or nc * pattern.n_basis != nd or nc not in (1, 3) or \
            n_cells != pattern.n_cells:
        raise ValueError("cell_mats does not match the pattern")
    if not cell_mats.is_contiguous():
        raise ValueError("cell_mats must be contiguous")
    prec = {torch.float64: 0, torch.float32: 1}[cell_mats.dtype]
    if out is None:
        out = torch.empty((max(pattern.nnz, 1), nc, nc),
                          dtype=cell_mats.dtype,
                          device=cell_mats.device)[:pattern.nnz]
    _lib.check(_lib.lib().fe_assemble_matrix(
        pattern._h, inc._h, _ptr(conn), nc, prec, _ptr(cell_mats),
        float(scale), _ptr(out), _stream_handle(stream)),
        "fe_assemble_matrix")
    return out


def energy_grad_workspace(plan, n_cells: int, device):
    """A zero-filled workspace for _energy_grad on n_cells cells."""
    import torch
    b = ctypes.c_size_t()
    _lib.check(_lib.lib().fe_energy_grad_workspace_size(plan._h, n_cells,
                                                        ctypes.byref(b)),
               "fe_energy_grad_workspace_size")
    return torch.zeros(b.value, dtype=torch.uint8, device=device)


def _energy_grad(plan, inc, coords, conn, material, dofs, scale,
                 want_mat=True, want_coords=True, stream=None, ws=None,
                 gm=None, gx=None, check=True):
    """dJ/dc and dJ/dx of the elasticity eval value (see fe_energy_grad).
    ws, gm, gx may be passed preallocated; check=False skips the
    synchronising fault check."""
    import torch
    n_cells = conn.shape[0]
    if ws is None:
        ws = energy_grad_workspace(plan, n_cells, coords.device)
    if gm is None and want_mat:
        gm = torch.empty_like(material)
    if gx is None and want_coords:
        gx = torch.empty_like(coords)
    _lib.check(_lib.lib().fe_energy_grad(
        plan._h, inc._h if inc is not None else None, n_cells,
        coords.shape[0], _ptr(coords), _ptr(conn), _ptr(material),
        _ptr(dofs), float(scale), _ptr(gm), _ptr(gx), _ptr(ws), ws.numel(),
        _stream_handle(stream)), "fe_energy_grad")
    if check:
        plan.check(ws, stream)
    return gm, gx


def eval_sum(plan, coords, conn, material=None, dofs=None, cell_values=None,
             stream=None):
    """fe_eval_sum: the eval-mode integral over the whole mesh, summed by the
    library in a fixed order in FP64; a 0-d float64 cuda tensor (the
    per-cell values go to cell_values, allocated if None)."""
    import torch
    if plan.mode != "eval":
        raise ValueError("eval_sum needs an eval plan")
    validate_inputs(plan.n_basis, plan.n_qp, plan.n_comp, plan.material,
                    plan.dtype, coords, conn, material, dofs)
    n_cells = conn.shape[0]
    if cell_values is None:
        cell_values = torch.empty(n_cells, dtype=plan.dtype,
                                  device=coords.device)
    total = torch.empty((), dtype=torch.float64, device=coords.device)
    ws = plan.workspace(n_cells, coords.device)
    _lib.check(_lib.lib().fe_eval_sum(
        plan._h, n_cells, coords.shape[0], _ptr(coords), _ptr(conn),
        _ptr(material), _ptr(dofs), _ptr(cell_values), _ptr(total),
        _ptr(ws), ws.numel(), _stream_handle(stream)), "fe_eval_sum")
    return total


class ElasticEnergyPlan:
    """Everything the elasticity energy J(c, x, u) = sum_e u_e^T K_e u_e
    needs for one mesh topology: eval and residual plans, the incidence and
    the gradient kernel's workspace."""

    def __init__(self, cell, order, conn, n_nodes, precision="fp64",
                 material="iso_qp"):
        self.conn = conn
        self.n_nodes = int(n_nodes)
        self.eval = Plan(cell, order, "elasticity", "eval", precision,
                         material=material)
        self.resid = Plan(cell, order, "elasticity", "residual", precision,
                          material=material)
        self.inc = Incidence(conn, n_nodes)
        self._gws = None

    def grad_workspace(self, device):
        """The gradient kernel's workspace, zero-filled once: its fault bits
        are cleared by check() and the rest is overwritten by every call."""
        n_cells = self.conn.shape[0]
        b = ctypes.c_size_t()
        _lib.check(_lib.lib().fe_energy_grad_workspace_size(
            self.eval._h, n_cells, ctypes.byref(b)),
            "fe_energy_grad_workspace_size")
        if self._gws is None or self._gws.numel() < b.value or \
                self._gws.device != device:
            self._gws = energy_grad_workspace(self.eval, n_cells, device)
        return self._gws

    def check(self, stream=None):
        """Synchronise and raise FeError if a kernel of the energy, of its
        gradient or of the residual saw det J <= 0 or an out-of-range node
        number since the last check.  Every workspace is read and cleared
        before the first fault found is raised."""
        import torch
        checks = [(self.eval, self.eval._ws), (self.resid, self.resid._ws)]
        if self._gws is not None:
            checks.append((self.eval, self._gws))
        checks = [(plan, ws) for plan, ws in checks if ws is not None]
        if not checks:
            return
        # one device-to-host read of every fault word (the first four bytes
        # of each workspace) on the stream the kernels ran on; the library's
        # check, which names the fault and clears the bits, runs only when
        # one of them is set
        with torch.cuda.stream(stream):  # a no-op for None (the current stream)
            words = torch.cat([ws[:4] for _, ws in checks]).cpu()
        if not bool(words.any()):
            return
        first = None
        for plan, ws in checks:
            try:
                plan.check(ws, stream)
            except FeError as err:
                first = first or err
        if first is not None:
            raise first


def _make_energy_function():
    import torch

    class _ElasticEnergy(torch.autograd.Function):
        """J = sum_e u_e^T K_e(c, x) u_e.  Backward: dJ/dc, dJ/dx from the
        adjoint kernel (geometry recomputed), dJ/du = 2 * assembled
        residual.  The forward does not synchronise; the backward checks
        the fault bits of both passes once, after its launches, and keeps
        the incoming gradient on the device (the kernels run with scale 1
        and their results are multiplied by it)."""

        @staticmethod
        def forward(ctx, c, x, u, ep):
            J = eval_sum(ep.eval, x, ep.conn, material=c, dofs=u)
            ctx.ep = ep
            ctx.save_for_backward(c, x, u)
            return J

        @staticmethod
        def backward(ctx, gJ):
            c, x, u = ctx.saved_tensors
            ep = ctx.ep
            gc = gx = gu = None
            need_c, need_x, need_u = ctx.needs_input_grad[:3]
            if need_c or need_x:
                gc, gx = _energy_grad(ep.eval, ep.inc, x, ep.conn, c, u, 1.0,
                                      want_mat=need_c, want_coords=need_x,
                                      ws=ep.grad_workspace(x.device),
                                      check=False)
            if need_u:
                r = ep.resid(x, ep.conn, material=c, dofs=u)
                gu = assemble(ep.inc, r, scale=2.0)
            for g in (gc, gx, gu):
                if g is not None:
                    g.mul_(gJ)
            # the one synchronisation, after every launch of the pass
            ep.check()
            return gc, gx, gu, None

    return _ElasticEnergy


_ELASTIC = None


def ElasticEnergy(c, x, u, ep: ElasticEnergyPlan):
    """Differentiable J(c, x, u) (a torch scalar) on the GPU.  Faults
    (det J <= 0, node numbers out of range) are raised by the backward pass,
    or by ep.check() when no backward pass runs."""
    global _ELASTIC
    if _ELASTIC is None:
        _ELASTIC = _make_energy_function()
    return _ELASTIC.apply(c, x, u, ep)


class Batch:
    """Uneven groups of cells (Q1/Q2 hexahedra, P1/P2 tetrahedra), each with
    its own mesh arrays and a set of forms (mass, Laplace, elasticity), run
    as ONE persistent kernel captured in a HIP graph.

    groups: list of dicts with keys cell, order, forms (iterable of
    "mass"/"laplace"/"elasticity"), coords, conn, material (lambda, mu per
    cell, for elasticity) and optionally tile.  Outputs are allocated here:
    batch.outputs[i][form] -> (n_cells, nd, nd) tensor."""

    def __init__(self, groups, precision: str = "fp32", autotune: bool = True,
                 cache: bool = True):
        """autotune: time tile candidates per group (fe_batch_create); with
        cache, tiles tuned before for the same groups on the same GPU
        architecture, ROCm and library version are taken from the autotune
        cache (FE_CACHE) instead, and new ones are stored there."""
        import torch
        from . import autotune as _at
        self.from_cache = False
        if autotune and cache:
            hit = _at.cached_batch_tiles(groups, precision)
            if hit is not None and len(hit) == len(groups):
                groups = [dict(g, tile=t) for g, t in zip(groups, hit)]
                autotune = False
                self.from_cache = True
        dt = {"fp64": torch.float64, "fp32": torch.float32}[precision]
        self.precision = precision
        self.outputs = []
        self._keep = []
        arr = (_lib.fe_group * len(groups))()
        for i, g in enumerate(groups):
            cell, order = g["cell"], int(g["order"])
            nb, _ = reference_sizes(cell, order)
            X, C = g["coords"], g["conn"]
            if X.dtype != torch.float64 or X.dim() != 2 or X.shape[1] != 3:
                raise ValueError(f"group {i}: coords must be (n_nodes, 3) "
                                 "float64")
            if C.dtype != torch.int32 or C.dim() != 2 or C.shape[1] != nb:
                raise ValueError(f"group {i}: conn must be (n_cells, {nb}) "
                                 "int32")
            n = C.shape[0]
            forms = set(g["forms"])
            unknown = forms - {"mass", "laplace", "elasticity"}
            if unknown:
                raise ValueError(f"group {i}: unknown forms {sorted(unknown)}")
            for name, t in (("coords", X), ("conn", C)):
                if not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"group {i}: {name} must be a "
                                     "contiguous cuda tensor")
            outs = {}
            mask = 0
            for f in forms:
                mask |= 1 << _lib.FORMS[f]
                nd = 3 * nb if f == "elasticity" else nb
                outs[f] = torch.empty((n, nd, nd), dtype=dt, device=X.device)
            mat = g.get("material")
            if mat is not None and mat.dtype != dt:
                raise ValueError(f"material must be {dt}")
            if "elasticity" in forms:
                if mat is None or mat.numel() != 2 * n or not mat.is_cuda \
                        or not mat.is_contiguous():
                    raise ValueError(f"group {i}: elasticity needs a "
                                     f"contiguous cuda (n_cells, 2) material")
            arr[i] = _lib.fe_group(
                _lib.CELLS[cell], order, mask, int(g.get("tile", 0)), n,
                X.shape[0], X.data_ptr(), C.data_ptr(),
                mat.data_ptr() if mat is not None else None,
                outs["mass"].data_ptr() if "mass" in outs else None,
                outs["laplace"].data_ptr() if "laplace" in outs else None,
                outs["elasticity"].data_ptr() if "elasticity" in outs
                else None)
            self.outputs.append(outs)
            self._keep += [X, C, mat]
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().fe_batch_create(len(groups), arr,
                                              _lib.PRECS[precision],
                                              1 if autotune else 0,
                                              ctypes.byref(h)),
                   "fe_batch_create")
        self._h = h
        tiles = (ctypes.c_int * len(groups))()
        ms, grid = ctypes.c_float(), ctypes.c_int()
        _lib.check(_lib.lib().fe_batch_tiles(h, tiles, ctypes.byref(ms),
                                             ctypes.byref(grid)),
                   "fe_batch_tiles")
        self.tiles = list(tiles)
        self.tuned_ms = ms.value
        self.grid = grid.value
        if autotune and cache:
            _at.store_batch_tiles(groups, precision, self.tiles, self.tuned_ms)

    def run(self, stream=None):
        _lib.check(_lib.lib().fe_batch_execute(self._h,
                                               _stream_handle(stream)),
                   "fe_batch_execute")
        return self.outputs

    def check(self, stream=None):
        _lib.check(_lib.lib().fe_batch_check(self._h, _stream_handle(stream)),
                   "fe_batch_check")

    def __del__(self):
        # the library handle is looked up defensively: at interpreter exit
        # module globals may already be gone
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.fe_batch_destroy(h)
            self._h = None


from .bilinear import BilinearPlan  # noqa: E402  (uses the helpers above)
