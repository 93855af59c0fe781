"""Plans of the library's generic bilinear kernel (fe_plan_create_bilinear):
any bilinear form of the generalized notation whose coupling the front-end
derives (transpile.transpile), evaluated without a dedicated kernel.
Argument marshalling only; the evaluation runs in the library."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FeError

__all__ = ["BilinearPlan", "describe"]

_OPS = {"value": 0, "grad": 1, "div": 1, "sym": 1}


def describe(t):
    """The fe_bilinear description of a transpiled bilinear form: operator
    kinds and component counts of the test and the unknown, and the coupling
    tables (W0, or P_test / P_trial with the material's shape)."""
    st = t.structure
    if st.get("kernel") is None or st.get("n_unknown") != 1:
        raise NotImplementedError(f"{t.expr!r} is not a bilinear form of one unknown: {t.reason}")
    d = dict(test_grad=_OPS[st["test_op"]], test_comp=st["test_comp"],
             trial_grad=_OPS[st["trial_op"]], trial_comp=st["trial_comp"])
    if st["W0"] is not None:
        d.update(W0=np.ascontiguousarray(st["W0"], dtype=np.float64), P_test=None, P_trial=None,
                 n_a=0, n_b=0, mat_transpose=0)
    else:
        Pt, Pu = st["P_test"], st["P_trial"]
        d.update(W0=None, P_test=np.ascontiguousarray(Pt, dtype=np.float64),
                 P_trial=np.ascontiguousarray(Pu, dtype=np.float64),
                 n_a=Pt.shape[1], n_b=Pu.shape[1], mat_transpose=1 if st["material_sides"] == (1, 0) else 0)
    return d


class BilinearPlan:
    """A plan of the generic bilinear kernel for one transpiled form, cell
    kind, order, mode and precision (FP64 or FP32).  Called like Plan:
    plan(coords, conn, material=None, dofs=None, out=None)."""

    def __init__(self, t, cell: str, order: int, mode: str = "matrix", precision: str = "fp64"):
        import torch
        self.t, self.cell, self.order, self.mode, self.precision = t, cell, int(order), mode, precision
        d = describe(t)
        self.desc = d
        dp = ctypes.POINTER(ctypes.c_double)

        def ptr(a):
            return None if a is None else a.ctypes.data_as(dp)

        c = _lib.fe_bilinear(d["test_grad"], d["test_comp"], d["trial_grad"], d["trial_comp"],
                             ptr(d["W0"]), ptr(d["P_test"]), ptr(d["P_trial"]), d["n_a"], d["n_b"],
                             d["mat_transpose"])
        self._keep = d
        h = ctypes.c_void_p()
        L = _lib.lib()
        kind = _lib.MATS["tensor_qp"] if d["W0"] is None else 0
        _lib.check(L.fe_plan_create_bilinear(_lib.CELLS[cell], self.order, _lib.MODES[mode],
                                             _lib.PRECS[precision], kind, ctypes.byref(c), None,
                                             ctypes.byref(h)), "fe_plan_create_bilinear")
        self._h = h
        ints = [ctypes.c_int() for _ in range(5)]
        _lib.check(L.fe_plan_info(h, *[ctypes.byref(i) for i in ints]), "fe_plan_info")
        self.n_basis, self.n_qp = ints[0].value, ints[1].value
        self.dtype = getattr(torch, {"fp64": "float64", "fp32": "float32"}[precision])
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.fe_plan_destroy(h)
            self._h = None

    def out_shape(self, n_cells: int):
        nb, d = self.n_basis, self.desc
        if self.mode == "matrix":
            return (n_cells, d["test_comp"] * nb, d["trial_comp"] * nb)
        if self.mode == "residual":
            return (n_cells, d["test_comp"], nb)
        return (n_cells,)

    def material_entries(self):
        d = self.desc
        return d["n_a"] * d["n_b"] * self.n_qp if d["W0"] is None else 0

    def __call__(self, coords, conn, material=None, dofs=None, out=None, workspace=None, stream=None):
        import torch
        from . import _ptr, _stream_handle
        n_cells, nb = conn.shape
        if nb != self.n_basis or conn.dtype != torch.int32:
            raise ValueError(f"conn must be (n_cells, {self.n_basis}) int32")
        if coords.dtype != torch.float64 or coords.dim() != 2 or coords.shape[1] != 3:
            raise ValueError("coords must be (n_nodes, 3) float64")
        per = self.material_entries()
        if per and (material is None or material.numel() != n_cells * per or material.dtype != self.dtype):
            raise ValueError(f"material must hold {per} {self.dtype} entries per cell "
                             f"([cell][point][{self.desc['n_a']}][{self.desc['n_b']}])")
        if self.mode != "matrix":
            nc = self.desc["trial_comp"]
            if dofs is None or dofs.numel() != coords.shape[0] * nc or dofs.dtype != self.dtype:
                raise ValueError(f"dofs must be (n_nodes, {nc}) {self.dtype}")
        for name, x in (("coords", coords), ("conn", conn), ("material", material), ("dofs", dofs)):
            if x is not None and (not x.is_cuda or not x.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous cuda tensor")
        if out is None:
            out = torch.empty(self.out_shape(n_cells), dtype=self.dtype, device=coords.device)
        if workspace is None:
            if self._ws is None or self._ws.device != coords.device:
                self._ws = torch.zeros(256, dtype=torch.uint8, device=coords.device)
            workspace = self._ws
        _lib.check(_lib.lib().fe_execute(self._h, n_cells, coords.shape[0], _ptr(coords), _ptr(conn),
                                         _ptr(material), _ptr(dofs if self.mode != "matrix" else None),
                                         _ptr(out), _ptr(workspace), workspace.numel(),
                                         _stream_handle(stream)), "fe_execute")
        return out

    def check(self, stream=None):
        from . import _ptr, _stream_handle
        if self._ws is None:
            return
        _lib.check(_lib.lib().fe_plan_check(self._h, _ptr(self._ws), _stream_handle(stream)), "fe_plan_check")


FeError = FeError
