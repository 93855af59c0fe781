"""Front-end for the generalized einsum-like weak-form notation.

An expression in the paper's notation (the table of notation symbols:
``0`` scalar, ``i`` vector component, ``0.i`` / ``i.j`` gradient, ``i:j``
symmetric gradient stored as ``s(i:j)->I``; material arrays named by their
index letters) together with its arguments, e.g.::

    ('0.i,0.i', 'v', 'u')                       weak Laplacian
    ('ij,i,j', 'M', 'v', 'u')                   weighted vector dot product
    ('i,i.j,j', 'v', 'u', 'u')                  Navier-Stokes convection
    ('IK,s(i:j)->I,s(k:l)->K', 'D', 'v', 'u')   linear elasticity

is parsed into terms, its index letters are renamed canonically, and it is
matched to one of the forms the C library evaluates.  The result gives

* the plain einsum expressions the form stands for in matrix, residual and
  eval mode, over the operands named in the section on expression examples
  (``det`` = w |J| per cell and point, ``bf``, physical ``bfg``, ``I``,
  ``Psg``, the material arrays, ``dofs``; for the convection also the state
  at the points, ``uq`` and ``guq``), with the convection matrix as the sum
  of two expressions (eq. fe4);
* plans of the C library for each mode (`WeakForm`), which are what is
  evaluated: every contraction runs in the library's kernels.

Layouts are given with the letters of the layout table (c cells, q points, g
gradient component, v variable component, d local DOF, 0 material axes); the
library's element-major output is the default 'cqgvd0', and for residuals
the cell axis may be last (cell-minor output of the sum-factorized kernels).
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

__all__ = ["Term", "Transpiled", "transpile", "WeakForm"]


@dataclass(frozen=True)
class Term:
    """One operand of an expression: kind is 'scalar', 'sgrad' (gradient of
    a scalar), 'vector', 'vgrad' (gradient of a vector), 'sym' (stored
    symmetric gradient) or 'material'; idx are its index letters."""
    kind: str
    idx: tuple
    arg: str


_PATTERNS = [
    ("scalar", re.compile(r"^0$")),
    ("sgrad", re.compile(r"^0\.([a-z])$")),
    ("vector", re.compile(r"^([a-z])$")),
    ("vgrad", re.compile(r"^([a-z])\.([a-z])$")),
    ("sym", re.compile(r"^s\(([a-z]):([a-z])\)->([A-Z])$")),
    ("material", re.compile(r"^([A-Za-z]{2,})$")),
]


def _parse_term(text: str, arg: str) -> Term:
    t = text.strip()
    for kind, pat in _PATTERNS:
        m = pat.match(t)
        if m:
            idx = tuple(m.groups()) if kind != "material" else tuple(m.group(1))
            return Term(kind, idx, arg)
    raise ValueError(f"cannot parse term {text!r}")


# einsum expressions of each form and mode, with their operand names
_EINSUM = {
    "mass": {
        "matrix": [("cq,qd,qe->cde", ["det", "bf", "bf"])],
        "residual": [("cq,qd,qe,ce->cd", ["det", "bf", "bf", "dofs"])],
        "eval": [("cq,qd,cd,qe,ce->c", ["det", "bf", "dofs", "bf", "dofs"])],
    },
    "vmass": {
        "matrix": [("cq,qd,ir,qe,is->crdse", ["det", "bf", "I", "bf", "I"])],
        "residual": [("cq,qd,ir,qe,cie->crd", ["det", "bf", "I", "bf", "dofs"])],
        "eval": [("cq,qd,cid,qe,cie->c", ["det", "bf", "dofs", "bf", "dofs"])],
    },
    "laplace": {
        "matrix": [("cq,cqjd,cqje->cde", ["det", "bfg", "bfg"])],
        "residual": [("cq,cqjd,cqje,ce->cd", ["det", "bfg", "bfg", "dofs"])],
        "eval": [("cq,cqjd,cd,cqje,ce->c", ["det", "bfg", "dofs", "bfg", "dofs"])],
    },
    "elasticity": {
        "matrix": [("cq,cqje,rjI,cqIK,cqlf,slK->cresf", ["det", "bfg", "Psg", "D", "bfg", "Psg"])],
        "residual": [("cq,cqje,rjI,cqIK,cqlf,slK,csf->cre", ["det", "bfg", "Psg", "D", "bfg", "Psg", "dofs"])],
        "eval": [("cq,cqje,rjI,cre,cqIK,cqlf,slK,csf->c",
                  ["det", "bfg", "Psg", "dofs", "D", "bfg", "Psg", "dofs"])],
    },
    "wdot": {
        "matrix": [("cq,cqrs,qd,qe->crdse", ["det", "M", "bf", "bf"])],
        "residual": [("cq,cqrs,qd,qe,cse->crd", ["det", "M", "bf", "bf", "dofs"])],
        "eval": [("cq,cqrs,qd,crd,qe,cse->c", ["det", "M", "bf", "dofs", "bf", "dofs"])],
    },
    "convect": {
        # eq. fe4: the two terms left when either u is omitted
        "matrix": [("cq,qd,rs,cqj,cqje->crdse", ["det", "bf", "I", "uq", "bfg"]),
                   ("cq,qd,cqrs,qe->crdse", ["det", "bf", "guq", "bf"])],
        "residual": [("cq,qd,cqrj,cqj->crd", ["det", "bf", "guq", "uq"])],
        "eval": [("cq,cqr,cqrj,cqj->c", ["det", "uq", "guq", "uq"])],
    },
}

# the state operands of the convection, themselves contractions of the DOFs
STATE_EINSUM = {"uq": ("qe,cje->cqj", ["bf", "dofs"]),
                "guq": ("cqse,cre->cqrs", ["bfg", "dofs"])}

_N_COMP = {"mass": 1, "laplace": 1, "vmass": 3, "elasticity": 3, "wdot": 3, "convect": 3}
_MATERIAL = {"elasticity": ("voigt_qp", "iso_cell", "iso_qp"), "wdot": ("tensor_qp",)}


@dataclass
class Transpiled:
    """The parsed expression matched to a library form."""
    expr: str
    terms: tuple
    form: str
    test: str
    unknown: str
    material: str | None = None
    einsum: dict = field(default_factory=dict)

    @property
    def n_comp(self) -> int:
        return _N_COMP[self.form]

    @property
    def material_kinds(self) -> tuple:
        return _MATERIAL.get(self.form, ())

    @property
    def linear(self) -> bool:
        return self.form != "convect"


def _canon(terms):
    """Rename index letters in order of first appearance (lower and upper
    case separately), so that e.g. 'k,k.l,l' and 'i,i.j,j' compare equal."""
    lower, upper = {}, {}
    out = []
    for t in terms:
        idx = []
        for ch in t.idx:
            table, base = (upper, "A") if ch.isupper() else (lower, "a")
            if ch not in table:
                table[ch] = chr(ord(base) + len(table))
            idx.append(table[ch])
        out.append((t.kind, tuple(idx)))
    return tuple(out)


# canonical term structures of the supported forms (variables in argument
# order: test first, then the unknown)
_SIGNATURES = {
    (("scalar", ()), ("scalar", ())): "mass",
    (("vector", ("a",)), ("vector", ("a",))): "vmass",
    (("sgrad", ("a",)), ("sgrad", ("a",))): "laplace",
    (("material", ("a", "b")), ("vector", ("a",)), ("vector", ("b",))): "wdot",
    (("material", ("A", "B")), ("sym", ("a", "b", "A")), ("sym", ("c", "d", "B"))): "elasticity",
    (("vector", ("a",)), ("vgrad", ("a", "b")), ("vector", ("b",))): "convect",
}


def transpile(expr: str, *args: str) -> Transpiled:
    """Parse an expression of the generalized notation with its argument
    names and match it to a library form.  Raises ValueError for malformed
    input and NotImplementedError for forms the library has no kernel for
    (e.g. the Stokes couplings)."""
    parts = [p for p in expr.split(",")]
    if len(parts) != len(args):
        raise ValueError(f"{expr!r} has {len(parts)} terms but {len(args)} arguments were given")
    terms = tuple(_parse_term(p, a) for p, a in zip(parts, args))
    sig = _canon(terms)
    form = _SIGNATURES.get(sig)
    if form is None:
        raise NotImplementedError(f"no kernel for {expr!r}; supported: mass '0,0', vector dot 'i,i', "
                                  "Laplacian '0.i,0.i', weighted dot 'ij,i,j', convection 'i,i.j,j', "
                                  "elasticity 'IK,s(i:j)->I,s(k:l)->K'")
    variables = [t.arg for t in terms if t.kind != "material"]
    materials = [t.arg for t in terms if t.kind == "material"]
    test, unknown = variables[0], variables[1]
    if test == unknown:
        raise ValueError("the first variable is the test function and must differ from the unknown")
    if form == "convect" and variables[2] != unknown:
        raise NotImplementedError("convection is supported with the advection velocity equal to the unknown")
    return Transpiled(expr=expr, terms=terms, form=form, test=test, unknown=unknown,
                      material=materials[0] if materials else None, einsum=_EINSUM[form])


_MODES = ("matrix", "residual", "eval")


class WeakForm:
    """A transpiled expression bound to a cell kind, order and precision,
    evaluated by the C library (one plan per mode, created on first use).

        wf = WeakForm(('i,i.j,j', 'v', 'u', 'u'), 'hex', 2)
        K = wf(coords, conn, mode='matrix', dofs=U)   # derivative at U
        r = wf(coords, conn, mode='residual', dofs=U)
    """

    def __init__(self, expression, cell: str, order: int, precision: str = "fp64",
                 material_kind: str | None = None, layout: str = "cqgvd0", variant: str = "auto"):
        if isinstance(expression, str):
            expression = (expression,)
        self.t = transpile(*expression)
        kinds = self.t.material_kinds
        if kinds:
            material_kind = material_kind or kinds[0]
            if material_kind not in kinds:
                raise ValueError(f"{self.t.form} takes material kinds {kinds}")
        elif material_kind is not None:
            raise ValueError(f"{self.t.form} takes no material")
        if sorted(layout) != sorted("cqgvd0"):
            raise ValueError("layout must be a permutation of the letters c, q, g, v, d, 0")
        if layout[0] == "c":
            self.layout = "cell_major"
        elif layout[-1] == "c":
            self.layout = "cell_minor"
        else:
            raise NotImplementedError("the library stores cells first or last")
        self.cell, self.order, self.precision = cell, order, precision
        self.material_kind, self.variant = material_kind, variant
        self._plans = {}

    @property
    def form(self) -> str:
        return self.t.form

    def einsum(self, mode: str):
        """The einsum expressions (with operand names) of a mode."""
        return self.t.einsum[mode]

    def plan(self, mode: str):
        from . import Plan
        if mode not in _MODES:
            raise ValueError(f"mode must be one of {_MODES}")
        if mode not in self._plans:
            layout = self.layout if mode == "residual" else "cell_major"
            self._plans[mode] = Plan(self.cell, self.order, self.t.form, mode, self.precision,
                                     material=self.material_kind, variant=self.variant, layout=layout)
        return self._plans[mode]

    def __call__(self, coords, conn, mode: str = "matrix", material=None, dofs=None, out=None):
        if mode == "matrix" and self.t.linear and dofs is not None:
            dofs = None  # the matrix of a linear form does not depend on the DOFs
        return self.plan(mode)(coords, conn, material=material, dofs=dofs, out=out)

    def check(self):
        for p in self._plans.values():
            p.check()
