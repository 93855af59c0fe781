"""Front-end for the generalized einsum-like weak-form notation.

An expression in the paper's notation (the table of the generalized
notation: ``0`` scalar, ``i`` vector component, ``0.i`` / ``i.j`` gradient,
``i.i`` divergence, ``s(i:j)->I`` symmetric gradient in vector storage;
material arrays named by their index letters) with its arguments, e.g.::

    ('0.i,0.i', 'v', 'u')                       weak Laplacian
    ('ij,i,j', 'M', 'v', 'u')                   weighted vector dot product
    ('i,i.j,j', 'v', 'u', 'u')                  Navier-Stokes convection
    ('IK,s(i:j)->I,s(k:l)->K', 'D', 'v', 'u')   linear elasticity
    ('i.i,0', 'v', 'p')                         Stokes coupling

is parsed term by term and transpiled to plain einsum expressions over the
operands of the paper's expression examples (``det`` = w |J| per cell and
point, ``bf`` basis values, physical gradients ``bfg``, the identity ``I``,
the symmetric-gradient extractor ``Psg``, material arrays, the cell DOFs
``dofs``), for each evaluation mode, following the weak form evaluation
function of the transpiler section:

1. transpile: every term contributes its operands -- a value term the basis
   values (and, for a vector, an identity that names its component), a
   gradient term the physical gradients, a symmetric gradient the gradients
   and the extractor, a material its array over cells and points; the test
   variable's operands come first after ``det``;
2. the mode decides which variables keep their local DOF axis in the output
   (the test variable in 'residual' and 'matrix' mode, the variable the
   matrix is the derivative by in 'matrix' mode) and which are bound to their
   DOFs (the rest; all of them in 'eval' mode); a non-linear form whose
   unknown appears twice gives one matrix expression per appearance (their
   sum is the derivative, eq. fe4);
3. layout: the letters of the layout table (c cells, q points, g gradient
   component, v variable component, d local DOF, 0 material axes) permute
   every data operand's axes; the cell axis of the output goes first, or
   last when the layout ends with c;
4. paths: every expression is given its cheapest pairwise contraction path
   under the flop model of `contraction`;
5. evaluation: the expression's structure -- the operator on the test and
   on the unknown (value, gradient, divergence, symmetric gradient), their
   component counts and the constant coupling between them that the
   identity and extractor operands leave after contraction -- selects the
   kernel: a dedicated one of the library where it has one (mass, vector
   mass, Laplacian, weighted dot, elasticity, convection), otherwise the
   library's generic bilinear kernel, which takes the derived coupling as
   tables.  Every contraction runs in the library's kernels.

Letters (a reading: the paper prints its examples but not its lettering
rule; these rules reproduce the printed expressions): ``c`` cells, ``q``
points; the local DOF axis of the argument at position k is ``'defgh'[k]``;
component axes that stay in the output take ``r, s, t, ...`` in order; the
index letters of the expression name contracted component and derivative
axes, except that a scalar gradient's letter is written as the next letter
the expression leaves free (the weak Laplacian '0.i,0.i' prints as
'cq,cqjd,cqje->cde').  Argument names starting with an upper-case letter are
materials, the others variables; the first variable is the test function.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np

from .contraction import optimal_path

__all__ = ["Term", "Transpiled", "transpile", "apply_layout", "WeakForm", "DEFAULT_LAYOUT"]

DEFAULT_LAYOUT = "cqgvd0"
_DOF_LETTERS = "defgh"
_AUX_LETTERS = "rstuvwxyz"


@dataclass(frozen=True)
class Term:
    """One term of an expression: kind is 'scalar', 'sgrad' (gradient of a
    scalar), 'vector', 'vgrad' (gradient of a vector), 'div' (divergence),
    'sym' (symmetric gradient in vector storage) or 'material'; idx are its
    index letters; arg its argument name."""
    kind: str
    idx: tuple
    arg: str


@dataclass(frozen=True)
class Operand:
    """One einsum operand: its subscript, its name (det, bf, bfg, I, Psg,
    dofs or a material name), the variable or material it belongs to and
    the role of each axis (letters of the layout table)."""
    sub: str
    name: str
    owner: str
    roles: str


def _is_material(arg: str) -> bool:
    return arg[:1].isupper()


_PATTERNS = [
    ("scalar", re.compile(r"^0$")),
    ("sgrad", re.compile(r"^0\.([a-z])$")),
    ("vgrad", re.compile(r"^([a-z])\.([a-z])$")),
    ("sym", re.compile(r"^s\(([a-z]):([a-z])\)->([A-Z])$")),
    ("letters", re.compile(r"^([A-Za-z]+)$")),
]


def _parse_term(text: str, arg: str) -> Term:
    t = text.strip()
    for kind, pat in _PATTERNS:
        m = pat.match(t)
        if not m:
            continue
        if kind == "letters":
            if _is_material(arg):
                return Term("material", tuple(m.group(1)), arg)
            if len(t) == 1 and t.islower():
                return Term("vector", (t,), arg)
            break
        if _is_material(arg):
            raise ValueError(f"material {arg!r} given the variable term {text!r}")
        if kind == "vgrad" and m.group(1) == m.group(2):
            return Term("div", (m.group(1),), arg)
        if kind == "sym" and m.group(1) == m.group(2):
            raise ValueError(f"cannot parse term {text!r}")
        return Term(kind, tuple(m.groups()), arg)
    raise ValueError(f"cannot parse term {text!r} of argument {arg!r}")


# operator kind of each variable term and the axes it contributes
_OP_OF = {"scalar": "value", "vector": "value", "sgrad": "grad", "vgrad": "grad", "div": "div", "sym": "sym"}


@dataclass
class Transpiled:
    """A parsed expression with its einsum expressions per mode.

    einsum[mode] is a list of (expression, operand names) whose sum is the
    mode's result (one entry, or one per appearance of the unknown for the
    matrix of a non-linear form); operands[mode] holds the same with full
    Operand records; paths[mode] the cheapest contraction path of each
    expression at the sizes given to `paths_for`."""
    expr: str
    args: tuple
    terms: tuple
    test: str | None
    unknown: str | None
    material: str | None
    einsum: dict = field(default_factory=dict)
    operands: dict = field(default_factory=dict)
    outputs: dict = field(default_factory=dict)
    form: str | None = None          # the library form with a dedicated kernel, or None
    structure: dict = field(default_factory=dict)
    reason: str = ""                 # why no kernel evaluates it, if none does

    @property
    def n_comp(self) -> int:
        return self.structure.get("trial_comp") or self.structure.get("test_comp") or 1

    @property
    def linear(self) -> bool:
        return sum(1 for t in self.terms if t.kind != "material" and t.arg == self.unknown) <= 1

    @property
    def material_kinds(self) -> tuple:
        return {"elasticity": ("voigt_qp", "iso_cell", "iso_qp"), "wdot": ("tensor_qp",)}.get(self.form, ())

    def paths_for(self, mode: str, sizes: dict):
        """Cheapest pairwise contraction path (a contraction.PathInfo) of
        every expression of the mode at the given index sizes."""
        out = []
        for expr, _ in self.einsum[mode]:
            s = {ch: sizes[ch] for ch in set(expr) if ch.isalpha()}
            out.append(optimal_path(expr, s))
        return out


class _Builder:
    """Letters and operands of one expression in one mode."""

    def __init__(self, terms, args):
        self.terms, self.args = terms, args
        used = set()
        for t in terms:
            used |= set(t.idx)
        self.used = used
        self.aux = iter(_AUX_LETTERS)
        self.sgrad_letter = {}
        for t in terms:  # a scalar gradient's letter is renamed everywhere
            if t.kind == "sgrad":
                self.grad_letter(t.idx[0])

    def L(self, ch):
        """The letter written for the expression's index letter ch."""
        return self.sgrad_letter.get(ch, ch)

    def dof_letter(self, term_pos):
        return _DOF_LETTERS[term_pos]

    def grad_letter(self, x):
        """The scalar gradient's derivative letter: the next letter after x
        that the expression does not use and no rule reserves."""
        if x not in self.sgrad_letter:
            reserved = set("cq") | set(_DOF_LETTERS) | set(_AUX_LETTERS) | self.used | set(self.sgrad_letter.values())
            ch = x
            while True:
                ch = chr(ord(ch) + 1)
                if ch > "z":
                    raise ValueError("no free letter for a scalar gradient")
                if ch not in reserved:
                    break
            self.sgrad_letter[x] = ch
        return self.sgrad_letter[x]


def _variable_operands(b, t, pos, bound):
    """Operands of variable term t (argument position pos); bound = its DOFs
    are contracted in (else its DOF axis, and its component axis, stay in
    the output).  Returns (operands, output letters, row letters) where the
    row letters are the component and derivative letters of its operator."""
    D = b.dof_letter(pos)
    ops, out = [], ""
    comp = deriv = None
    if t.kind == "scalar":
        ops.append(Operand("q" + D, "bf", t.arg, "qd"))
        if bound:
            ops.append(Operand("c" + D, "dofs", t.arg, "cd"))
    elif t.kind == "sgrad":
        g = b.grad_letter(t.idx[0])
        deriv = g
        ops.append(Operand("cq" + g + D, "bfg", t.arg, "cqgd"))
        if bound:
            ops.append(Operand("c" + D, "dofs", t.arg, "cd"))
    elif t.kind in ("vector", "vgrad", "div"):
        x = b.L(t.idx[0])
        if t.kind == "vector":
            ops.append(Operand("q" + D, "bf", t.arg, "qd"))
        else:
            deriv = b.L(t.idx[1]) if t.kind == "vgrad" else x
            ops.append(Operand("cq" + deriv + D, "bfg", t.arg, "cqgd"))
        if bound:
            ops.append(Operand("c" + x + D, "dofs", t.arg, "cvd"))
        else:
            comp = next(b.aux)
            ops.append(Operand(x + comp, "I", t.arg, "vv"))
    elif t.kind == "sym":
        x, y, Z = (b.L(ch) for ch in t.idx)
        comp = next(b.aux)
        deriv = y
        ops.append(Operand("cq" + y + D, "bfg", t.arg, "cqgd"))
        ops.append(Operand(comp + y + Z, "Psg", t.arg, "vg0"))
        if bound:
            ops.append(Operand("c" + comp + D, "dofs", t.arg, "cvd"))
    else:
        raise AssertionError(t.kind)
    if not bound:
        out = (comp or "") + D
    return ops, out, (comp, deriv)


def _build(terms, args, mode, diff_pos=None):
    """Operands and output of one expression.  Variable occurrence positions
    are term positions; the test is the first variable term; diff_pos is
    the term position the matrix is the derivative by."""
    b = _Builder(terms, args)
    var_pos = [k for k, t in enumerate(terms) if t.kind != "material"]
    test_pos = var_pos[0]
    order = [test_pos] + [k for k in range(len(terms)) if k != test_pos]
    ops = [Operand("cq", "det", "", "cq")]
    out = "c"
    rows = {}
    for k in order:
        t = terms[k]
        if t.kind == "material":
            ops.append(Operand("cq" + "".join(b.L(ch) for ch in t.idx), t.arg, t.arg, "cq" + "0" * len(t.idx)))
            continue
        if mode == "eval":
            bound = True
        elif k == test_pos:
            bound = False
        else:
            bound = not (mode == "matrix" and k == diff_pos)
        o, letters, row = _variable_operands(b, t, k, bound)
        ops += o
        out += letters
        rows[k] = row
    expr = ",".join(o.sub for o in ops) + "->" + out
    return expr, ops, out, rows


def _coupling(terms, test_pos, trial_pos, ops, rows):
    """The constant part of a bilinear form's coupling: with the basis
    operands of the test and of the unknown taken out, the identity and
    extractor operands (and, where the test and the unknown share a
    derivative letter, the identity on it) map the test's (component,
    derivative) axes and the unknown's to each other or to the material
    axes.  Returns (P_test, P_trial, W0, material letters on each side)
    with P_test[(r, j), a] (rows component-major, derivative fastest),
    P_trial likewise, and W0 the full coupling when there is no material."""
    tv, tu = terms[test_pos], terms[trial_pos]
    nct = 3 if tv.kind in ("vector", "vgrad", "div", "sym") else 1
    ncu = 3 if tu.kind in ("vector", "vgrad", "div", "sym") else 1
    ndt = 1 if _OP_OF[tv.kind] == "value" else 3
    ndu = 1 if _OP_OF[tu.kind] == "value" else 3
    (ct, gt), (cu, gu) = rows[test_pos], rows[trial_pos]
    consts = [o for o in ops if o.name in ("I", "Psg")]
    mats = [o for o in ops if o.name not in ("I", "Psg", "det", "bf", "bfg", "dofs")]
    I3 = np.eye(3)
    P = np.zeros((3, 3, 6))
    for K, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        P[i, j, K] = P[j, i, K] = 1.0
    arrays = {"I": I3, "Psg": P}
    # rename the unknown's derivative letter when it is also the test's
    rename = {}
    if gt is not None and gu is not None and gt == gu:
        rename[gu] = "Z"
    const_subs, const_arrays = [], []
    for o in consts:
        sub = o.sub
        if o.owner == tu.arg:
            sub = "".join(rename.get(ch, ch) for ch in sub)
        const_subs.append(sub)
        const_arrays.append(arrays[o.name])
    if rename:
        const_subs.append(gt + rename[gu])
        const_arrays.append(I3)
    gu2 = rename.get(gu, gu)
    # placeholder letters for absent axes: a value operator has no
    # derivative axis, a scalar no component axis
    row_t = (ct or "") + (gt or "")
    row_u = (cu or "") + (gu2 or "")
    if not mats:
        subs = ",".join(const_subs) if const_subs else ""
        if subs:
            W = np.einsum(subs + "->" + row_t + row_u, *const_arrays) if (row_t + row_u) else \
                np.einsum(subs + "->", *const_arrays)
        else:
            W = np.ones(())
        W = np.asarray(W, dtype=float).reshape(nct * ndt if row_t else 1, ncu * ndu if row_u else 1)
        return None, None, W, None
    if len(mats) != 1 or len(mats[0].sub) != 4:
        raise NotImplementedError("the generic bilinear kernel takes one two-index material per point")
    m = mats[0].sub[2:]
    # split constants by side: those touching the test's row letters
    side_t = [(s, a) for s, a, o in zip(const_subs, const_arrays, consts) if o.owner == tv.arg]
    side_u = [(s, a) for s, a, o in zip(const_subs, const_arrays, consts) if o.owner != tv.arg]
    letters_t = set(row_t)
    mt = [ch for ch in m if any(ch in s for s, _ in side_t) or ch in letters_t]
    mu = [ch for ch in m if ch not in mt]
    if len(mt) != 1 or len(mu) != 1:
        raise NotImplementedError("the material must couple one test axis with one unknown axis")

    def proj(side, row, letter, n_rows):
        if side:
            Pm = np.einsum(",".join(s for s, _ in side) + "->" + row + letter, *[a for _, a in side])
        else:  # the material letter is the row letter itself
            Pm = np.eye(3)
        return np.asarray(Pm, dtype=float).reshape(n_rows, -1)

    Pt = proj(side_t, row_t, mt[0], nct * ndt)
    Pu = proj(side_u, row_u, mu[0], ncu * ndu)
    return Pt, Pu, None, (m.index(mt[0]), m.index(mu[0]))


def transpile(expr: str, *args: str) -> Transpiled:
    """Parse an expression of the generalized notation with its argument
    names and derive its einsum expressions in every mode.  Raises
    ValueError for malformed input and NotImplementedError for expressions
    no kernel of the library evaluates (with the reason)."""
    parts = expr.split(",")
    if len(parts) != len(args):
        raise ValueError(f"{expr!r} has {len(parts)} terms but {len(args)} arguments were given")
    if len(args) > len(_DOF_LETTERS):
        raise ValueError("too many arguments")
    terms = tuple(_parse_term(p, a) for p, a in zip(parts, args))
    var_pos = [k for k, t in enumerate(terms) if t.kind != "material"]
    if not var_pos:
        raise ValueError("an expression needs at least one variable")
    # index letters: every letter must be contracted (a weak form integrates
    # to a scalar per test function) -- appear exactly twice -- except the
    # one-letter derivative of a divergence
    counts = {}
    for t in terms:
        if t.kind == "div":
            letters = (t.idx[0], t.idx[0])
        elif t.kind == "sym":
            letters = (t.idx[2],)  # i, j are absorbed into the storage index
        else:
            letters = t.idx
        for ch in letters:
            counts[ch] = counts.get(ch, 0) + 1
    free = sorted(ch for ch, n in counts.items() if n != 2)
    if free:
        raise ValueError(f"indices {free} are not contracted exactly once: the expression is not a scalar integrand")
    test = terms[var_pos[0]].arg
    others = [terms[k].arg for k in var_pos[1:]]
    if test in others:
        raise ValueError("the first variable is the test function and must differ from the unknown")
    unknowns = sorted(set(others))
    if len(unknowns) > 1:
        raise NotImplementedError(f"more than one unknown ({unknowns}): the library evaluates forms of one "
                                  "unknown")
    unknown = unknowns[0] if unknowns else None
    materials = [t.arg for t in terms if t.kind == "material"]
    t = Transpiled(expr=expr, args=args, terms=terms, test=test, unknown=unknown,
                   material=materials[0] if materials else None)
    occ = [k for k in var_pos[1:]]
    modes = ["residual", "eval"] + (["matrix"] if occ else [])
    for mode in modes:
        entries = []
        diffs = occ if mode == "matrix" else [None]
        for dpos in diffs:
            e, ops, out, rows = _build(terms, args, mode, dpos)
            entries.append((e, ops, out, rows))
        t.einsum[mode] = [(e, [o.name for o in ops]) for e, ops, _, _ in entries]
        t.operands[mode] = [ops for _, ops, _, _ in entries]
        t.outputs[mode] = [out for _, _, out, _ in entries]
    _classify(t)
    return t


def _classify(t: Transpiled):
    """Derive the structure of the form and the library kernel that
    evaluates it (t.form for a dedicated kernel, 'bilinear' structure for
    the generic one, else t.reason)."""
    terms = t.terms
    var_pos = [k for k, x in enumerate(terms) if x.kind != "material"]
    test_pos = var_pos[0]
    occ = var_pos[1:]
    tv = terms[test_pos]
    ncomp = {"scalar": 1, "sgrad": 1}.get
    st = dict(test_op=_OP_OF[tv.kind], test_comp=ncomp(tv.kind, 3), n_unknown=len(occ))
    t.structure = st
    if len(occ) == 0:
        t.reason = "a linear form without an unknown: the library evaluates forms of an unknown"
        return
    if len(occ) == 2:
        # trilinear: the convection v_i du_i/dx_j u_j with both u the unknown
        a, b2 = terms[occ[0]], terms[occ[1]]
        conv = (tv.kind == "vector" and a.kind == "vgrad" and b2.kind == "vector"
                and a.idx[0] == tv.idx[0] and a.idx[1] == b2.idx[0] and not t.material)
        if conv:
            t.form = "convect"
            st.update(trial_op="grad", trial_comp=3, kernel="convect")
        else:
            t.reason = "a non-linear form other than the convection 'i,i.j,j': no kernel"
        return
    if len(occ) > 2:
        t.reason = "forms of degree above three are not evaluated"
        return
    tu = terms[occ[0]]
    st.update(trial_op=_OP_OF[tu.kind], trial_comp=ncomp(tu.kind, 3))
    ops = t.operands["matrix"][0]
    _, _, _, rows = _build(terms, t.args, "matrix", occ[0])
    try:
        Pt, Pu, W0, mside = _coupling(terms, test_pos, occ[0], ops, rows)
    except NotImplementedError as e:
        t.reason = str(e)
        return
    st.update(P_test=Pt, P_trial=Pu, W0=W0, material_sides=mside)
    key = (st["test_op"], st["test_comp"], st["trial_op"], st["trial_comp"])
    eye = lambda n: W0 is not None and W0.shape == (n, n) and np.array_equal(W0, np.eye(n))  # noqa: E731
    if key == ("value", 1, "value", 1) and eye(1):
        t.form = "mass"
    elif key == ("value", 3, "value", 3) and eye(3):
        t.form = "vmass"
    elif key == ("grad", 1, "grad", 1) and eye(3):
        t.form = "laplace"
    elif key == ("value", 3, "value", 3) and Pt is not None and mside == (0, 1) and \
            np.array_equal(Pt, np.eye(3)) and np.array_equal(Pu, np.eye(3)):
        t.form = "wdot"
    elif key == ("sym", 3, "sym", 3) and Pt is not None and mside == (0, 1) and Pt.shape == (9, 6) and \
            np.array_equal(Pt, Pu):
        t.form = "elasticity"
    st["kernel"] = t.form or "bilinear"


def apply_layout(t: Transpiled, mode: str, layout: str = DEFAULT_LAYOUT):
    """The mode's einsum expressions with every data operand's axes permuted
    into the order of the layout letters (c, q, g, v, d, 0; the constant
    identity and extractor operands keep theirs) and the output's cell axis
    first, or last when the layout ends with c.  Returns (expressions,
    output cell position 'first' | 'last')."""
    if sorted(layout) != sorted(DEFAULT_LAYOUT):
        raise ValueError("layout must be a permutation of the letters c, q, g, v, d, 0")
    rank = {ch: k for k, ch in enumerate(layout)}
    out_exprs = []
    cell_last = layout[-1] == "c"
    for ops, out in zip(t.operands[mode], t.outputs[mode]):
        subs = []
        for o in ops:
            if o.name in ("I", "Psg"):
                subs.append(o.sub)
                continue
            axes = sorted(range(len(o.sub)), key=lambda k: (rank[o.roles[k]], k))
            subs.append("".join(o.sub[k] for k in axes))
        o2 = (out[1:] + "c") if cell_last and len(out) > 1 else out
        out_exprs.append(",".join(subs) + "->" + o2)
    return out_exprs, ("last" if cell_last and len(t.outputs[mode][0]) > 1 else "first")


def layout_support(t: Transpiled, mode: str, layout: str):
    """(supported, reason): the library reads material arrays as
    [cell][point][axes] and writes outputs with the cell axis first, or last
    for residuals of the sum-factorized kernels; the other data operands
    (det, bf, bfg, the cell DOFs) live in registers and LDS only, so their
    order is free."""
    if sorted(layout) != sorted(DEFAULT_LAYOUT):
        return False, "layout must be a permutation of the letters c, q, g, v, d, 0"
    rank = {ch: k for k, ch in enumerate(layout)}
    if t.material and not (rank["c"] < rank["q"] < rank["0"]):
        return False, "material arrays are read cell-major: [cell][point][material axes] (c before q before 0)"
    if layout[0] == "c":
        return True, "cell-major output"
    if layout[-1] == "c":
        if mode == "residual":
            return True, "cell-minor residual output (sum-factorized kernels)"
        return False, f"{mode} outputs are written with the cell axis first"
    return False, "outputs are written with the cell axis first (or last for residuals)"


_MODES = ("matrix", "residual", "eval")


class WeakForm:
    """A transpiled expression bound to a cell kind, order and precision,
    evaluated by the C library (one plan per mode, created on first use).

        wf = WeakForm(('i,i.j,j', 'v', 'u', 'u'), 'hex', 2)
        K = wf(coords, conn, mode='matrix', dofs=U)   # derivative at U
        r = wf(coords, conn, mode='residual', dofs=U)
    """

    def __init__(self, expression, cell: str, order: int, precision: str = "fp64",
                 material_kind: str | None = None, layout: str = DEFAULT_LAYOUT, variant: str = "auto"):
        if isinstance(expression, str):
            expression = (expression,)
        self.t = transpile(*expression)
        if self.t.structure.get("kernel") is None:
            raise NotImplementedError(f"no kernel for {self.t.expr!r}: {self.t.reason}")
        kinds = self.t.material_kinds
        if self.t.form is None:  # the generic bilinear kernel
            if material_kind not in (None, "tensor_qp"):
                raise ValueError("the generic bilinear kernel takes a per-point matrix material (tensor_qp)")
            if self.t.material:
                material_kind = "tensor_qp"
        elif kinds:
            material_kind = material_kind or kinds[0]
            if material_kind not in kinds:
                raise ValueError(f"{self.t.form} takes material kinds {kinds}")
        elif material_kind is not None:
            raise ValueError(f"{self.t.form} takes no material")
        ok, why = layout_support(self.t, "residual", layout)
        if sorted(layout) != sorted(DEFAULT_LAYOUT):
            raise ValueError(why)
        if not ok:
            raise NotImplementedError(f"layout {layout!r}: {why}")
        self.layout = "cell_minor" if layout[-1] == "c" else "cell_major"
        self.layout_letters = layout
        self.cell, self.order, self.precision = cell, order, precision
        self.material_kind, self.variant = material_kind, variant
        self._plans = {}

    @property
    def form(self) -> str:
        return self.t.form or "bilinear"

    def einsum(self, mode: str):
        """The einsum expressions (with operand names) of a mode."""
        return self.t.einsum[mode]

    def plan(self, mode: str):
        from . import Plan
        if mode not in _MODES:
            raise ValueError(f"mode must be one of {_MODES}")
        if mode not in self.t.einsum:
            raise ValueError(f"{self.t.expr!r} has no {mode} mode")
        ok, why = layout_support(self.t, mode, self.layout_letters)
        if not ok:
            raise NotImplementedError(f"layout {self.layout_letters!r} in {mode} mode: {why}")
        if mode not in self._plans:
            layout = self.layout if mode == "residual" else "cell_major"
            if self.t.form is None:
                from . import BilinearPlan
                self._plans[mode] = BilinearPlan(self.t, self.cell, self.order, mode, self.precision)
            else:
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
