"""Plan creation over every (cell, order, form, mode, precision, material
kind) agrees with the support table documented at fe_plan_create: the
documented combinations get a plan, every other one is refused with
FE_ERR_UNSUPPORTED (never a silent fallback)."""
import itertools

import pytest

pytestmark = pytest.mark.gpu

KINDS = {"elasticity": ["iso_cell", "iso_qp", "voigt_qp"], "wdot": ["tensor_qp"]}
FORMS = ["mass", "vmass", "laplace", "elasticity", "wdot", "convect"]
CELLS = [("hex", p) for p in range(1, 6)] + [("tet", 1), ("tet", 2)]


def documented(cell, p, form, mode, prec, kind):
    if mode in ("residual", "eval"):
        return prec in ("fp64", "fp32")
    if prec in ("fp64", "fp32"):
        return True
    # bf16x3 matrices
    return (cell == "hex" and 2 <= p <= 5 and
            (form in ("mass", "vmass", "laplace") or (form == "elasticity" and kind == "iso_cell")))


def test_support_table():
    import paper_2107_04121_amd as fe
    mismatches = []
    n = 0
    for (cell, p), form, mode, prec in itertools.product(CELLS, FORMS, ["matrix", "residual", "eval"],
                                                         ["fp64", "fp32", "bf16x3"]):
        for kind in KINDS.get(form, [None]):
            n += 1
            want = documented(cell, p, form, mode, prec, kind)
            try:
                fe.Plan(cell, p, form, mode, prec, material=kind)
                got = True
            except fe.FeError as ex:
                if ex.status != 2:
                    mismatches.append((cell, p, form, mode, prec, kind, f"status {ex.status}"))
                    continue
                got = False
            if got != want:
                mismatches.append((cell, p, form, mode, prec, kind, "plan" if got else "refused"))
    print(f"[support] {n} combinations checked", flush=True)
    assert not mismatches, mismatches
