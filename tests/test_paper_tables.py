"""Sizes and shapes the paper prints, checked against this library's
conventions (CPU only): the cell/DOF/size table and the operand shapes of the
expression examples."""
import os

import numpy as np
import pytest

import meshgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("row", _rows("table_cdc.txt"),
                         ids=lambda r: f"{r[0]}xQ{r[1]}")
def test_table_cdc_sizes(orc, row):
    n_c, p, nqp, dofs = (int(v) for v in row[:4])
    r_s, M_s, r_v, M_v = (float(v) for v in row[4:])
    nb, nq = orc.sizes("hex", p)
    assert nq == nqp
    mb = lambda entries: round(entries * 8 / 1e6, 1)  # noqa: E731
    assert mb(n_c * nb) == r_s
    assert mb(n_c * nb * nb) == M_s
    assert mb(3 * n_c * nb) == r_v
    assert mb(9 * n_c * nb * nb) == M_v
    # the paper's mesh: a 1-D bar of n_c hexahedra
    if n_c * nb <= 300_000:
        bar = meshgen.hex_mesh((n_c, 1, 1), p)
        assert bar.n_nodes == dofs
        assert bar.conn.shape == (n_c, nb)


@pytest.mark.parametrize("row", _rows("paper_shapes.txt"),
                         ids=lambda r: r[0])
def test_expression_example_shapes(orc, row):
    name, form, mode, p, n_c = row[0], row[1], row[2], int(row[3]), int(row[4])
    want = tuple(int(v) for v in row[5].split(","))
    bar = meshgen.hex_mesh((n_c, 1, 1), p)
    nb, nq = orc.sizes("hex", p)
    nc = orc.n_comp(form)
    mat, kind = None, None
    if form == "elasticity":
        mat, kind = meshgen.lame_cell(n_c), "iso_cell"
    if mode == "matrix":
        out = orc.matrix(bar, form, mat, kind)
        got = out.reshape((n_c, nc, nb, nc, nb) if nc == 3 else out.shape)
    else:
        U = meshgen.dofs(bar.n_nodes, nc)
        got = orc.residual(bar, form, U, mat, kind)
    assert got.shape == want
    ops = dict(op.split(":") for op in row[6].split(";"))
    sizes = {"det": (n_c, nq), "bfg": (n_c, nq, 3, nb), "bf": (nq, nb),
             "dofs": (n_c, nc, nb), "Psg": (3, 3, 6), "D": (n_c, nq, 6, 6)}
    for k, v in ops.items():
        assert sizes[k] == tuple(int(x) for x in v.split(",")), k
    assert np.isfinite(got).all()
