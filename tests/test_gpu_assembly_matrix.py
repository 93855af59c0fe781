"""GPU global matrix assembly through the C ABI: the pattern (CSR over nodes)
equals the node graph of the oracle's assembled matrix, bit for bit; the
block-CSR values assembled from the library's element matrices match the
oracle's assembly of the oracle's element matrices (FP64 1e-12, FP32 1e-5 of
the largest entry); two runs agree bitwise; a bad connectivity is reported."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _mesh(cell, p):
    if cell == "hex":
        return meshgen.hex_mesh((5, 4, 3), p, alpha=0.15, seed=80 + p, curved=0.04)
    return meshgen.tet_mesh((3, 3, 2), p, alpha=0.1, seed=80 + p)


def _bsr_to_csr(row_ptr, cols, vals, n_nodes, nc):
    import scipy.sparse as sp
    rp, cl, v = row_ptr.cpu().numpy(), cols.cpu().numpy(), vals.cpu().numpy().astype(np.float64)
    return sp.bsr_matrix((v, cl, rp), shape=(n_nodes * nc, n_nodes * nc)).tocsr()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form,kind", [("laplace", None), ("elasticity", "iso_cell")])
@pytest.mark.parametrize("cell,p", [("hex", 1), ("hex", 2), ("tet", 1), ("tet", 2)])
def test_assemble_matrix(orc, cell, p, form, kind, prec):
    import torch
    import paper_2107_04121_amd as fe
    mesh = _mesh(cell, p)
    nc = orc.n_comp(form)
    lm = meshgen.lame_cell(mesh.n_cells, seed=81) if kind else None
    X, C = _t(mesh.coords), _t(mesh.conn)
    plan = fe.Plan(cell, p, form, "matrix", prec, material=kind)
    Ke = plan(X, C, material=None if lm is None else _t(lm).to(plan.dtype))
    plan.check()
    pat = fe.Pattern(C, mesh.n_nodes)
    inc = fe.Incidence(C, mesh.n_nodes)
    vals = fe.assemble_matrix(pat, inc, C, Ke)
    print(f"[asm] {cell}{p} {form} {prec} nnz={pat.nnz}", flush=True)
    # pattern = node graph of the oracle's scalar assembly
    S = orc.assemble_matrix(mesh, orc.matrix(mesh, "mass"), 1)
    S.sort_indices()
    assert np.array_equal(pat.row_ptr.cpu().numpy(), S.indptr)
    assert np.array_equal(pat.cols.cpu().numpy(), S.indices)
    ref = orc.assemble_matrix(mesh, orc.matrix(mesh, form, lm, kind), nc)
    got = _bsr_to_csr(pat.row_ptr, pat.cols, vals, mesh.n_nodes, nc)
    err = abs(got - ref).max() / abs(ref).max()
    assert err < TOL[prec], err
    again = fe.assemble_matrix(pat, inc, C, Ke)
    torch.cuda.synchronize()
    assert torch.equal(vals, again)


def test_pattern_rejects_bad_connectivity():
    import paper_2107_04121_amd as fe
    mesh = _mesh("hex", 1)
    conn = mesh.conn.copy()
    conn[3, 2] = mesh.n_nodes + 7
    with pytest.raises(fe.FeError) as ei:
        fe.Pattern(_t(conn), mesh.n_nodes)
    assert ei.value.status == 4
