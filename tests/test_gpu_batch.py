"""GPU parity of the batched, graph-captured evaluation of uneven groups
(P1/P2 tetrahedra, Q1/Q2 hexahedra; mass, Laplace and elasticity matrices in
one persistent launch) against the FP64 oracle, with graph replays checked
against each other and against the single-form plans."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _err(got, ref):
    n = ref.shape[0]
    g = got.reshape(n, -1).astype(np.float64)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.abs(r).max(1)).max())


def _groups(dt):
    meshes = [("tet", 1, meshgen.tet_mesh((5, 4, 3), 1, alpha=0.15, seed=1)),
              ("tet", 2, meshgen.tet_mesh((4, 3, 3), 2, alpha=0.15, seed=2)),
              ("hex", 1, meshgen.hex_mesh((7, 5, 4), 1, alpha=0.15, seed=3)),
              ("hex", 2, meshgen.hex_mesh((4, 3, 3), 2, alpha=0.15, seed=4,
                                          curved=0.03))]
    groups, refs = [], []
    for k, (cell, p, m) in enumerate(meshes):
        lm = meshgen.lame_cell(m.n_cells, seed=10 + k)
        groups.append(dict(cell=cell, order=p, coords=_t(m.coords),
                           conn=_t(m.conn), material=_t(lm, dt),
                           forms=("mass", "laplace", "elasticity")))
        refs.append((m, lm))
    return groups, refs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("autotune", [False, True])
def test_batch_matches_oracle(orc, prec, autotune):
    import torch
    import paper_2107_04121_amd as fe
    dt = {"fp64": torch.float64, "fp32": torch.float32}[prec]
    groups, refs = _groups(dt)
    b = fe.Batch(groups, precision=prec, autotune=autotune)
    print(f"[batch] {prec} autotune={autotune} tiles={b.tiles} "
          f"grid={b.grid}", flush=True)
    outs = b.run()
    b.check()
    first = [{k: v.clone() for k, v in o.items()} for o in outs]
    for (m, lm), o in zip(refs, outs):
        for form in ("mass", "laplace", "elasticity"):
            mat, kind = (lm, "iso_cell") if form == "elasticity" else (None,
                                                                       None)
            ref = orc.matrix(m, form, mat, kind)
            err = _err(o[form].cpu().numpy(), ref)
            print(f"[batch] {m.cell}{m.order} {form} {err:.2e}", flush=True)
            assert err < TOL[prec], (m.cell, m.order, form, err)
    # graph replays with eager work in between give identical results
    for _ in range(3):
        for o in outs:
            for v in o.values():
                v.fill_(-1.0)
        torch.cuda.synchronize()
        b.run()
        b.check()
        for o, f in zip(outs, first):
            for k in o:
                assert torch.equal(o[k], f[k])


def test_batch_form_subset_and_faults(orc):
    import paper_2107_04121_amd as fe
    m = meshgen.tet_mesh((3, 2, 2), 2, alpha=0.15, seed=7)
    conn = m.conn.copy()
    b = fe.Batch([dict(cell="tet", order=2, coords=_t(m.coords),
                       conn=_t(conn), forms=("laplace",))],
                 precision="fp64", autotune=False)
    o = b.run()
    b.check()
    assert set(o[0]) == {"laplace"}
    assert _err(o[0]["laplace"].cpu().numpy(),
                orc.matrix(m, "laplace")) < 1e-12
    conn[4, [0, 1]] = conn[4, [1, 0]]      # inverted tetrahedron
    b2 = fe.Batch([dict(cell="tet", order=2, coords=_t(m.coords),
                        conn=_t(conn), forms=("mass",))],
                  precision="fp64", autotune=False)
    b2.run()
    with pytest.raises(fe.FeError) as ei:
        b2.check()
    assert ei.value.status == 3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_p1_tets_passes_and_subsets(orc, prec):
    """P1 tetrahedra take the affine routine: 256 cells per pass.  3,024
    cells in items of 512 (a ragged last pass and item) and a form subset
    without elasticity, against the oracle."""
    import torch
    import paper_2107_04121_amd as fe
    dt = {"fp64": torch.float64, "fp32": torch.float32}[prec]
    m = meshgen.tet_mesh((9, 8, 7), 1, alpha=0.2, seed=21)
    lm = meshgen.lame_cell(m.n_cells, seed=22)
    b = fe.Batch([dict(cell="tet", order=1, coords=_t(m.coords),
                       conn=_t(m.conn), material=_t(lm, dt),
                       forms=("mass", "laplace", "elasticity"), tile=300),
                  dict(cell="tet", order=1, coords=_t(m.coords),
                       conn=_t(m.conn[:700]), forms=("mass", "laplace"))],
                 precision=prec, autotune=False)
    print(f"[batch-p1] {prec} tiles={b.tiles} cells={m.n_cells}", flush=True)
    assert b.tiles[0] == 512
    o = b.run()
    b.check()
    sub = meshgen.Mesh(coords=m.coords, conn=m.conn[:700], cell="tet",
                       order=1, h=m.h)
    for form in ("mass", "laplace", "elasticity"):
        mat, kind = (lm, "iso_cell") if form == "elasticity" else (None, None)
        ref = orc.matrix(m, form, mat, kind)
        err = _err(o[0][form].cpu().numpy(), ref)
        print(f"[batch-p1] {form} {err:.2e}", flush=True)
        assert err < TOL[prec], (form, err)
        if form != "elasticity":
            assert _err(o[1][form].cpu().numpy(),
                        orc.matrix(sub, form)) < TOL[prec]
    assert set(o[1]) == {"mass", "laplace"}


def test_batch_p1_tet_faults():
    import paper_2107_04121_amd as fe
    m = meshgen.tet_mesh((4, 3, 3), 1, alpha=0.15, seed=23)
    conn = m.conn.copy()
    conn[200, [0, 1]] = conn[200, [1, 0]]     # inverted tetrahedron
    b = fe.Batch([dict(cell="tet", order=1, coords=_t(m.coords),
                        conn=_t(conn), forms=("laplace",))],
                 precision="fp32", autotune=False)
    b.run()
    with pytest.raises(fe.FeError) as ei:
        b.check()
    assert ei.value.status == 3
    conn = m.conn.copy()
    conn[17, 2] = m.n_nodes                   # node number out of range
    b = fe.Batch([dict(cell="tet", order=1, coords=_t(m.coords),
                        conn=_t(conn), forms=("mass",))],
                 precision="fp64", autotune=False)
    b.run()
    with pytest.raises(fe.FeError) as ei:
        b.check()
    assert ei.value.status == 4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_empty_and_single_cell_groups(orc, prec):
    """An empty group next to single-cell groups of every routine: the empty
    group takes no work item, the others match the oracle."""
    import torch
    import paper_2107_04121_amd as fe
    dt = {"fp64": torch.float64, "fp32": torch.float32}[prec]
    specs = [("tet", 1, meshgen.tet_mesh((2, 2, 1), 1, alpha=0.1, seed=31), 0),
             ("hex", 2, meshgen.hex_mesh((2, 1, 1), 2, alpha=0.1, seed=32), 1),
             ("tet", 2, meshgen.tet_mesh((1, 1, 1), 2, alpha=0.1, seed=33), 1),
             ("hex", 1, meshgen.hex_mesh((2, 2, 1), 1, alpha=0.1, seed=34), 3),
             ("tet", 1, meshgen.tet_mesh((1, 1, 1), 1, alpha=0.1, seed=35), 1)]
    groups, refs = [], []
    for k, (cell, p, m, n) in enumerate(specs):
        lm = meshgen.lame_cell(max(n, 1), seed=40 + k)[:n]
        groups.append(dict(cell=cell, order=p, coords=_t(m.coords),
                           conn=_t(m.conn[:n]), material=_t(lm, dt),
                           forms=("mass", "laplace", "elasticity")))
        refs.append((meshgen.Mesh(coords=m.coords, conn=m.conn[:n], cell=cell,
                                  order=p, h=m.h), lm))
    b = fe.Batch(groups, precision=prec, autotune=True)
    print(f"[batch-edge] {prec} tiles={b.tiles}", flush=True)
    o = b.run()
    b.check()
    for (m, lm), out in zip(refs, o):
        for form in ("mass", "laplace", "elasticity"):
            assert out[form].shape[0] == m.conn.shape[0]
            if m.conn.shape[0] == 0:
                continue
            mat, kind = (lm, "iso_cell") if form == "elasticity" else (None, None)
            err = _err(out[form].cpu().numpy(), orc.matrix(m, form, mat, kind))
            assert err < TOL[prec], (m.cell, m.order, form, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", [None, 24])
def test_batch_partial_passes(orc, prec, tile):
    """The low-order passes take 8 P2 tetrahedra or 8/16 Q1 hexahedra at a
    time, and their output loops write groups of adjacent columns while
    stepping rows and cells by constant strides.  Cell counts that leave a
    partial last pass (108 P2 tets, 45 Q1 hexahedra; with tile 24 also a
    partial pass in every item) and every form, against the oracle."""
    import torch
    import paper_2107_04121_amd as fe
    dt = {"fp64": torch.float64, "fp32": torch.float32}[prec]
    meshes = [("tet", 2, meshgen.tet_mesh((3, 3, 2), 2, alpha=0.15, seed=31)),
              ("hex", 1, meshgen.hex_mesh((5, 3, 3), 1, alpha=0.15, seed=32))]
    groups, refs = [], []
    for k, (cell, p, m) in enumerate(meshes):
        lm = meshgen.lame_cell(m.n_cells, seed=40 + k)
        g = dict(cell=cell, order=p, coords=_t(m.coords), conn=_t(m.conn), material=_t(lm, dt),
                 forms=("mass", "laplace", "elasticity"))
        if tile:
            g["tile"] = tile
        groups.append(g)
        refs.append((m, lm))
    assert [m.n_cells for _, _, m in meshes] == [108, 45]
    b = fe.Batch(groups, precision=prec, autotune=False)
    print(f"[batch-partial] {prec} tiles={b.tiles}", flush=True)
    outs = b.run()
    b.check()
    for (m, lm), o in zip(refs, outs):
        for form in ("mass", "laplace", "elasticity"):
            mat, kind = (lm, "iso_cell") if form == "elasticity" else (None, None)
            err = _err(o[form].cpu().numpy(), orc.matrix(m, form, mat, kind))
            print(f"[batch-partial] {m.cell}{m.order} {form} {err:.2e}", flush=True)
            assert err < TOL[prec], (m.cell, m.order, form, err)
