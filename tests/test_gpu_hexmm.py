"""GPU parity of the matrix-core kernel for Q2/Q3 hexahedra (mass, vector
mass, Laplace, elasticity with per-cell Lame coefficients) in FP64, FP32 and
BF16X3, through the C ABI.

Meshes have more cells than the persistent grid has workgroups, so every
workgroup walks several cells and the XCD ranges end unevenly.  Sampled cells
(first, last, range boundaries, random) are compared with the FP64 oracle
element by element; every cell of the output is checked for symmetry and
for the property its form fixes (Laplace rows sum to zero, elasticity
annihilates rigid translations, the scalar mass matrix sums to the cell
volume, the vector mass matrix is I_3 (x) M).

Gates as in the other parity tests: FP64 1e-12, FP32 1e-5, BF16X3 1e-4 of
each cell's max-norm.
"""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}
# 1100 Q2 / 1056 Q3 cells: more than the 256-512 resident workgroups
DIMS = {2: (11, 10, 10), 3: (12, 11, 8)}


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


def _sample(n, k=24, seed=5):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    for x in range(9):
        c = min(n - 1, x * ((n + 7) // 8))
        idx.update({c, max(0, c - 1)})
    return np.array(sorted(idx))


def _sub(mesh, idx):
    return meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[idx], cell=mesh.cell, order=mesh.order, h=mesh.h)


def _err(got, ref):
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.abs(r).max(1)).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("form", ["mass", "vmass", "laplace", "elasticity"])
@pytest.mark.parametrize("p", [2, 3])
def test_hexmm_matrix(orc, p, form, prec):
    import torch
    import paper_2107_04121_amd as fe
    if p == 2 and form == "elasticity":
        pytest.skip("Q2 elasticity has its own matrix-core kernel (test_gpu_parity)")
    mesh = meshgen.hex_mesh(DIMS[p], p, alpha=0.15, seed=20 + p, curved=0.04)
    kind = "iso_cell" if form == "elasticity" else None
    lm = meshgen.lame_cell(mesh.n_cells, seed=21) if kind else None
    plan = fe.Plan("hex", p, form, "matrix", prec, material=kind)
    print(f"[hexmm] q{p} {form} {prec} variant={plan.variant} cells={mesh.n_cells}", flush=True)
    assert plan.variant == "mfma"
    K = plan(_t(mesh.coords), _t(mesh.conn), material=None if lm is None else _t(lm, plan.dtype))
    plan.check()
    idx = _sample(mesh.n_cells)
    ref = orc.matrix(_sub(mesh, idx), form, None if lm is None else lm[idx], kind)
    err = _err(K[_t(idx)].cpu().numpy(), ref)
    print(f"[hexmm] sampled err {err:.2e}", flush=True)
    assert err < TOL[prec], err

    tol = TOL[prec]
    Kd = K.double()
    scale = Kd.abs().amax(dim=(1, 2))
    asym = ((Kd - Kd.transpose(1, 2)).abs().amax(dim=(1, 2)) / scale).max().item()
    assert asym < 4 * tol, asym
    nb = (p + 1) ** 3
    if form == "laplace":
        rows = (Kd.sum(dim=2).abs().amax(dim=1) / scale).max().item()
        assert rows < 50 * tol, rows
    elif form == "elasticity":
        for c in range(3):
            t = torch.zeros(3 * nb, dtype=torch.float64, device=K.device)
            t[c * nb:(c + 1) * nb] = 1
            row = ((Kd @ t).abs().amax(dim=1) / scale).max().item()
            assert row < 50 * tol, (c, row)
    elif form == "mass":
        # u = 1 gives the cell volume as u^T M u (oracle, every cell)
        vol = torch.from_numpy(orc.energy(mesh, "mass", np.ones(mesh.n_nodes))).to(K.device)
        assert ((Kd.sum(dim=(1, 2)) - vol).abs() / vol).max().item() < 10 * tol
    else:  # vector mass = I_3 (x) M: diagonal blocks equal, the others zero
        B = Kd.reshape(-1, 3, nb, 3, nb)
        for r in range(3):
            for s in range(3):
                if r == s:
                    assert torch.equal(B[:, r, :, r, :], B[:, 0, :, 0, :])
                else:
                    assert float(B[:, r, :, s, :].abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [2, 3])
def test_hexmm_matches_generic(p, prec):
    """Matrix-core and generic kernels agree on Q2/Q3 Laplace matrices of a
    curved mesh, cell by cell (both against each other, no oracle)."""
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh((5, 4, 3), p, alpha=0.15, seed=30 + p, curved=0.04)
    X, C = _t(mesh.coords), _t(mesh.conn)
    a = fe.Plan("hex", p, "laplace", "matrix", prec)(X, C)
    b = fe.Plan("hex", p, "laplace", "matrix", prec, variant="generic")(X, C)
    assert _err(a.cpu().numpy(), b.cpu().numpy().astype(np.float64)) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["mfma_jobs", "mfma_ws"])
def test_q2_elasticity_variants(orc, variant, prec):
    """The other two matrix-core kernels of Q2 elasticity (per-cell Lame
    coefficients): tile jobs stored straight from the accumulators, and the
    same jobs on consumer waves while producer waves build the next cell's
    operand.  1100 cells (several per workgroup, uneven XCD ranges): sampled
    cells against the FP64 oracle, every cell for symmetry and rigid
    translations, and the staged kernel's output to the same gate."""
    import torch
    import paper_2107_04121_amd as fe
    mesh = meshgen.hex_mesh(DIMS[2], 2, alpha=0.15, seed=22, curved=0.04)
    lm = meshgen.lame_cell(mesh.n_cells, seed=23)
    plan = fe.Plan("hex", 2, "elasticity", "matrix", prec, material="iso_cell", variant=variant)
    print(f"[q2-elast] {variant} {prec} variant={plan.variant} cells={mesh.n_cells}", flush=True)
    assert plan.variant == variant
    X, C, M = _t(mesh.coords), _t(mesh.conn), _t(lm, plan.dtype)
    K = plan(X, C, material=M)
    plan.check()
    idx = _sample(mesh.n_cells)
    ref = orc.matrix(_sub(mesh, idx), "elasticity", lm[idx], "iso_cell")
    err = _err(K[_t(idx)].cpu().numpy(), ref)
    print(f"[q2-elast] sampled err {err:.2e}", flush=True)
    assert err < TOL[prec], err
    tol = TOL[prec]
    Kd = K.double()
    scale = Kd.abs().amax(dim=(1, 2))
    assert ((Kd - Kd.transpose(1, 2)).abs().amax(dim=(1, 2)) / scale).max().item() < 4 * tol
    for c in range(3):
        t = torch.zeros(81, dtype=torch.float64, device=K.device)
        t[c * 27:(c + 1) * 27] = 1
        assert ((Kd @ t).abs().amax(dim=1) / scale).max().item() < 50 * tol
    staged = fe.Plan("hex", 2, "elasticity", "matrix", prec, material="iso_cell")(X, C, material=M)
    assert _err(K.cpu().numpy(), staged.double().cpu().numpy()) < tol
