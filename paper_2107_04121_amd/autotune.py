"""Autotuner: picks, per problem, the kernel variant, output layout and
XCD mapping of a plan, seeded by the contraction-path flop model and decided
by timing the candidates on the caller's data; the choices persist in a JSON
cache keyed by GPU architecture, ROCm version, library version and problem.

The paper chooses contraction paths with the optimizers of its einsum
backends (section "Tensor Contraction Path Optimization") and studies
operand layouts (the layout table and its layout experiments); here each
candidate kernel implements one contraction order (gradient-first sum
factorization, gradient-first on reference tables, matrix first, a
per-element product on the matrix cores or one cell per lane), so the
model prices the candidate's expressions with `contraction.optimal_path`,
adds the bytes it must move, and the measured time decides.

Environment:
  FE_AUTOTUNE  0/off: no timing, the model's cheapest feasible candidate;
               1/on (default): time on a cache miss; force: always time.
  FE_CACHE     path of the JSON cache (default
               ~/.cache/paper_2107_04121_amd/autotune.json).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

from .contraction import optimal_path
from .transpile import transpile

__all__ = ["Candidate", "model_cost", "candidates", "tune", "cache_path", "problem_key", "HBM_BPS"]

HBM_BPS = 8.0e12
# rates the model prices flops at: the matrix cores per precision, and the
# vector ALUs (FP32 runs unpacked, at the FP64 rate)
MFMA_FLOPS = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2500e12 / 3}
VALU_FLOPS = 78.6e12

_EXPR = {"mass": ("0,0", "v", "u"), "vmass": ("i,i", "v", "u"), "laplace": ("0.i,0.i", "v", "u"),
         "elasticity": ("IK,s(i:j)->I,s(k:l)->K", "D", "v", "u"), "wdot": ("ij,i,j", "M", "v", "u"),
         "convect": ("i,i.j,j", "v", "u", "u")}


@dataclass
class Candidate:
    variant: str
    layout: str = "cell_major"
    xcd_remap: bool = True
    model_s: float = 0.0
    model_flops: float = 0.0
    measured_ms: float | None = None
    notes: dict = field(default_factory=dict)

    def label(self):
        return f"{self.variant}/{self.layout}/xcd{int(self.xcd_remap)}"


def _sizes(cell, order, nc=3):
    nb = (order + 1) ** 3 if cell == "hex" else (4 if order == 1 else 10)
    nq = (order + 1) ** 3
    s = dict(c=1, q=nq, d=nb, e=nb, f=nb, g=nb, i=3, j=3, k=3, l=3, m=3, r=3, s=3, I=6, K=6)
    return s, nb, nq


def _geometry_flops(cell, order, sumfact):
    """FP64 geometry per cell: the Jacobian by the einsum of the node
    coordinates with the reference gradients (or, sum-factorized, three
    one-dimensional passes per coordinate and direction), plus the inverse
    and determinant (45 flops per point)."""
    s, nb, nq = _sizes(cell, order)
    if sumfact and cell == "hex":
        n = order + 1
        one = optimal_path("cxyz,qx,ry,sz->cqrs", dict(c=1, x=n, y=n, z=n, q=n, r=n, s=n)).flops
        jac = 9 * one
    else:
        jac = optimal_path("cdi,qjd->cqij", dict(c=1, d=nb, i=3, q=nq, j=3)).flops
    return jac + 45 * nq


def model_cost(cell, order, form, mode, precision, cand: Candidate, n_cells=1):
    """(seconds, flops) the model predicts for n_cells cells: the cheapest
    path of the candidate's expressions plus the geometry, priced at the
    candidate's arithmetic unit, against the bytes at 8 TB/s; the larger
    bound wins."""
    t = transpile(*_EXPR[form])
    s, nb, nq = _sizes(cell, order)
    nc = t.n_comp
    esz = 8 if precision == "fp64" else 4
    v = cand.variant
    flops = _geometry_flops(cell, order, v == "sumfact")
    if mode == "matrix" or v == "matrix_first":
        flops += sum(p.flops for p in t.paths_for("matrix", s))
        if v == "matrix_first":
            nd = nc * nb
            flops += optimal_path("cde,ce->cd", dict(c=1, d=nd, e=nd)).flops
    elif v == "sumfact" and cell == "hex":
        n = order + 1
        one = optimal_path("cxyz,qx,ry,sz->cqrs", dict(c=1, x=n, y=n, z=n, q=n, r=n, s=n)).flops
        flops += 2 * 3 * nc * one + 60 * nq  # gradients of u, test contraction, point-wise flux
    else:
        flops += sum(p.flops for p in t.paths_for("residual" if mode == "residual" else "eval", s))
    out_b = {"matrix": (nc * nb) ** 2, "residual": nc * nb, "eval": 1}[mode] * esz
    in_b = nb * 4 + 24 * 1.0 + (nc * esz if mode != "matrix" else 0)
    moved = (out_b + in_b) * n_cells
    if v == "matrix_first":
        moved += 2 * (nc * nb) ** 2 * esz * n_cells  # the chunk is written and read back
    rate = MFMA_FLOPS.get(precision, VALU_FLOPS) if v.startswith("mfma") else VALU_FLOPS
    return max(flops * n_cells / rate, moved / HBM_BPS), flops


def candidates(cell, order, form, mode, precision, material=None, layouts=("cell_major",)):
    """Every variant / layout / XCD mapping the library accepts for the
    problem (plans that fail to create are left out)."""
    from . import FeError, Plan
    out = []
    variants = ["auto", "mfma", "mfma_jobs", "cellwise", "sumfact", "generic", "matrix_first"]
    seen = set()
    for v in variants:
        for layout in (layouts if mode == "residual" else ("cell_major",)):
            try:
                p = Plan(cell, order, form, mode, precision, material=material, variant=v, layout=layout)
            except FeError:
                continue
            key = (p.variant, layout)
            if key in seen:
                continue
            seen.add(key)
            for xcd in (True, False):
                out.append(Candidate(variant=p.variant, layout=layout, xcd_remap=xcd))
    return out


def cache_path() -> str:
    return os.environ.get("FE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                      "paper_2107_04121_amd", "autotune.json")


def _mode_env() -> str:
    v = os.environ.get("FE_AUTOTUNE", "1").strip().lower()
    return {"0": "off", "off": "off", "false": "off", "force": "force"}.get(v, "on")


def problem_key(cell, order, form, mode, precision, material, n_cells, layouts):
    import torch
    from . import _lib
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name)
    rocm = getattr(torch.version, "hip", None) or "none"
    lib = _lib.lib().fe_version().decode()
    bucket = 2 ** max(0, int(round(math.log2(max(1, n_cells)))))
    return (f"{arch}|rocm {rocm}|{lib}|{cell}{order}|{form}|{mode}|{precision}|{material or 'none'}|"
            f"cells~{bucket}|layouts={','.join(layouts)}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(cell, order, form, mode, precision, coords, conn, material=None, material_kind=None, dofs=None,
         layouts=("cell_major",), reps=3, top=None):
    """The fastest plan for the problem on these inputs.  Returns (Plan,
    record) where record holds the key, the chosen candidate, the model's
    and the measured times of every candidate timed and whether the cache
    answered."""
    import torch
    from . import Plan
    n_cells = conn.shape[0]
    key = problem_key(cell, order, form, mode, precision, material_kind, n_cells, layouts)
    path = cache_path()
    env = _mode_env()
    cache = _load(path)
    cands = candidates(cell, order, form, mode, precision, material_kind, layouts)
    if not cands:
        raise ValueError("no kernel accepts this problem")
    for c in cands:
        c.model_s, c.model_flops = model_cost(cell, order, form, mode, precision, c, n_cells)
    cands.sort(key=lambda c: c.model_s)
    hit = cache.get(key)
    if hit and env != "force":
        ch = hit["choice"]
        plan = Plan(cell, order, form, mode, precision, material=material_kind, variant=ch["variant"],
                    layout=ch["layout"], xcd_remap=ch["xcd_remap"])
        return plan, dict(hit, cached=True)
    if env == "off":
        c = cands[0]
        plan = Plan(cell, order, form, mode, precision, material=material_kind, variant=c.variant,
                    layout=c.layout, xcd_remap=c.xcd_remap)
        return plan, dict(key=key, cached=False, timed=False, choice=dict(variant=c.variant, layout=c.layout,
                                                                          xcd_remap=c.xcd_remap))
    timed = cands if top is None else cands[:top]
    best = None
    for c in timed:
        plan = Plan(cell, order, form, mode, precision, material=material_kind, variant=c.variant,
                    layout=c.layout, xcd_remap=c.xcd_remap)
        out = torch.empty(plan.out_shape(n_cells), dtype=plan.dtype, device=coords.device)
        ws = plan.workspace(n_cells, coords.device)
        d = dofs if (mode != "matrix" or form == "convect") else None
        plan(coords, conn, material=material, dofs=d, out=out, workspace=ws)  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            plan(coords, conn, material=material, dofs=d, out=out, workspace=ws)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        plan.check(ws)
        c.measured_ms = min(ts)
        if best is None or c.measured_ms < best[0].measured_ms:
            best = (c, plan)
        del out
    c, plan = best
    record = dict(key=key, cached=False, timed=True, when=time.strftime("%Y-%m-%dT%H:%M:%S"),
                  choice=dict(variant=c.variant, layout=c.layout, xcd_remap=c.xcd_remap),
                  candidates={x.label(): dict(model_ms=x.model_s * 1e3, model_flops_per_cell=x.model_flops,
                                              measured_ms=x.measured_ms) for x in cands})
    cache[key] = {k: v for k, v in record.items() if k != "cached"}
    _store(path, cache)
    if c.layout != "cell_major" and len(layouts) == 1:
        raise AssertionError("layout outside the allowed set")
    return plan, record


def batch_key(groups, precision):
    """Cache key of a batch: architecture, ROCm and library version, and
    each group's cell kind, order, forms and cell count."""
    import torch
    from . import _lib
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name)
    parts = [f"{g['cell']}{int(g['order'])}:{'+'.join(sorted(g['forms']))}:{int(g['conn'].shape[0])}"
             for g in groups]
    return (f"{arch}|rocm {getattr(torch.version, 'hip', None)}|{_lib.lib().fe_version().decode()}|batch|"
            f"{precision}|" + ";".join(parts))


def cached_batch_tiles(groups, precision):
    if _mode_env() == "force":
        return None
    hit = _load(cache_path()).get(batch_key(groups, precision))
    return None if hit is None else hit["tiles"]


def store_batch_tiles(groups, precision, tiles, tuned_ms):
    path = cache_path()
    cache = _load(path)
    cache[batch_key(groups, precision)] = dict(tiles=list(tiles), tuned_ms=tuned_ms,
                                               when=time.strftime("%Y-%m-%dT%H:%M:%S"))
    _store(path, cache)
