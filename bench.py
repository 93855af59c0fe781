"""Throughput benchmark: linear-elasticity element matrices, Q2 hexahedra
(27 nodes, 81 DOFs), 3x3x3 Gauss, 48^3 = 110,592 cells on the unit cube with
vertices perturbed by +-0.15h (seed 0), per-cell Lame lambda, mu ~
lognormal(0, 0.5).  Output 110592 x 81 x 81.

One step = one full evaluation of the hot path on the whole mesh (connectivity
gather, FP64 geometry, contraction, element-matrix store), inputs resident in
HBM.  Prints one JSON line.  The primary value is FP64; FP32 and BF16X3 (FP64
geometry, mixed contraction) are timed the same way and reported with their
measured error against the FP64 oracle on sampled cells.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(workload="linear elasticity element matrices, Q2 hex, "
                "48^3 cells, 3x3x3 Gauss", cells=110592, order=2,
                n_basis=27, n_qp=27, alpha=0.15, seed=0,
                material="per-cell lambda,mu lognormal(0,0.5)")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=48, help="cells per axis")
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other precisions")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="GiB copied by one torch copy before the run (a "
                    "plain copy kernel of known size, used to scale HBM "
                    "byte counters)")
    return ap.parse_args()


def alg_bytes_per_cell(mesh, out_itemsize, mat_itemsize):
    """Algorithmic HBM bytes per cell: output written once, connectivity and
    material read once, each unique node's coordinates read once."""
    nd = 3 * mesh.n_basis
    return (nd * nd * out_itemsize + mesh.n_basis * 4 + 2 * mat_itemsize
            + mesh.n_nodes * 24.0 / mesh.n_cells)


def time_plan(plan, X, C, M, out, steps, warmup):
    import torch
    for _ in range(warmup):
        plan(X, C, material=M, out=out)
    plan.check()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        plan(X, C, material=M, out=out)
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.check()
    per = [a.elapsed_time(b) for a, b in evs]  # ms, each bracketing 1 launch
    return wall, per


def sampled_error(orc, mesh, lm, out, n=48, seed=0):
    import numpy as np
    import meshgen
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(mesh.n_cells, size=min(n, mesh.n_cells),
                             replace=False))
    idx = np.concatenate([idx, [0, mesh.n_cells - 1]])
    sub = meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[idx], cell="hex",
                       order=mesh.order, h=mesh.h)
    ref = orc.matrix(sub, "elasticity", lm[idx], "iso_cell")
    import torch
    got = out[torch.as_tensor(idx, device=out.device)].double().cpu().numpy()
    scale = np.abs(ref).reshape(len(idx), -1).max(1)
    err = np.abs(got - ref).reshape(len(idx), -1).max(1) / scale
    return float(err.max())


def cpu_baseline(orc, mesh, lm, budget_s):
    """The oracle (as it stands) on a bounded sample of the same workload."""
    import numpy as np
    import meshgen

    def run(k):
        sub = meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[:k],
                           cell="hex", order=mesh.order, h=mesh.h)
        t = time.perf_counter()
        orc.matrix(sub, "elasticity", lm[:k], "iso_cell")
        return time.perf_counter() - t

    k = 256
    t = run(k)
    while t < 1.0 and k < mesh.n_cells:
        k = min(mesh.n_cells, k * 4)
        t = run(k)
    # sample: the first k2 cells (at most the whole mesh), repeated until the
    # budget is spent; the output of one pass is 52 KB per cell
    k2 = int(min(mesh.n_cells, max(k, k * budget_s / max(t, 1e-3))))
    reps, total_t = 0, 0.0
    while total_t < budget_s and reps < 50:
        total_t += run(k2)
        reps += 1
    return dict(value=k2 * reps / total_t / 1e9, unit="GElem/s",
                cores=orc.num_threads(), kind="oracle",
                sample=f"first {k2} cells of the 48^3 Q2 mesh x {reps} "
                       f"passes, FP64 element matrices, {total_t:.1f} s",
                seconds=total_t, cells=k2 * reps)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "--gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import meshgen
    import paper_2107_04121_amd as fe

    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * 2**30)
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    mesh = meshgen.hex_mesh(n, 2, alpha=0.15, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)

    import oracle  # test infrastructure: error vs FP64 oracle, CPU baseline
    oracle.build()

    results = {}
    precs = [args.precision] + ([] if args.no_extra else
                                [p for p in ("fp64", "fp32", "bf16x3")
                                 if p != args.precision])
    for prec in precs:
        try:
            plan = fe.Plan("hex", 2, "elasticity", "matrix", prec,
                           material="iso_cell", variant=args.variant)
        except fe.FeError as e:
            results[prec] = {"error": str(e)}
            continue
        dt = plan.dtype
        M = torch.from_numpy(lm).to(dev).to(dt)
        out = torch.empty(plan.out_shape(mesh.n_cells), dtype=dt, device=dev)
        wall, per = time_plan(plan, X, C, M, out, args.steps, args.warmup)
        ms = wall * 1e3 / args.steps
        kern_ms = float(np.mean(per))
        bpc = alg_bytes_per_cell(mesh, out.element_size(), M.element_size())
        gbs = bpc * mesh.n_cells / (kern_ms * 1e-3) / 1e9
        err = sampled_error(oracle, mesh, lm, out)
        results[prec] = dict(ms_per_step=ms, kernel_ms=kern_ms,
                             kernel_ms_min=float(np.min(per)),
                             gelem_s=mesh.n_cells / (ms * 1e-3) / 1e9,
                             alg_bytes_per_cell=bpc, hbm_gbs=gbs,
                             variant=plan.variant, max_rel_err=err)
        del out
        torch.cuda.empty_cache()
    prim = results[args.precision]
    if "error" in prim:
        print(json.dumps({"error": prim["error"]}))
        sys.exit(1)
    line = {
        "metric": "element matrices/s (GElem/s) + HBM GB/s; FP64 vs mixed "
                  "precision at stated error",
        "value": prim["gelem_s"],
        "unit": "GElem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[
            args.precision],
        "data": "synthetic",
        "config": dict(WORKLOAD, cells=mesh.n_cells, parallelism="none"),
        "hbm_gbs": prim["hbm_gbs"],
        "max_rel_err_vs_fp64_oracle": prim["max_rel_err"],
        "roofline": {
            "bound": "hbm",
            "achieved": prim["hbm_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": prim["hbm_gbs"] / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "element-matrix kernel (" + prim["variant"] + ")",
            "kernel_ms": prim["kernel_ms"],
        },
        "precisions": results,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(oracle, mesh, lm,
                                            args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
