"""Throughput benchmark of the per-element weak-form evaluation on one GPU.

Headline workload (c2): linear-elasticity element matrices, Q2
hexahedra (27 nodes, 81 DOFs), 3x3x3 Gauss, 48^3 = 110,592 cells on the unit
cube with vertices perturbed by +-0.15h (seed 0), per-cell Lame lambda, mu ~
lognormal(0, 0.5).  Output 110592 x 81 x 81.  One step = one full
evaluation of the hot path on the whole mesh (connectivity gather, FP64
geometry, contraction, element-matrix store), inputs resident in HBM.  The
primary value is FP64; FP32 and BF16X3 are timed the same way and reported
with their measured error against the FP64 oracle on sampled cells.

Other configurations of the same hot path (--config):
  c1  Q1 Laplace, 16^3 cells (+-0.2h): element matrices and residual, FP64,
      plus a size sweep up to 128^3 for the HBM roof;
  c3  Q3 residuals (Laplace, elasticity), 96^3 cells, FP32 with FP64
      geometry: sum-factorized gradient-first (cell-major and cell-minor
      output), generic gradient-first, matrix-first;
  c4  one batched graph launch: 300k P1 tets, 120k P2 tets, 200k Q1 hex,
      40k Q2 hex, mass + Laplace + elasticity each, FP32; vs separate
      launches and vs untuned tiles;
  c5  energy J = sum u_e^T K_e u_e of Q2 elasticity on 32^3 cells with
      per-point coefficients: forward + adjoint (dJ/dc, dJ/dx, dJ/du);
  c6  Q3 linear-elasticity element matrices (64 nodes, 192 DOFs, 4x4x4
      Gauss), 32^3 cells, per-cell Lame coefficients, FP64 / FP32 / BF16X3:
      the matrix-core-bound case, reported against the matrix-core peak;
  c7  the paper's two other benchmark forms on Q2 hexahedra, 32^3 cells,
      FP64 and FP32: weighted vector dot product (per-point 3x3 M) and
      Navier-Stokes convection (matrix = derivative at u ~ N(0,1)), matrix
      (on the matrix cores) and residual modes;
  c8  orders 4 and 5 at the paper's cell count for them, 1,024 cells: the
      paper's five forms (Laplace, vector dot, weighted dot, convection,
      elasticity) as element matrices (on the matrix cores, reported against
      their peak) and sum-factorized residuals; primary Q5 elasticity
      matrices.
With no --config (the default, "all") bench.py prints ONE JSON line: the
c2 headline record, with the complete records of c1, c3, c4 and c5 (value,
roofline, cpu_baseline, errors against the oracle) under its "configs" key.
With --config it prints that configuration's line alone.
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
FP64_PEAK_TFLOPS = 78.6
# dense matrix-core peaks (TFLOP/s); BF16X3 does three bf16 products per
# product of the contraction, so its contraction rate peaks at a third of bf16
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3}
# HBM bytes per launch of a kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for a 1 GiB
# copy (fetch x2.0, write x1.0).  A figure holds only for the sources it was
# measured on: when their hash differs the field is reported as null.
MEASURED_TRAFFIC = {
    "k_elast_q2<0>": dict(bytes=5983546000, sha256="6ef548f20797550a",
                          sources=["k_mfma.hip", "q2_device.h",
                                   "fe_device.h"]),
    "k_elast_q3ws<0>": dict(bytes=9696687281, sha256="e72b02810c95e020",
                            sources=["k_hexmm.hip", "mm_device.h",
                                     "q2_device.h", "fe_device.h"]),
    "k_hexmc<5,3,0>": dict(bytes=3534367966, sha256="e72b02810c95e020",
                           sources=["k_hexmm.hip", "mm_device.h",
                                    "q2_device.h", "fe_device.h"]),
    "k_cw_scalar<hex,1,laplace,double>@128^3": dict(
        bytes=1195579701, sha256="fb152f97c8e4eef5",
        sources=["k_cellwise.hip", "cw_device.h", "fe_device.h"]),
    "k_sf<3,elasticity,float>@96^3": dict(
        bytes=2067873756, sha256="7bfc61c550fd7cfd",
        sources=["k_sumfact.hip", "cw_device.h", "fe_device.h"]),
    "k_batch<float>@c4": dict(
        bytes=2797008333, sha256="da3868d0322718fc",
        sources=["k_batch.hip", "q2_device.h", "fe_device.h"]),
    "k_hexgm<2,convect,fp64>@32^3": dict(
        bytes=1777911343, sha256="6f59da7c0f2b2c14",
        sources=["k_hexgm.hip", "mm_device.h", "q2_device.h",
                 "fe_device.h"]),
}


def source_hash(files):
    """First 16 hex digits of the sha256 of the named csrc files, in order
    (the stamp carried by every measured figure and profile summary)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2107_04121_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(kernel):
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None:
        return None
    return m["bytes"] if source_hash(m["sources"]) == m["sha256"] else None


METRIC = ("element matrices/s (GElem/s) + HBM GB/s; FP64 vs mixed precision "
          "at stated error")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="all",
                    choices=["all", "c1", "c2", "c3", "c4", "c5", "c6", "c7",
                             "c8"],
                    help="all (default): the c2 line, with c1, c3, c4 and c5 "
                    "under its 'configs' key")
    ap.add_argument("--n", type=int, default=0, help="cells per axis")
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other precisions/variants")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=6.0,
                    help="seconds of each oracle timing (all threads, then "
                    "one thread)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="GiB copied by one torch copy before the run (a "
                    "plain copy kernel of known size, used to scale HBM "
                    "byte counters)")
    return ap.parse_args()


# --------------------------------------------------------------- helpers ---

def time_calls(fn, steps, warmup):
    """Wall time of `steps` calls (synchronised on both sides) and the HIP
    event time of each call on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def mean(v):
    return float(sum(v) / len(v))


def tww_mean(v):
    """Mean without the worst repetition (the paper's statistic)."""
    v = sorted(v)
    return mean(v[:-1]) if len(v) > 1 else float(v[0])


def rel_err(got, ref):
    import numpy as np
    n = ref.shape[0]
    g = np.asarray(got, dtype=np.float64).reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.abs(g - r).max(1) / np.abs(r).max(1)).max())


def sample_cells(n_cells, k=48, seed=0):
    import numpy as np
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n_cells, size=min(k, n_cells), replace=False))
    return np.unique(np.concatenate([idx, [0, n_cells - 1]]))


def submesh(mesh, idx):
    import meshgen
    return meshgen.Mesh(coords=mesh.coords, conn=mesh.conn[idx],
                        cell=mesh.cell, order=mesh.order, h=mesh.h)


def oracle_rate(orc_call, n_cells, budget_s):
    """Time the oracle (as it stands) on the first k cells, k grown until the
    run takes about 1 s, then repeated until budget_s; cells/s."""
    k = 64
    t = orc_call(k)
    while t < 1.0 and k < n_cells:
        k = min(n_cells, k * 4)
        t = orc_call(k)
    k2 = int(min(n_cells, max(k, k * budget_s / max(t, 1e-3))))
    reps, total = 0, 0.0
    while total < budget_s and reps < 100000:
        total += orc_call(k2)
        reps += 1
    return k2 * reps / total, k2, reps, total


def host_cpu():
    """Model name and usable cores of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)),
            "cpu_count": os.cpu_count()}


def cpu_baseline(orc, call, n_cells, budget_s, what):
    """The oracle, as it stands, timed on the host: all OpenMP threads (the
    reported value) and one thread (the paper's single-thread mode), each
    for about budget_s on a prefix of the workload; cells/s in GElem/s.
    `what(k, reps, seconds)` describes the sample."""
    threads = orc.num_threads()
    rate, k, reps, tot = oracle_rate(call, n_cells, budget_s)
    orc.set_num_threads(1)
    try:
        rate1, k1, reps1, tot1 = oracle_rate(call, n_cells, budget_s)
    finally:
        orc.set_num_threads(threads)
    return {"value": rate / 1e9, "unit": "GElem/s", "cores": threads,
            "kind": "oracle", "sample": what(k, reps, tot),
            "single_thread": {"value": rate1 / 1e9, "unit": "GElem/s",
                              "cores": 1, "sample": what(k1, reps1, tot1)},
            "host": host_cpu()}


def copy_calibration(gib):
    import torch
    if gib <= 0:
        return
    nbytes = int(gib * 2**30)
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def base_line(args, value, ms, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "GElem/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic",
            "config": dict(config, parallelism="none")}


# ------------------------------------------------------------------- c2 ---

def alg_bytes_per_cell(mesh, nd, out_itemsize, mat_itemsize):
    """Algorithmic HBM bytes per cell: output written once, connectivity and
    material read once, each unique node's coordinates read once."""
    return (nd * nd * out_itemsize + mesh.n_basis * 4 + 2 * mat_itemsize
            + mesh.n_nodes * 24.0 / mesh.n_cells)


def run_c2(args, orc):
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 48
    mesh = meshgen.hex_mesh(n, 2, alpha=0.15, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)
    idx = sample_cells(mesh.n_cells)
    ref = orc.matrix(submesh(mesh, idx), "elasticity", lm[idx], "iso_cell")
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
        M = torch.from_numpy(lm).to(dev).to(plan.dtype)
        out = torch.empty(plan.out_shape(mesh.n_cells), dtype=plan.dtype,
                          device=dev)
        wall, per = time_calls(lambda: plan(X, C, material=M, out=out),
                               args.steps, args.warmup)
        plan.check()
        ms = wall * 1e3 / args.steps
        kern_ms = mean(per)
        bpc = alg_bytes_per_cell(mesh, 81, out.element_size(),
                                 M.element_size())
        err = rel_err(out[torch.as_tensor(idx, device=dev)].cpu().numpy(),
                      ref)
        results[prec] = dict(ms_per_step=ms, kernel_ms=kern_ms,
                             kernel_ms_tww=tww_mean(per),
                             kernel_ms_min=float(min(per)),
                             gelem_s=mesh.n_cells / (ms * 1e-3) / 1e9,
                             alg_bytes_per_cell=bpc,
                             hbm_gbs=bpc * mesh.n_cells / (kern_ms * 1e-3)
                             / 1e9,
                             variant=plan.variant, max_rel_err=err)
        del out
        torch.cuda.empty_cache()
    prim = results[args.precision]
    if "error" in prim:
        return {"error": prim["error"]}
    line = base_line(args, prim["gelem_s"], prim["ms_per_step"],
                     {"fp64": "f64", "fp32": "f32",
                      "bf16x3": "bf16x3"}[args.precision],
                     dict(workload="linear elasticity element matrices, Q2 "
                          "hex, 48^3 cells, 3x3x3 Gauss", cells=mesh.n_cells,
                          order=2, n_basis=27, n_qp=27, alpha=0.15, seed=0,
                          material="per-cell lambda,mu lognormal(0,0.5)"))
    line["hbm_gbs"] = prim["hbm_gbs"]
    line["max_rel_err_vs_fp64_oracle"] = prim["max_rel_err"]
    line["roofline"] = {"bound": "hbm", "achieved": prim["hbm_gbs"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": prim["hbm_gbs"] / HBM_PEAK_GBS,
                        "traffic": (traffic("k_elast_q2<0>")
                                    if args.precision == "fp64"
                                    and prim["variant"] == "mfma" else None),
                        "kernel": "k_elast_q2 (" + prim["variant"] + ")",
                        "kernel_ms": prim["kernel_ms"]}
    line["precisions"] = results
    if not args.no_extra:
        line["assembly"] = c2_assembly(args, mesh, lm, X, C)
    if not args.no_cpu:
        def call(k):
            t = time.perf_counter()
            orc.matrix(submesh(mesh, slice(0, k)), "elasticity", lm[:k],
                       "iso_cell")
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"first {k2} cells of the 48^3 Q2 mesh x "
            f"{reps} passes, FP64 element matrices, {tot:.1f} s")
    return line


def c2_assembly(args, mesh, lm, X, C):
    """Global block-CSR assembly of the FP64 elasticity matrices (the step
    after the element loop): pattern build once, then the assembly kernel
    timed; bytes = element matrices read once + values written once."""
    import torch
    import paper_2107_04121_amd as fe
    plan = fe.Plan("hex", 2, "elasticity", "matrix", "fp64",
                   material="iso_cell")
    K = plan(X, C, material=torch.from_numpy(lm).to(X.device))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pat = fe.Pattern(C, mesh.n_nodes)
    inc = fe.Incidence(C, mesh.n_nodes)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    vals = torch.empty((pat.nnz, 3, 3), dtype=torch.float64, device=X.device)
    _, per = time_calls(lambda: fe.assemble_matrix(pat, inc, C, K, out=vals),
                        args.steps, args.warmup)
    kms = mean(per)
    nbytes = K.numel() * 8 + vals.numel() * 8
    res = dict(kernel="k_asm_rows<double,3>", kernel_ms=kms,
               pattern_and_incidence_ms=setup_ms, nnz_blocks=pat.nnz,
               bytes=nbytes, hbm_gbs=nbytes / (kms * 1e-3) / 1e9)
    del K, vals, pat, inc
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------- c1 ---

def run_c1(args, orc):
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 16
    mesh = meshgen.hex_mesh(n, 1, alpha=0.2, seed=0)
    U = meshgen.dofs(mesh.n_nodes, 1, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)
    Ut = torch.from_numpy(U).to(dev)
    pm = fe.Plan("hex", 1, "laplace", "matrix", "fp64")
    pr = fe.Plan("hex", 1, "laplace", "residual", "fp64")
    K = torch.empty(pm.out_shape(mesh.n_cells), dtype=torch.float64,
                    device=dev)
    r = torch.empty(pr.out_shape(mesh.n_cells), dtype=torch.float64,
                    device=dev)

    def step():
        pm(X, C, out=K)
        pr(X, C, dofs=Ut, out=r)

    wall, per = time_calls(step, args.steps, args.warmup)
    pm.check()
    pr.check()
    _, per_m = time_calls(lambda: pm(X, C, out=K), args.steps, 1)
    _, per_r = time_calls(lambda: pr(X, C, dofs=Ut, out=r), args.steps, 1)
    # error against the oracle: every cell, or sampled cells on large meshes
    idx = (sample_cells(mesh.n_cells, 256) if mesh.n_cells > 65536
           else slice(None))
    sub = submesh(mesh, idx) if mesh.n_cells > 65536 else mesh
    sel = torch.as_tensor(idx, device=dev) if mesh.n_cells > 65536 else slice(None)
    err_m = rel_err(K[sel].cpu().numpy(), orc.matrix(sub, "laplace"))
    err_r = rel_err(r[sel].cpu().numpy(), orc.residual(sub, "laplace", U))
    ms = wall * 1e3 / args.steps
    # size sweep of the matrix kernel for the HBM roof
    sweep = {}
    for m in ([16, 32, 64, 96, 128] if not args.no_extra else []):
        msh = meshgen.hex_mesh(m, 1, alpha=0.2, seed=0)
        Xs = torch.from_numpy(msh.coords).to(dev)
        Cs = torch.from_numpy(msh.conn).to(dev)
        Ks = torch.empty(pm.out_shape(msh.n_cells), dtype=torch.float64,
                         device=dev)
        _, p2 = time_calls(lambda: pm(Xs, Cs, out=Ks), 10, 2)
        bpc = 512 + 32 + msh.n_nodes * 24.0 / msh.n_cells
        kms = mean(p2)
        sweep[f"{m}^3"] = dict(cells=msh.n_cells, kernel_ms=kms,
                               gelem_s=msh.n_cells / (kms * 1e-3) / 1e9,
                               hbm_gbs=bpc * msh.n_cells / (kms * 1e-3) / 1e9)
        del Ks, Xs, Cs
    torch.cuda.empty_cache()
    bpc = 512 + 32 + mesh.n_nodes * 24.0 / mesh.n_cells
    kms = mean(per_m)
    line = base_line(args, mesh.n_cells / (ms * 1e-3) / 1e9, ms, "f64",
                     dict(workload="Q1 Laplace element matrices + residual, "
                          f"{n}^3 cells, 2x2x2 Gauss", cells=mesh.n_cells,
                          order=1, alpha=0.2, seed=0))
    line["matrix"] = dict(kernel_ms=kms, variant=pm.variant,
                          gelem_s=mesh.n_cells / (kms * 1e-3) / 1e9,
                          hbm_gbs=bpc * mesh.n_cells / (kms * 1e-3) / 1e9,
                          max_rel_err=err_m)
    line["residual"] = dict(kernel_ms=mean(per_r), variant=pr.variant,
                            gelem_s=mesh.n_cells / (mean(per_r) * 1e-3)
                            / 1e9, max_rel_err=err_r)
    kname = ("k_cw_scalar<hex,1,laplace,double>" if pm.variant == "cellwise"
             else "k_matrix<hex,1,laplace>")
    # the roofline of the workload itself: at 16^3 the 2.3 MB of the matrix
    # launch fit in the L2/MALL and the launch is latency-bound
    line["roofline"] = {"bound": "hbm", "achieved": line["matrix"]["hbm_gbs"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": line["matrix"]["hbm_gbs"] / HBM_PEAK_GBS,
                        "traffic": None, "kernel": f"{kname} at {n}^3",
                        "kernel_ms": kms,
                        "note": f"{n}^3 cells move {bpc * mesh.n_cells / 1e6:.1f}"
                        " MB per launch: launch-latency bound, not an HBM "
                        "measurement; see roofline_128cube"}
    big = sweep.get("128^3")
    if big:
        line["roofline_128cube"] = {
            "bound": "hbm", "achieved": big["hbm_gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": big["hbm_gbs"] / HBM_PEAK_GBS,
            "traffic": (traffic("k_cw_scalar<hex,1,laplace,double>@128^3")
                        if pm.variant == "cellwise" else None),
            "kernel": f"{kname} at 128^3 (2,097,152 cells, the same kernel "
                      "and launch configuration as the workload)",
            "kernel_ms": big["kernel_ms"]}
    line["sweep"] = sweep
    if not args.no_cpu:
        def call(k):
            t = time.perf_counter()
            sub = submesh(mesh, slice(0, k))
            orc.matrix(sub, "laplace")
            orc.residual(sub, "laplace", U)
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"{k2} cells x {reps} passes of matrix + "
            f"residual, {tot:.1f} s")
    return line


# ------------------------------------------------------------------- c3 ---

def run_c3(args, orc):
    import numpy as np
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 96
    mesh = meshgen.hex_mesh(n, 3, alpha=0.15, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)
    M = torch.from_numpy(lm).to(dev).float()
    idx = sample_cells(mesh.n_cells, 24)
    sub = submesh(mesh, idx)
    res = {}
    for form, nc in (("laplace", 1), ("elasticity", 3)):
        U = meshgen.dofs(mesh.n_nodes, nc, seed=0)
        Ut = torch.from_numpy(U).to(dev).float()
        mat, kind = (M, "iso_cell") if form == "elasticity" else (None, None)
        ref = orc.residual(sub, form, U, lm[idx] if mat is not None else None,
                           kind)
        variants = [("sumfact", "cell_major"), ("sumfact", "cell_minor")]
        if not args.no_extra:
            variants += [("generic", "cell_major"),
                         ("matrix_first", "cell_major")]
        for variant, layout in variants:
            plan = fe.Plan("hex", 3, form, "residual", "fp32", material=kind,
                           variant=variant, layout=layout)
            out = torch.empty(plan.out_shape(mesh.n_cells),
                              dtype=torch.float32, device=dev)
            ws = plan.workspace(mesh.n_cells, dev)
            steps = args.steps if variant == "sumfact" else 1
            warm = args.warmup if variant == "sumfact" else 0
            wall, per = time_calls(
                lambda: plan(X, C, material=mat, dofs=Ut, out=out,
                             workspace=ws), steps, warm)
            plan.check()
            got = out.cpu().numpy()
            if layout == "cell_minor":
                got = np.moveaxis(got, -1, 0)
            err = rel_err(got[idx], ref)
            bpc = (mesh.n_nodes * (24 + 4 * nc) / mesh.n_cells + 64 * 4
                   + 64 * nc * 4 + (8 if kind else 0))
            kms = mean(per)
            res[f"{form}/{variant}/{layout}"] = dict(
                kernel_ms=kms, gelem_s=mesh.n_cells / (kms * 1e-3) / 1e9,
                hbm_gbs=bpc * mesh.n_cells / (kms * 1e-3) / 1e9,
                max_rel_err=err, steps=steps)
            del out, ws
            plan._ws = None
            torch.cuda.empty_cache()
    prim = res["elasticity/sumfact/cell_major"]
    tot_ms = prim["kernel_ms"] + res["laplace/sumfact/cell_major"][
        "kernel_ms"]
    line = base_line(args, mesh.n_cells / (prim["kernel_ms"] * 1e-3) / 1e9,
                     tot_ms, "f32",
                     dict(workload="Q3 hex residuals (Laplace + elasticity),"
                          f" {n}^3 cells, 4x4x4 Gauss, FP32 with FP64 "
                          "geometry", cells=mesh.n_cells, order=3,
                          alpha=0.15, seed=0))
    # algorithmic flops of the sum-factorized gradient-first residual per cell
    # (N1 = 4 points per axis): three 1-D passes of 8 N1^4 FMA per scalar
    # field for the three coordinate fields (FP64) and the u fields, the
    # same for the transposed test contraction per component, plus the
    # inverse (45 flops) and the flux (129 flops, elasticity) per point.
    # FP32 runs at the FP64 vector rate here (packed FP32 is not used), so
    # both count against 78.6 TFLOP/s.
    n4 = 4 ** 4
    flops = (3 * 16 * n4 + 45 * 64) + (3 * 16 * n4 + 129 * 64 + 3 * 16 * n4)
    achieved = flops * mesh.n_cells / (prim["kernel_ms"] * 1e-3) / 1e12
    line["roofline"] = {"bound": "alu", "achieved": achieved,
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP64_PEAK_TFLOPS,
                        "traffic": (traffic("k_sf<3,elasticity,float>@96^3")
                                    if n == 96 else None),
                        "kernel": "k_sf<3,elasticity,float>",
                        "flops_per_cell": flops,
                        "kernel_ms": prim["kernel_ms"],
                        "hbm_frac": prim["hbm_gbs"] / HBM_PEAK_GBS}
    line["paths"] = res
    if not args.no_cpu:
        U3 = meshgen.dofs(mesh.n_nodes, 3, seed=0)

        def call(k):
            t = time.perf_counter()
            orc.residual(submesh(mesh, slice(0, k)), "elasticity", U3,
                         lm[:k], "iso_cell")
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"{k2} Q3 cells x {reps} passes, "
            f"elasticity residual FP64, {tot:.1f} s")
    return line


# ------------------------------------------------------------------- c4 ---

C4_GROUPS = [("tet", 1, (50, 40, 25)), ("tet", 2, (40, 25, 20)),
             ("hex", 1, (100, 50, 40)), ("hex", 2, (40, 40, 25))]


def run_c4(args, orc):
    import numpy as np
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    ss = np.random.SeedSequence(0).spawn(4)
    groups, meshes = [], []
    for (cell, p, dims), s in zip(C4_GROUPS, ss):
        seed = int(s.generate_state(1)[0])
        m = (meshgen.tet_mesh(dims, p, alpha=0.15, seed=seed) if cell == "tet"
             else meshgen.hex_mesh(dims, p, alpha=0.15, seed=seed))
        lm = meshgen.lame_cell(m.n_cells, seed=seed)
        meshes.append((m, lm))
        groups.append(dict(cell=cell, order=p,
                           coords=torch.from_numpy(m.coords).to(dev),
                           conn=torch.from_numpy(m.conn).to(dev),
                           material=torch.from_numpy(lm).to(dev).float(),
                           forms=("mass", "laplace", "elasticity")))
    n_cells = sum(m.n_cells for m, _ in meshes)
    out_bytes = sum(m.n_cells * 4 * (2 * m.n_basis ** 2 + 9 * m.n_basis ** 2)
                    for m, _ in meshes)
    tuned = fe.Batch(groups, precision="fp32", autotune=True)
    wall, per = time_calls(tuned.run, args.steps, args.warmup)
    tuned.check()
    errs = {}
    for (m, lm), o in zip(meshes, tuned.outputs):
        idx = sample_cells(m.n_cells, 16)
        sub = submesh(m, idx)
        ti = torch.as_tensor(idx, device=dev)
        errs[f"{m.cell}{m.order}"] = max(
            rel_err(o["mass"][ti].cpu().numpy(), orc.matrix(sub, "mass")),
            rel_err(o["laplace"][ti].cpu().numpy(),
                    orc.matrix(sub, "laplace")),
            rel_err(o["elasticity"][ti].cpu().numpy(),
                    orc.matrix(sub, "elasticity", lm[idx], "iso_cell")))
    tiles = tuned.tiles
    del tuned
    torch.cuda.empty_cache()
    extra = {}
    if not args.no_extra:
        default = fe.Batch(groups, precision="fp32", autotune=False)
        _, pd = time_calls(default.run, args.steps, args.warmup)
        extra["untuned_batch_ms"] = mean(pd)
        extra["untuned_tiles"] = default.tiles
        del default
        torch.cuda.empty_cache()
        # the same work as 12 separate single-form launches
        plans = []
        for g, (m, lm) in zip(groups, meshes):
            for form in ("mass", "laplace", "elasticity"):
                kind = "iso_cell" if form == "elasticity" else None
                pl = fe.Plan(g["cell"], g["order"], form, "matrix", "fp32",
                             material=kind)
                o = torch.empty(pl.out_shape(m.n_cells), dtype=torch.float32,
                                device=dev)
                plans.append((pl, g, o, kind))

        def separate():
            for pl, g, o, kind in plans:
                pl(g["coords"], g["conn"],
                   material=g["material"] if kind else None, out=o)

        _, ps = time_calls(separate, args.steps, args.warmup)
        extra["separate_launches_ms"] = mean(ps)
        extra["separate_variants"] = [pl.variant for pl, *_ in plans]
        del plans
        torch.cuda.empty_cache()
    ms = wall * 1e3 / args.steps
    kms = mean(per)
    gbs = out_bytes / (kms * 1e-3) / 1e9
    line = base_line(args, n_cells / (ms * 1e-3) / 1e9, ms, "f32",
                     dict(workload="batched uneven mesh in one graph launch:"
                          " 300k P1 tet, 120k P2 tet, 200k Q1 hex, 40k Q2 "
                          "hex; mass + Laplace + elasticity each",
                          cells=n_cells, alpha=0.15, seed=0))
    line["batch_ms"] = kms
    line["tiles"] = tiles
    line["out_gb"] = out_bytes / 1e9
    line["max_rel_err_vs_fp64_oracle"] = errs
    line["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "traffic": traffic("k_batch<float>@c4"),
                        "kernel": "k_batch<float>",
                        "kernel_ms": kms}
    line.update(extra)
    if not args.no_cpu:
        def call(k):
            # the same fraction k / n_cells of every group, all three forms
            t = time.perf_counter()
            for m, lm in meshes:
                kg = max(1, int(round(m.n_cells * k / n_cells)))
                sub = submesh(m, slice(0, kg))
                orc.matrix(sub, "mass")
                orc.matrix(sub, "laplace")
                orc.matrix(sub, "elasticity", lm[:kg], "iso_cell")
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"the first {k2 / n_cells:.2%} of every "
            f"group ({k2} cells) x {reps} passes, mass + Laplace + elasticity"
            f" matrices FP64, {tot:.1f} s")
    return line


# ------------------------------------------------------------------- c5 ---

def run_c5(args, orc):
    import numpy as np
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 32
    mesh = meshgen.hex_mesh(n, 2, alpha=0.15, seed=0)
    c = meshgen.lame_qp(mesh.n_cells, 27, seed=0)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=0)
    C = torch.from_numpy(mesh.conn).to(dev)
    gm_ref, gx_ref = orc.energy_grad(mesh, c, U)
    J_ref = orc.energy(mesh, "elasticity", U, c, "iso_qp").sum()
    out = {}
    for prec in ("fp64", "fp32"):
        ep = fe.ElasticEnergyPlan("hex", 2, C, mesh.n_nodes, prec)
        dt = ep.eval.dtype
        ct = torch.from_numpy(c).to(dev).to(dt).requires_grad_(True)
        xt = torch.from_numpy(mesh.coords).to(dev).requires_grad_(True)
        ut = torch.from_numpy(U).to(dev).to(dt).requires_grad_(True)

        def step():
            ct.grad = xt.grad = ut.grad = None
            J = fe.ElasticEnergy(ct, xt, ut, ep)
            J.backward()
            return J

        wall, per = time_calls(step, args.steps, args.warmup)
        J = step()
        torch.cuda.synchronize()

        def rel(a, b):
            return float(np.abs(a - b).max() / np.abs(b).max())

        # the adjoint launch chain alone (pencil adjoint kernel + CSR node
        # sums), buffers preallocated, timed with events on its stream
        from paper_2107_04121_amd import _energy_grad, energy_grad_workspace
        ws = energy_grad_workspace(ep.eval, mesh.n_cells, dev)
        gmb, gxb = torch.empty_like(ct), torch.empty_like(xt)
        cd, ud = ct.detach(), ut.detach()
        _, per_adj = time_calls(
            lambda: _energy_grad(ep.eval, ep.inc, xt.detach(), C, cd, ud, 1.0,
                                 ws=ws, gm=gmb, gx=gxb, check=False),
            args.steps, args.warmup)
        ep.eval.check(ws)
        esz = cd.element_size()
        # algorithmic bytes: coords, conn, c, u read once; dJ/dc, dJ/dx
        # written once
        adj_bytes = (mesh.n_nodes * 24 * 2 + mesh.n_cells * 27 * 4
                     + cd.numel() * esz * 2 + ud.numel() * esz)
        out[prec] = dict(ms_per_step=wall * 1e3 / args.steps,
                         event_ms=mean(per),
                         adjoint_kernel_ms=mean(per_adj),
                         adjoint_alg_bytes=adj_bytes,
                         err_J=abs(float(J) - J_ref) / abs(J_ref),
                         err_dJdc=rel(ct.grad.cpu().numpy(), gm_ref),
                         err_dJdx=rel(xt.grad.cpu().numpy(), gx_ref))
        del ep, ws, gmb, gxb
        torch.cuda.empty_cache()
    p = out["fp64"]
    line = base_line(args, mesh.n_cells / (p["ms_per_step"] * 1e-3) / 1e9,
                     p["ms_per_step"], "f64",
                     dict(workload="adjoint of J = sum u^T K u, Q2 "
                          f"elasticity, {n}^3 cells, per-point lambda,mu: "
                          "forward + dJ/dc, dJ/dx, dJ/du", cells=mesh.n_cells,
                          order=2, alpha=0.15, seed=0))
    line["precisions"] = out
    gbs = p["adjoint_alg_bytes"] / (p["adjoint_kernel_ms"] * 1e-3) / 1e9
    line["roofline"] = {
        "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
        "kernel": "k_sf<2,elasticity,double,adjoint> + CSR node sums",
        "kernel_ms": p["adjoint_kernel_ms"],
        "note": f"{p['adjoint_alg_bytes'] / 1e6:.0f} MB per launch chain "
                "(6.5 us at 8 TB/s): latency-bound, a chain of short "
                "dependent launches"}
    if not args.no_cpu:
        def call(k):
            t = time.perf_counter()
            sub = submesh(mesh, slice(0, k))
            orc.energy(sub, "elasticity", U, c[:k], "iso_qp")
            orc.energy_grad(sub, c[:k], U)
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"{k2} cells x {reps} passes of energy + "
            f"gradient, {tot:.1f} s")
    return line

# ------------------------------------------------------------------- c6 ---

# matrix-core work per Q3 elasticity cell: the 78 upper 16x16 tiles of
# P = g^T g (192 x 192, depth 64 points), 2 flops per multiply-add
C6_MFMA_FLOPS = 78 * 16 * 16 * 64 * 2


def run_c6(args, orc):
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 32
    mesh = meshgen.hex_mesh(n, 3, alpha=0.15, seed=0)
    lm = meshgen.lame_cell(mesh.n_cells, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)
    idx = sample_cells(mesh.n_cells, 24)
    ref = orc.matrix(submesh(mesh, idx), "elasticity", lm[idx], "iso_cell")
    results = {}
    precs = [args.precision] + ([] if args.no_extra else
                                [p for p in ("fp64", "fp32", "bf16x3")
                                 if p != args.precision])
    for prec in precs:
        plan = fe.Plan("hex", 3, "elasticity", "matrix", prec,
                       material="iso_cell", variant=args.variant)
        M = torch.from_numpy(lm).to(dev).to(plan.dtype)
        out = torch.empty(plan.out_shape(mesh.n_cells), dtype=plan.dtype,
                          device=dev)
        wall, per = time_calls(lambda: plan(X, C, material=M, out=out),
                               args.steps, args.warmup)
        plan.check()
        ms = wall * 1e3 / args.steps
        kern_ms = mean(per)
        bpc = alg_bytes_per_cell(mesh, 192, out.element_size(),
                                 M.element_size())
        tflops = C6_MFMA_FLOPS * mesh.n_cells / (kern_ms * 1e-3) / 1e12
        err = rel_err(out[torch.as_tensor(idx, device=dev)].cpu().numpy(),
                      ref)
        results[prec] = dict(ms_per_step=ms, kernel_ms=kern_ms,
                             kernel_ms_min=float(min(per)),
                             gelem_s=mesh.n_cells / (ms * 1e-3) / 1e9,
                             mfma_tflops=tflops,
                             mfma_frac=tflops / MFMA_PEAK_TFLOPS[prec],
                             hbm_gbs=bpc * mesh.n_cells / (kern_ms * 1e-3)
                             / 1e9,
                             variant=plan.variant, max_rel_err=err)
        del out
        torch.cuda.empty_cache()
    prim = results[args.precision]
    line = base_line(args, prim["gelem_s"], prim["ms_per_step"],
                     {"fp64": "f64", "fp32": "f32",
                      "bf16x3": "bf16x3"}[args.precision],
                     dict(workload="linear elasticity element matrices, Q3 "
                          f"hex, {n}^3 cells, 4x4x4 Gauss",
                          cells=mesh.n_cells, order=3, n_basis=64, n_qp=64,
                          alpha=0.15, seed=0,
                          material="per-cell lambda,mu lognormal(0,0.5)"))
    line["max_rel_err_vs_fp64_oracle"] = prim["max_rel_err"]
    line["roofline"] = {"bound": "mfma", "achieved": prim["mfma_tflops"],
                        "peak": MFMA_PEAK_TFLOPS[args.precision],
                        "unit": "TFLOP/s", "frac": prim["mfma_frac"],
                        "traffic": (traffic("k_elast_q3ws<0>")
                                    if args.precision == "fp64" else None),
                        "kernel": "k_elast_q3ws",
                        "kernel_ms": prim["kernel_ms"],
                        "flops_per_cell": C6_MFMA_FLOPS,
                        "hbm_frac": prim["hbm_gbs"] / HBM_PEAK_GBS}
    line["precisions"] = results
    if not args.no_cpu:
        def call(k):
            t = time.perf_counter()
            orc.matrix(submesh(mesh, slice(0, k)), "elasticity", lm[:k],
                       "iso_cell")
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"first {k2} cells of the {n}^3 Q3 mesh x "
            f"{reps} passes, FP64 element matrices, {tot:.1f} s")
    return line


# ------------------------------------------------------------------- c7 ---

def run_c7(args, orc):
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    n = args.n or 32
    mesh = meshgen.hex_mesh(n, 2, alpha=0.15, seed=0)
    nb, nq = mesh.n_basis, 27
    Mt = meshgen.tensor_qp(mesh.n_cells, nq, seed=0)
    U = meshgen.dofs(mesh.n_nodes, 3, seed=0)
    X = torch.from_numpy(mesh.coords).to(dev)
    C = torch.from_numpy(mesh.conn).to(dev)
    idx = sample_cells(mesh.n_cells, 24)
    sub = submesh(mesh, idx)
    paths = {}
    for form in ("wdot", "convect"):
        kind = "tensor_qp" if form == "wdot" else None
        mat = Mt[idx] if kind else None
        refs = {"matrix": orc.matrix(sub, form, mat, kind, u=U),
                "residual": orc.residual(sub, form, U, mat, kind)}
        for mode in ("matrix", "residual"):
            for prec in ("fp64", "fp32"):
                if args.no_extra and prec != "fp64":
                    continue
                plan = fe.Plan("hex", 2, form, mode, prec, material=kind)
                dt = plan.dtype
                Md = torch.from_numpy(Mt).to(dev).to(dt) if kind else None
                Ud = torch.from_numpy(U).to(dev).to(dt)
                out = torch.empty(plan.out_shape(mesh.n_cells), dtype=dt,
                                  device=dev)
                wall, per = time_calls(
                    lambda: plan(X, C, material=Md, dofs=Ud, out=out),
                    args.steps, args.warmup)
                plan.check()
                kms = mean(per)
                esz = out.element_size()
                nd = 3 * nb
                outb = nd * nd * esz if mode == "matrix" else nd * esz
                bpc = (outb + nb * 4 + mesh.n_nodes * (24 + 3 * esz)
                       / mesh.n_cells + (nq * 9 * esz if kind else 0))
                err = rel_err(out[torch.as_tensor(idx, device=dev)].cpu()
                              .numpy(), refs[mode])
                paths[f"{form}/{mode}/{prec}"] = dict(
                    kernel_ms=kms, ms_per_step=wall * 1e3 / args.steps,
                    gelem_s=mesh.n_cells / (kms * 1e-3) / 1e9,
                    alg_bytes_per_cell=bpc,
                    hbm_gbs=bpc * mesh.n_cells / (kms * 1e-3) / 1e9,
                    variant=plan.variant, max_rel_err=err)
                del out
                torch.cuda.empty_cache()
    prim = paths["convect/matrix/fp64"]
    line = base_line(args, prim["gelem_s"], prim["ms_per_step"], "f64",
                     dict(workload="weighted vector dot product and "
                          "Navier-Stokes convection, Q2 hex, "
                          f"{n}^3 cells, 3x3x3 Gauss, matrix and residual",
                          cells=mesh.n_cells, order=2, alpha=0.15, seed=0))
    line["max_rel_err_vs_fp64_oracle"] = prim["max_rel_err"]
    line["roofline"] = {"bound": "hbm", "achieved": prim["hbm_gbs"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": prim["hbm_gbs"] / HBM_PEAK_GBS,
                        "traffic": (traffic("k_hexgm<2,convect,fp64>@32^3")
                                    if n == 32 else None),
                        "kernel": "k_hexgm<2,convect,fp64>",
                        "kernel_ms": prim["kernel_ms"]}
    line["paths"] = paths
    if not args.no_cpu:
        def call(k):
            t = time.perf_counter()
            orc.matrix(submesh(mesh, slice(0, k)), "convect", u=U)
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"first {k2} cells of the {n}^3 Q2 mesh x "
            f"{reps} passes, FP64 convection matrices, {tot:.1f} s")
    return line


# ------------------------------------------------------------------- c8 ---

def c8_flops(form, p):
    """Matrix-core work per cell, counted on the unpadded operands, 2 flops
    per multiply-add over the n_q points: the entries each form needs of its
    products (scalar Laplace: the upper triangle of each of the three
    gradient blocks summed; vector mass: the upper triangle of the scalar
    mass; elasticity: upper triangles of the three diagonal blocks of
    P = g^T g and the three full blocks r < s; weighted dot and convection:
    the nine full blocks Phi^T W_rs; elasticity with per-point D: the nine
    full blocks over 3 n_q (point, gradient component) pairs)."""
    nb = (p + 1) ** 3
    upper = nb * (nb + 1) // 2
    if form == "elasticity_voigt":  # nine full blocks over 3 n_q (point, component) pairs
        return 9 * nb * nb * 2 * 3 * nb
    entries = {"laplace": 3 * upper, "vmass": upper, "elasticity": 3 * upper + 3 * nb * nb,
               "wdot": 9 * nb * nb, "convect": 9 * nb * nb}[form]
    return entries * 2 * nb


def run_c8(args, orc):
    import torch
    import meshgen
    import paper_2107_04121_amd as fe
    dev = torch.device("cuda:0")
    dims = (16, 8, 8)
    paths = {}
    keep = {}
    for p in (4, 5):
        mesh = meshgen.hex_mesh(dims, p, alpha=0.15, seed=0, box=(16.0, 8.0, 8.0),
                                curved=0.02 if p == 4 else 0.005)
        lm = meshgen.lame_cell(mesh.n_cells, seed=0)
        X = torch.from_numpy(mesh.coords).to(dev)
        C = torch.from_numpy(mesh.conn).to(dev)
        idx = sample_cells(mesh.n_cells, 12)
        sub = submesh(mesh, idx)
        keep[p] = (mesh, lm)
        Mt = meshgen.tensor_qp(mesh.n_cells, mesh.n_basis, seed=0)
        Dv = meshgen.voigt_random_spd((mesh.n_cells, mesh.n_basis), seed=0)
        for label in ("laplace", "vmass", "wdot", "convect", "elasticity", "elasticity_voigt"):
            form = "elasticity" if label.startswith("elasticity") else label
            kind = {"elasticity": "iso_cell", "elasticity_voigt": "voigt_qp", "wdot": "tensor_qp"}.get(label)
            mat = {"iso_cell": lm, "tensor_qp": Mt, "voigt_qp": Dv}.get(kind)
            nc = 1 if form == "laplace" else 3
            nd = nc * mesh.n_basis
            U = meshgen.dofs(mesh.n_nodes, nc, seed=0)
            refs = {"matrix": orc.matrix(sub, form, mat[idx] if kind else None, kind,
                                         u=U if form == "convect" else None),
                    "residual": orc.residual(sub, form, U, mat[idx] if kind else None, kind)}
            mprecs = (("fp64", "fp32") if form in ("wdot", "convect") or kind == "voigt_qp"
                      else ("fp64", "fp32", "bf16x3"))
            for mode, precs in (("matrix", mprecs), ("residual", ("fp64", "fp32"))):
                for prec in precs:
                    primary = (p == 5 and label == "elasticity" and mode == "matrix"
                               and prec == args.precision)
                    if args.no_extra and not primary:
                        continue
                    plan = fe.Plan("hex", p, form, mode, prec, material=kind)
                    dt = plan.dtype
                    M = torch.from_numpy(mat).to(dev).to(dt) if kind else None
                    Ud = (torch.from_numpy(U).to(dev).to(dt)
                          if mode == "residual" or form == "convect" else None)
                    out = torch.empty(plan.out_shape(mesh.n_cells), dtype=dt, device=dev)
                    wall, per = time_calls(lambda: plan(X, C, material=M, dofs=Ud, out=out),
                                           args.steps, args.warmup)
                    plan.check()
                    kms = mean(per)
                    esz = out.element_size()
                    outb = nd * nd * esz if mode == "matrix" else nd * esz
                    matb = {"iso_cell": 2 * esz, "tensor_qp": 9 * mesh.n_basis * esz,
                            "voigt_qp": 36 * mesh.n_basis * esz}.get(kind, 0)
                    bpc = (outb + mesh.n_basis * 4 + matb
                           + mesh.n_nodes * (24 + (nc * esz if Ud is not None else 0)) / mesh.n_cells)
                    err = rel_err(out[torch.as_tensor(idx, device=dev)].cpu().numpy(), refs[mode])
                    r = dict(kernel_ms=kms, ms_per_step=wall * 1e3 / args.steps,
                             gelem_s=mesh.n_cells / (wall / args.steps) / 1e9,
                             hbm_gbs=bpc * mesh.n_cells / (kms * 1e-3) / 1e9,
                             alg_bytes_per_cell=bpc, variant=plan.variant, max_rel_err=err)
                    if mode == "matrix":
                        fl = c8_flops(label, p)
                        tf = fl * mesh.n_cells / (kms * 1e-3) / 1e12
                        r.update(mfma_tflops=tf, mfma_frac=tf / MFMA_PEAK_TFLOPS[prec], flops_per_cell=fl)
                    paths[f"q{p}/{label}/{mode}/{prec}"] = r
                    del out
                    torch.cuda.empty_cache()
    prim = paths[f"q5/elasticity/matrix/{args.precision}"]
    line = base_line(args, prim["gelem_s"], prim["ms_per_step"],
                     {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[args.precision],
                     dict(workload="orders 4-5 of the table of cell and DOF counts: 1,024 "
                          "hexahedra (16 x 8 x 8 unit cells); primary Q5 linear-elasticity "
                          "element matrices (216 nodes, 648 DOFs, 6x6x6 Gauss, 3.4 GB in FP64)",
                          cells=1024, order=5, n_basis=216, n_qp=216, alpha=0.15, seed=0,
                          material="per-cell lambda,mu lognormal(0,0.5)"))
    line["max_rel_err_vs_fp64_oracle"] = prim["max_rel_err"]
    line["roofline"] = {"bound": "mfma", "achieved": prim["mfma_tflops"],
                        "peak": MFMA_PEAK_TFLOPS[args.precision], "unit": "TFLOP/s",
                        "frac": prim["mfma_frac"],
                        "traffic": (traffic("k_hexmc<5,3,0>") if args.precision == "fp64" else None),
                        "kernel": "k_hexmc<5,elasticity>", "kernel_ms": prim["kernel_ms"],
                        "flops_per_cell": prim["flops_per_cell"],
                        "hbm_frac": prim["hbm_gbs"] / HBM_PEAK_GBS}
    line["paths"] = paths
    if not args.no_cpu:
        mesh, lm = keep[5]

        def call(k):
            t = time.perf_counter()
            orc.matrix(submesh(mesh, slice(0, k)), "elasticity", lm[:k], "iso_cell")
            return time.perf_counter() - t
        line["cpu_baseline"] = cpu_baseline(
            orc, call, mesh.n_cells, args.cpu_seconds,
            lambda k2, reps, tot: f"first {k2} cells of the 1,024-cell Q5 mesh x {reps} "
            f"passes, FP64 elasticity matrices, {tot:.1f} s")
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (the "
                          "multi-GPU sharding is designed, not built); "
                          "--gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch  # noqa: F401
    import oracle  # test infrastructure: error vs FP64 oracle, CPU baseline
    oracle.build()
    copy_calibration(args.copy_calibration)
    runs = {"c1": run_c1, "c2": run_c2, "c3": run_c3, "c4": run_c4,
            "c5": run_c5, "c6": run_c6, "c7": run_c7, "c8": run_c8}
    if args.config != "all":
        line = runs[args.config](args, oracle)
        print(json.dumps(line))
        sys.exit(1 if "error" in line else 0)
    # the headline workload (c2), then the other four configurations, each a
    # complete record of its own (value, roofline, cpu_baseline, errors)
    line = run_c2(args, oracle)
    if "error" in line:
        print(json.dumps(line))
        sys.exit(1)
    print(f"c2 done: {line['ms_per_step']:.3f} ms/step", file=sys.stderr,
          flush=True)
    line["configs"] = {}
    for name in ("c1", "c3", "c4", "c5"):
        t0 = time.perf_counter()
        try:
            sub = runs[name](args, oracle)
        except Exception as e:  # recorded, the headline stands
            sub = {"error": f"{type(e).__name__}: {e}"}
        line["configs"][name] = sub
        import torch
        torch.cuda.empty_cache()
        print(f"{name} done in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
