"""Benchmark: implicit gas-kinetic scheme iterations on one MI355X.

A step is one full nonlinear iteration (Eq.16 residual with the GKS face
flux, Eq.25 CFL law, LU-SGS forward and backward sweeps, update) over
every cell of the workload mesh; the metric is cell-updates per second
(cells x iterations / wall time), inputs resident in HBM.

Default workload: Joukowski airfoil hybrid mesh (128 wall points, 30 quad
layers, first height 1e-4 chord, growth 1.12, seeded Delaunay triangles out
to 20 chords, ~40k cells, colour-ordered), Ma 0.5, Re 5000, alpha 2 deg,
laminar, FP64.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "jouk40k": dict(flow=(0.5, 2.0, 5000.0, -1.0), desc="Joukowski hybrid, 128 wall pts, 30 quad layers (1e-4, 1.12), "
                                                       "seeded Delaunay to r=20 chords, Ma 0.5 Re 5000 alpha 2, laminar"),
    "jouk250k": dict(flow=(0.15, 4.0, 6e6, 3.0), desc="Joukowski hybrid, 512 wall pts, 60 quad layers (2e-6, 1.15), "
                                                      "Ma 0.15 Re 6e6 alpha 4, SA nu~/nu = 3"),
    "jouk2m": dict(flow=(0.15, 4.0, 6e6, 3.0), desc="Joukowski hybrid, 2048 wall pts, 90 quad layers (1e-6, 1.10), "
                                                    "Ma 0.15 Re 6e6 alpha 4, SA nu~/nu = 3"),
    "plate64x32": dict(flow=(0.3, 0.0, 1e4, -1.0), desc="laminar flat plate 64x32 quads, Ma 0.3 Re_L 1e4"),
}

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_VALU_PEAK_TFS = 78.6   # MI355X FP64 vector
# FP64 operations per face of k_flux, counted with rocprofv3
# (SQ_INSTS_VALU_FMA_F64 x 2 + MUL + ADD + TRANS, per wave / faces per wave)
FLUX_FLOP_PER_FACE = 3918.0
KSRC = os.path.join(ROOT, "paper_1709_00803_amd", "csrc", "igks_kernels.hip")


def kernel_bytes(n, f, e, sa, mixed):
    """Compulsory HBM bytes per launch of each kernel class: every array
    element the kernel needs is counted once (neighbour re-reads assumed
    cached).  n cells, f faces, e cell-face entries."""
    d = 8
    dw = 4 if mixed else 8
    b = {}
    b["prep"] = 5 * d * n + 4 * n + (4 + 4 + 8 + 8) * e + 3 * d * f + (3 + 1) * d * n + (3 + 8) * d * n
    b["flux"] = (8 + 3 * d + 4 * d + 3 * d) * f + (5 + 8) * d * n + (4 + 1 + (2 if sa else 0)) * d * f
    b["gather"] = 4 * n + 8 * e + (4 + 2) * d * f + (5 + 1) * d * n + (5 + 1 + (1 if sa else 0)) * d * n \
        + ((2 + 3) * d * f + 4 * e if sa else 0)
    sweep = (5 + 1 + 1 + 1 + (1 if sa else 0)) * d * n + 4 * n + 12 * e + 4 * d * f + 5 * dw * n
    b["sweep_fwd"] = sweep + 5 * d * n                      # + M
    b["sweep_bwd"] = sweep + 5 * dw * n                     # + own dW*
    b["update"] = 5 * d * n + 5 * dw * n + 5 * d * n
    b["reduce"] = 2 * d * ((n + 255) // 256)
    return b


def kernel_source_hash():
    import hashlib
    return hashlib.sha256(open(KSRC, "rb").read()).hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (profiles/traffic_<workload>.json), or None when the kernels
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


def time_to_drop(igks, mg, precision, target=1e-10, max_it=20000):
    """Iterations and seconds from the impulsive start to a density-residual
    drop of `target` on the laminar flat plate (64x32, natural order)."""
    import torch
    m = mg.flat_plate()
    s = igks.Solver(m, precision=precision, cfl_init=10.0, chunk=100)
    s.set_freestream(*WORKLOADS["plate64x32"]["flow"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < max_it:
        s.iterate(100)
        it += 100
        if s.residual()["res_drop"] <= target:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    wl = s.wall_loads()
    return dict(iterations=it, seconds=round(dt, 4), drop=s.residual()["res_drop"], cd=wl["cd"],
                cell_updates_per_s=m.n_cells * it / dt)


def run_cpu_baseline(mesh, flow, budget_s=12.0, max_it=60):
    from oracle import pyoracle as po
    o = po.Oracle(mesh)
    o.set_freestream(*flow)
    o.iterate(1)     # the impulsive-start iteration, untimed
    t0 = time.perf_counter()
    it = 0
    while it < max_it:
        o.iterate(1)
        it += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=mesh.n_cells * it / dt, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{it} iterations of the same workload after one untimed start iteration, "
                       f"single-threaded FP64 C oracle, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="jouk40k", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--chunk", type=int, default=20)
    ap.add_argument("--profile-iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-drop", action="store_true", help="skip the time-to-1e-10 runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the batched and single-mesh paths are single-GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_00803_amd import igks
    from paper_1709_00803_amd import meshgen as mg

    wl = WORKLOADS[args.workload]
    t = time.perf_counter()
    mesh = mg.workload(args.workload)
    t_mesh = time.perf_counter() - t
    mixed = args.precision == "mixed"
    torch.cuda.set_device(0)
    solver = igks.Solver(mesh, precision=igks.IGKS_MIXED if mixed else igks.IGKS_FP64, chunk=args.chunk)
    solver.set_freestream(*wl["flow"])
    sa = wl["flow"][3] >= 0
    print(f"# mesh {args.workload}: {mesh.n_cells} cells, {solver.nf} faces, {solver.nlev} wavefronts, "
          f"generated in {t_mesh:.1f}s", file=sys.stderr, flush=True)

    solver.iterate(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.iterate(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n = mesh.n_cells
    value = n * args.steps / elapsed
    res = solver.residual()
    print(f"# timed {args.steps} iterations in {elapsed:.3f}s, drop {res['res_drop']:.3e}", file=sys.stderr,
          flush=True)

    # per-kernel durations: HIP events on the library's stream, direct launches
    solver.set_profiling(True)
    solver.iterate(args.profile_iters)
    kt = solver.kernel_times()      # ms per iteration, per kernel class
    solver.set_profiling(False)
    e = int(np.sum(np.diff(mesh.cell_ptr)))
    kb = kernel_bytes(n, solver.nf, e, sa, mixed)
    dom = max(kt, key=lambda k: kt[k])
    launches = {"sweep_fwd": solver.nlev, "sweep_bwd": solver.nlev}.get(dom, 1)
    t_ms = kt[dom]
    if dom == "flux":
        achieved = FLUX_FLOP_PER_FACE * solver.nf / (t_ms * 1e-3) / 1e12 if t_ms > 0 else 0.0
        roofline = dict(kernel=dom, bound="alu", achieved=achieved, peak=FP64_VALU_PEAK_TFS, unit="TFLOP/s",
                        frac=achieved / FP64_VALU_PEAK_TFS)
    else:
        achieved = kb[dom] / launches / (t_ms / launches * 1e-3) / 1e9 if t_ms > 0 else 0.0
        roofline = dict(kernel=dom, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=achieved / HBM_PEAK_GBS)
    tr = measured_traffic(args.workload, dom) if not mixed else None
    roofline.update(traffic=tr, launches_per_step=launches, ms_per_step=t_ms,
                    algorithmic_bytes_per_step=kb[dom],
                    kernel_ms_per_step={k: round(v, 5) for k, v in kt.items()})
    # the face-flux kernel against the FP64 vector peak, whatever dominates
    tf = kt.get("flux", 0.0)
    roofline["flux_fp64_tflops"] = FLUX_FLOP_PER_FACE * solver.nf / (tf * 1e-3) / 1e12 if tf > 0 else 0.0

    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "cells": n, "faces": solver.nf,
                   "wavefronts": solver.nlev, "precision": args.precision, "ordering": "colour",
                   "chunk": args.chunk, "res_drop_after": res["res_drop"]},
        "roofline": roofline,
    }
    if not args.no_drop:
        out["time_to_1e-10"] = {"workload": "plate64x32 (natural order), Ma 0.3 Re_L 1e4, CFL 10 -> Eq.25",
                                "fp64": time_to_drop(igks, mg, igks.IGKS_FP64),
                                "mixed": time_to_drop(igks, mg, igks.IGKS_MIXED)}
    if not args.no_cpu:
        out["cpu_baseline"] = run_cpu_baseline(mesh, wl["flow"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
