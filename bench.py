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
import math
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
    "batch64": dict(flow=None, desc="64 seeded instances (default_rng(1000+b)): even b flat plate, odd b Joukowski "
                                    "hybrid, cells log-uniform 5e3-2e5, Ma U[0.1,0.6], alpha U[-4,12] (airfoils), "
                                    "Re log-uniform 1e4-1e7, SA iff Re>1e5; one graph launch per chunk, autotuned"),
}
# plate variants of the batched time-to-1e-10 comparison: (Ma, Re_L)
DROP_BATCH = [(0.2, 5e3), (0.25, 8e3), (0.3, 1e4), (0.35, 1.5e4), (0.4, 2e4), (0.3, 6e3), (0.2, 1.2e4), (0.4, 1e4)]

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_VALU_PEAK_TFS = 78.6   # MI355X FP64 vector
# FP64 operations per face of k_flux, counted with rocprofv3: FP64 VALU
# instructions per wave (2 x FMA + MUL + ADD + TRANS); one face per lane, so
# this is also the operation count of one face.
FLUX_FLOP_PER_FACE = 3488.0
KSRC = os.path.join(ROOT, "paper_1709_00803_amd", "csrc", "igks_kernels.hip")


def kernel_bytes(n, f, e, sa, mixed):
    """Compulsory HBM bytes per iteration of each kernel class: every array
    element a kernel needs is counted once (re-reads of neighbour data are
    assumed to hit in cache); limiter off.  n cells, f faces, e cell-face
    entries; sa: the SA equation is on."""
    d, i4 = 8, 4
    dw = 4 if mixed else 8
    s = 1 if sa else 0
    b = {}
    # W, cinst, cf_ptr; cf_face/cf_nbr/cf_dx/cf_dy; face normal and length;
    # lsinv, area; writes nu, lamc, vort, gradients
    b["prep"] = 5 * d * n + 2 * i4 * n + (2 * i4 + 2 * d) * e + 3 * d * f + 4 * d * n + (3 + 8) * d * n
    # fl, fr, finst; normal, length, face-centre offsets, distances; W and
    # gradients of both sides; writes flux, lam (+ SA saf, sag, sak)
    b["flux"] = (3 * i4 + 10 * d) * f + (5 + 8) * d * n + (4 + 1 + 3 * s) * d * f
    # cinst, cf_ptr, ipos; cf_face/cf_flag; flux, lam, length (+ SA: saf, sag,
    # sak, normal); W (+ SA: nu, wall distance, vorticity, area); writes M,
    # lsum, r2 (+ SA diagonal)
    b["gather"] = 3 * i4 * n + 2 * i4 * e + 6 * d * f + 5 * d * n + (5 + 1 + 2) * d * n \
        + s * (5 * d * f + 4 * d * n + d * n)
    b["reduce"] = 2 * d * n
    # cinst, cf_ptr; cf_nbr/cf_flag/cf_face; normal, length, lam (+ sak) of
    # the faces swept; W, lamc, lsum (+ SA diagonal); writes dW
    sweep = 2 * i4 * n + 3 * i4 * e + (4 + s) * d * f + (5 + 2 + s) * d * n + 5 * dw * n
    b["sweep_fwd"] = sweep + 5 * d * n                      # + M
    b["sweep_bwd"] = sweep + 5 * dw * n + 5 * d * n         # + own dW*, writes W^{n+1}
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


def time_to_drop(igks, mg, precision, target=1e-10, max_it=20000, scheme=0, cfl=10.0, chunk=100):
    """Iterations and seconds from the impulsive start to a density-residual
    drop of `target` on the laminar flat plate (64x32, natural order);
    scheme 1: the explicit scheme (Eq.15, local steps at a fixed CFL)."""
    import torch
    m = mg.flat_plate()
    s = igks.Solver(m, precision=precision, cfl_init=cfl, chunk=chunk, scheme=scheme)
    s.set_freestream(*WORKLOADS["plate64x32"]["flow"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < max_it:
        s.iterate(chunk)
        it += chunk
        if s.residual()["res_drop"] <= target:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    wl = s.wall_loads()
    return dict(iterations=it, seconds=round(dt, 4), drop=s.residual()["res_drop"], cd=wl["cd"],
                cell_updates_per_s=m.n_cells * it / dt)


def time_to_converge_cavity(igks, mg, max_it=20000, chunk=200):
    """The lid-driven cavity (100x100, Re 1000, Ma 0.1 sqrt 3, isothermal
    walls) from rest, implicit CFL 1000 growing by Eq.25, to the paper's
    criterion Eq.40 <= 3e-8."""
    import torch
    m = mg.cavity(100)
    s = igks.Solver(m, cfl_init=1000.0, chunk=chunk, wall_temp=1.0)
    s.set_freestream(0.1 * math.sqrt(3.0), 0.0, 1000.0)
    W = s.get_state()
    W[3] -= 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0]
    W[1] = W[2] = 0.0
    s.set_state(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < max_it:
        s.iterate(chunk)
        it += chunk
        if s.residual()["eq40"] <= 3e-8:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = s.residual()
    return dict(workload="cavity100: 100x100 uniform, Re 1000, Ma 0.1 sqrt(3), isothermal walls, from rest",
                criterion="Eq.40 <= 3e-8", iterations=it, seconds=round(dt, 4), eq40=r["eq40"],
                drop=r["res_drop"], cfl=r["cfl"], ms_per_iteration=round(1e3 * dt / it, 4),
                paper_iterations=4430, paper_seconds=543.2)


def time_to_converge_turbulent_plate(igks, mg, max_it=30000, chunk=500):
    """The turbulent flat plate (SA, Ma 0.2, Re 5e6 per unit length, 7680
    cells, natural order) from the free stream at CFL 10 growing by Eq.25,
    to the paper's criterion Eq.40 <= 3e-8."""
    import torch
    m = mg.turbulent_plate()
    s = igks.Solver(m, cfl_init=10.0, chunk=chunk)
    s.set_freestream(0.2, 0.0, 5e6, 3.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < max_it:
        s.iterate(chunk)
        it += chunk
        if s.residual()["eq40"] <= 3e-8:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = s.residual()
    return dict(workload="turbulent flat plate: 120x64 quads, y+ ~ 1, Ma 0.2, Re 5e6/unit length, SA, from the free stream",
                criterion="Eq.40 <= 3e-8", iterations=it, seconds=round(dt, 4), eq40=r["eq40"],
                drop=r["res_drop"], cd=s.wall_loads()["cd"], ms_per_iteration=round(1e3 * dt / it, 4),
                paper_iterations=5340, paper_seconds=1087.7)


def time_to_drop_batch(igks, mg, target=1e-10, max_it=20000):
    """Eight plate flow conditions (DROP_BATCH) to a `target` drop: one mixed-
    precision batch against the eight FP64 single runs one after another."""
    import torch
    m = mg.flat_plate()
    flows = [(ma, 0.0, re, -1.0) for ma, re in DROP_BATCH]
    b = igks.BatchSolver([m] * len(flows), precision=igks.IGKS_MIXED, cfl_init=10.0, chunk=100)
    for i, f in enumerate(flows):
        b.set_freestream(i, *f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, first = 0, [None] * len(flows)
    while it < max_it and any(x is None for x in first):
        b.iterate(100)
        it += 100
        for i in range(len(flows)):
            if first[i] is None and b.residual(i)["res_drop"] <= target:
                first[i] = it
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t_seq, its_seq = 0.0, []
    for f in flows:
        s = igks.Solver(m, precision=igks.IGKS_FP64, cfl_init=10.0, chunk=100)
        s.set_freestream(*f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = 0
        while k < max_it:
            s.iterate(100)
            k += 100
            if s.residual()["res_drop"] <= target:
                break
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        its_seq.append(k)
    return dict(instances=len(flows), flows_ma_re=DROP_BATCH, batch_mixed_seconds=round(t_batch, 4),
                batch_iterations_to_target=first, fp64_sequential_seconds=round(t_seq, 4),
                fp64_iterations_to_target=its_seq, speedup=round(t_seq / t_batch, 3))


def run_cpu_baseline(cases, budget_s=12.0, max_it=60):
    """The oracle on a bounded sample: iterations of the given (mesh, flow)
    cases in turn after one untimed start iteration each, ~budget_s."""
    from oracle import pyoracle as po
    cells, its, dt = 0, 0, 0.0
    names = []
    for mesh, flow in cases:
        o = po.Oracle(mesh)
        o.set_freestream(*flow)
        o.iterate(1)     # the impulsive-start iteration, untimed
        t0 = time.perf_counter()
        it = 0
        while it < max_it:
            o.iterate(1)
            it += 1
            if dt + time.perf_counter() - t0 > budget_s:
                break
        dt += time.perf_counter() - t0
        cells += mesh.n_cells * it
        its += it
        names.append(f"{mesh.n_cells} cells x {it}")
        if dt > budget_s:
            break
    return dict(value=cells / dt, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"iterations of the same workload ({'; '.join(names)}) after one untimed start iteration "
                       f"each, single-threaded FP64 C oracle, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed iterations; at least --chunk, so the timed chunks replay an already captured graph")
    ap.add_argument("--workload", default="jouk40k", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64, mixed for batch64")
    ap.add_argument("--chunk", type=int, default=100,
                    help="iterations per captured HIP graph (one host synchronisation per chunk)")
    ap.add_argument("--profile-iters", type=int, default=20)
    ap.add_argument("--autotune", type=int, default=None, help="autotuner iterations per candidate (default 5, 0: off)")
    ap.add_argument("--cfl-init", type=float, default=None, help="initial implicit CFL (default: 1000, 10 for batch64)")
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
    batched = args.workload == "batch64"
    precision = args.precision or ("mixed" if batched else "fp64")
    mixed = precision == "mixed"
    tune = args.autotune if args.autotune is not None else 5
    t = time.perf_counter()
    if batched:
        meshes, flows = mg.batch(64)
    else:
        meshes, flows = [mg.workload(args.workload)], [wl["flow"]]
    t_mesh = time.perf_counter() - t
    torch.cuda.set_device(0)
    prec = igks.IGKS_MIXED if mixed else igks.IGKS_FP64
    cfl0 = args.cfl_init if args.cfl_init is not None else (10.0 if batched else 1000.0)
    if batched:
        solver = igks.BatchSolver(meshes, precision=prec, chunk=args.chunk, cfl_init=cfl0)
        for i, f in enumerate(flows):
            solver.set_freestream(i, *f)
        nfs = solver.nf
    else:
        solver = igks.Solver(meshes[0], precision=prec, chunk=args.chunk, cfl_init=cfl0)
        solver.set_freestream(*flows[0])
        nfs = [solver.nf]
    n = solver.total_cells
    print(f"# {args.workload}: {len(meshes)} instance(s), {n} cells, {solver.total_faces} faces, "
          f"{solver.nlev} wavefronts, generated in {t_mesh:.1f}s", file=sys.stderr, flush=True)
    schedule = solver.autotune(tune).tolist() if tune > 0 else solver.schedule().tolist()

    def run(k):
        """k iterations; a batch instance frozen by a rejected update is
        reported, not fatal: the others go on."""
        try:
            solver.iterate(k)
        except igks.IgksError as e:
            if not batched or e.code != igks.IGKS_ENONPHYS:
                raise
            print(f"# {e}", file=sys.stderr, flush=True)

    def committed():
        if batched:
            return [solver.residual(i)["iteration"] for i in range(len(meshes))]
        return [solver.residual()["iteration"]]

    run(args.warmup)
    c0 = committed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # cell updates actually committed (frozen instances do not count)
    updates = sum(m.n_cells * (b - a) for m, a, b in zip(meshes, c0, committed()))
    value = updates / elapsed
    if batched:
        drops = [solver.residual(i)["res_drop"] for i in range(len(meshes))]
        frozen = [i for i in range(len(meshes)) if solver.status(i)]
        res_info = dict(res_drop_after_min=min(drops), res_drop_after_median=float(np.median(drops)),
                        res_drop_after_max=max(drops), frozen_instances=frozen)
    else:
        res_info = dict(res_drop_after=solver.residual()["res_drop"])
    print(f"# timed {args.steps} iterations in {elapsed:.3f}s, {res_info}", file=sys.stderr, flush=True)

    # per-kernel durations: HIP events on the library's stream, direct launches
    solver.set_profiling(True)
    run(args.profile_iters)
    kt = solver.kernel_times()      # ms per iteration, per kernel class
    solver.set_profiling(False)
    kb = {}
    for m, f, nf in zip(meshes, flows, nfs):
        e = int(np.sum(np.diff(m.cell_ptr)))
        for k, v in kernel_bytes(m.n_cells, nf, e, f[3] >= 0, mixed).items():
            kb[k] = kb.get(k, 0) + v
    faces = solver.total_faces
    dom = max(kt, key=lambda k: kt[k])
    sweep_wg = schedule[4] == 2
    if not sweep_wg and solver.nlev > 1:
        # one launch per wavefront: the forward class covers wavefronts
        # 1 .. nlev-1 (the first wavefront's forward increments are formed
        # where they are read), the backward class wavefronts nlev-2 .. 0 (the
        # last one's backward step runs in the forward class's last launch);
        # their bytes are the per-cell model over the cells they process
        sizes = solver.wavefront_sizes()
        ntot = float(sizes.sum())
        kb["sweep_fwd"] *= (ntot - sizes[0]) / ntot
        kb["sweep_bwd"] *= (ntot - sizes[-1]) / ntot
    launches = {"sweep_fwd": 1 if sweep_wg else max(solver.nlev - 1, 1),
                "sweep_bwd": 1 if sweep_wg else max(solver.nlev - 1, 1)}.get(dom, 1)
    t_ms = kt[dom]
    # the launch duration of the dominant kernel: the residual-phase kernels
    # (which only write derived arrays) are timed over back-to-back launches
    # between two events, so the events' own cost is spread over them; the
    # sweeps (which change the state) by their event interval in the pass above
    launch_ms = solver.time_kernel(dom, 50) if dom in ("prep", "flux", "gather") else t_ms / launches
    if dom == "flux":
        achieved = FLUX_FLOP_PER_FACE * faces / (launch_ms * 1e-3) / 1e12 if launch_ms > 0 else 0.0
        roofline = dict(kernel=dom, bound="alu", achieved=achieved, peak=FP64_VALU_PEAK_TFS, unit="TFLOP/s",
                        frac=achieved / FP64_VALU_PEAK_TFS)
    else:
        achieved = kb[dom] / launches / (launch_ms * 1e-3) / 1e9 if launch_ms > 0 else 0.0
        roofline = dict(kernel=dom, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=achieved / HBM_PEAK_GBS)
    tr = measured_traffic(args.workload, dom) if not mixed or batched else None
    roofline.update(traffic=tr, launches_per_step=launches, ms_per_step=t_ms, ms_per_launch=launch_ms,
                    algorithmic_bytes_per_step=kb.get(dom),
                    kernel_ms_per_step={k: round(v, 5) for k, v in kt.items()})
    tf = launch_ms if dom == "flux" else solver.time_kernel("flux", 50)
    roofline["flux_fp64_tflops"] = FLUX_FLOP_PER_FACE * faces / (tf * 1e-3) / 1e12 if tf > 0 else 0.0
    roofline["hbm_gbs_per_kernel"] = {k: round(kb[k] / (kt[k] * 1e-3) / 1e9, 1) for k in kb if kt.get(k, 0) > 0}

    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": dict({"workload": f"{args.workload}: {wl['desc']}", "instances": len(meshes), "cells": n,
                        "faces": faces, "wavefronts": solver.nlev, "precision": precision, "ordering": "colour",
                        "cfl_init": cfl0, "chunk": args.chunk, "schedule": schedule,
                        "cell_updates_timed": updates}, **res_info),
        "roofline": roofline,
    }
    if not args.no_drop:
        out["time_to_1e-10"] = {"workload": "plate64x32 (natural order), Ma 0.3 Re_L 1e4, CFL 10 -> Eq.25",
                                "fp64": time_to_drop(igks, mg, igks.IGKS_FP64),
                                "mixed": time_to_drop(igks, mg, igks.IGKS_MIXED),
                                "batched_plates": time_to_drop_batch(igks, mg),
                                "explicit_fp64_cfl0.9": time_to_drop(igks, mg, igks.IGKS_FP64, scheme=1, cfl=0.9,
                                                                     chunk=1000, max_it=400000)}
        out["cavity_to_eq40"] = time_to_converge_cavity(igks, mg)
        out["turbulent_plate_to_eq40"] = time_to_converge_turbulent_plate(igks, mg)
    if not args.no_cpu:
        out["cpu_baseline"] = run_cpu_baseline(list(zip(meshes, flows))[:4])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
