"""Benchmark: implicit gas-kinetic scheme iterations on one MI355X.

A step is one full nonlinear iteration (Eq.16 residual with the GKS face
flux, Eq.25 CFL law, LU-SGS forward and backward sweeps, Eq.17 update) over
every cell of the workload mesh; the metric is cell-updates per second
(cells x iterations / wall time), inputs resident in HBM.

Default workload: the 2M-cell SA Joukowski hybrid mesh (2048 wall points,
90 quad layers from 1e-6 chord growing by 1.10, seeded Delaunay triangles out
to 20 chords, colour-ordered), Ma 0.15, Re 6e6, alpha 4 deg, SA with
nu~_inf = 3 nu_inf, FP64; also measured on it: the mixed-precision form, and
beside it the 64-instance batch (mixed), the time to a 1e-10 residual drop
of the laminar plate (FP64, mixed, batched, explicit), the lid-driven
cavity and the turbulent plate to the Eq.40 criterion, and the CPU oracle
on a sample of the same workload.

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
                                                    "seeded Delaunay to r=20 chords, Ma 0.15 Re 6e6 alpha 4, SA nu~/nu = 3"),
    "plate64x32": dict(flow=(0.3, 0.0, 1e4, -1.0), desc="laminar flat plate 64x32 quads, Ma 0.3 Re_L 1e4"),
    "batch64": dict(flow=None, desc="64 seeded instances (default_rng(1000+b)): even b flat plate, odd b Joukowski "
                                    "hybrid, cells log-uniform 5e3-2e5, Ma U[0.1,0.6], alpha U[-4,12] (airfoils), "
                                    "Re log-uniform 1e4-1e7, SA iff Re>1e5; one graph launch per chunk"),
}
# launch schedules (block sizes of prep, flux, gather, sweep; sweep schedule;
# lanes per face) found by igks_autotune on these workloads; block sizes never
# change results
SCHEDULES = {"jouk2m": [256, 64, 64, 256, 1, 1], "batch64": [256, 256, 256, 128, 1, 1],
             "jouk40k": [128, 64, 64, 64, 1, 1]}
# plate variants of the batched time-to-1e-10 comparison: (Ma, Re_L)
DROP_BATCH = [(0.2, 5e3), (0.25, 8e3), (0.3, 1e4), (0.35, 1.5e4), (0.4, 2e4), (0.3, 6e3), (0.2, 1.2e4), (0.4, 1e4)]

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_VALU_PEAK_TFS = 78.6   # MI355X FP64 vector: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
# FP64 operations per face of the face flux, counted with rocprofv3 as FP64
# VALU instructions per wave (2 x FMA + MUL + ADD + TRANS) of a one-lane
# kernel (one face per lane).  Algorithmic: the direct evaluation of the
# scheme's formulas (IEEE divides, library erfc, every moment product
# formed separately), profiles/flops_flux_direct_jouk40k.json; the figure
# for either flux kernel.  Executed: what the current one-lane kernel issues
# (refined reciprocals, moments regrouped by powers of u, series erfc),
# profiles/flops_flux_jouk40k.json.
FLUX_FLOP_PER_FACE = 3498.6
FLUX_EXEC_FLOP_PER_FACE = 2267.6
KSRC = os.path.join(ROOT, "paper_1709_00803_amd", "csrc", "igks_kernels.hip")


def say(*a):
    print("#", *a, file=sys.stderr, flush=True)


def ratio(a, b):
    """a / b, or None when b is 0 (an impulsive start whose mass residual is
    exactly zero)."""
    return a / b if b else None


class Progress:
    """A line on stderr at most every `every` seconds from a long run (the
    runs to a residual drop print nothing else for minutes)."""

    def __init__(self, label, every=20.0):
        self.label, self.every, self.t = label, every, time.perf_counter()

    def __call__(self, it, drop):
        now = time.perf_counter()
        if now - self.t >= self.every:
            self.t = now
            say(f"{self.label}: iteration {it}, drop {drop:.3e}")


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
    # gradients of both sides; writes the 64-byte face record (flux, lam,
    # SA saf, sag, sak; zeros for the SA terms when laminar) and the packed
    # lam (+ SA sak) the sweeps read
    b["flux"] = (3 * i4 + 10 * d) * f + (5 + 8) * d * n + (8 + 1 + s) * d * f
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


def traffic_summary(workload):
    """The committed counter summary (profiles/traffic_<workload>.json), or
    None when it is missing or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d


def measured_traffic(workload, cls):
    """HBM bytes per launch of a kernel class from the counter summary, or
    None."""
    d = traffic_summary(workload)
    return None if d is None else d.get("bytes_per_launch", {}).get(cls)


ITERATION_CLASSES = ("prep", "flux", "flux2", "gather", "reduce", "sweep_fwd", "sweep_top", "sweep_bwd", "update",
                     "commit")


def measured_iteration_bytes(workload):
    """Counted bytes (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of one whole
    iteration: every kernel class of the iteration times its dispatches per
    iteration (dispatches over those of k_prep, one per iteration), or None."""
    d = traffic_summary(workload)
    if d is None or not d.get("dispatches", {}).get("prep"):
        return None
    n = d["dispatches"]["prep"]
    return sum(d["bytes_per_launch"][c] * d["dispatches"][c] / n for c in ITERATION_CLASSES
               if c in d["bytes_per_launch"] and c in d["dispatches"])


def load_meshes(mg, name, cache):
    """The workload's meshes and flow conditions, generated from their seeds
    or, with a cache directory, read back from an earlier generation."""
    path = os.path.join(cache, f"{name}.npz") if cache else None
    if path and os.path.exists(path):
        d = np.load(path, allow_pickle=False)
        n = int(d["n"])
        meshes = [mg.Mesh(xy=d[f"xy{i}"], cell_ptr=d[f"cp{i}"], cell_nodes=d[f"cn{i}"], bface_nodes=d[f"bn{i}"],
                          bface_tag=d[f"bt{i}"], meta={}) for i in range(n)]
        return meshes, [tuple(f) for f in d["flows"]]
    if name == "batch64":
        meshes, flows = mg.batch(64)
    else:
        meshes, flows = [mg.workload(name)], [WORKLOADS[name]["flow"]]
    if path:
        os.makedirs(cache, exist_ok=True)
        arrs = {"n": len(meshes), "flows": np.array(flows, dtype=float)}
        for i, m in enumerate(meshes):
            arrs.update({f"xy{i}": m.xy, f"cp{i}": m.cell_ptr, f"cn{i}": m.cell_nodes, f"bn{i}": m.bface_nodes,
                         f"bt{i}": m.bface_tag})
        np.savez(path + ".tmp.npz", **arrs)
        os.replace(path + ".tmp.npz", path)
    return meshes, flows


def graph_chunk(chunk, steps, warmup):
    """Iterations per captured graph: at most `chunk`, `steps` and (when there
    is a warm-up) `warmup`, and a divisor of `steps`, so that the warm-up
    captures the graph and every timed iteration is a graph replay."""
    c = max(1, min(chunk, steps, warmup if warmup > 0 else steps))
    while steps % c:
        c -= 1
    return c


def time_windows(solver, steps, repeats, batched):
    """`repeats` windows of exactly `steps` iterations, each bracketed by a
    device synchronisation; returns the seconds of each window."""
    import torch
    times = []
    for r in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(solver, steps, batched)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times


def run(solver, k, batched):
    """k iterations; a batch instance frozen by a rejected update is
    reported, not fatal: the others go on."""
    from paper_1709_00803_amd import igks
    try:
        solver.iterate(k)
    except igks.IgksError as e:
        if not batched or e.code != igks.IGKS_ENONPHYS:
            raise
        say(str(e))


def committed(solver, batched, n_inst):
    if batched:
        return [solver.residual(i)["iteration"] for i in range(n_inst)]
    return [solver.residual()["iteration"]]


def measure(igks, meshes, flows, precision, args, schedule, label):
    """Throughput of one context: warm-up, `repeats` timed windows of `steps`
    iterations (median reported), then a profiling pass of direct launches
    timed per kernel class with HIP events on the library's stream."""
    import torch
    batched = len(meshes) > 1
    mixed = precision == igks.IGKS_MIXED
    cfl0 = args.cfl_init if args.cfl_init is not None else (10.0 if batched else 1000.0)
    chunk = graph_chunk(args.chunk, args.steps, args.warmup)
    t = time.perf_counter()
    if batched:
        solver = igks.BatchSolver(meshes, precision=precision, chunk=chunk, cfl_init=cfl0)
        for i, f in enumerate(flows):
            solver.set_freestream(i, *f)
        nfs = solver.nf
    else:
        solver = igks.Solver(meshes[0], precision=precision, chunk=chunk, cfl_init=cfl0)
        solver.set_freestream(*flows[0])
        nfs = [solver.nf]
    torch.cuda.synchronize()
    say(f"{label}: {len(meshes)} instance(s), {solver.total_cells} cells, {solver.total_faces} faces, "
        f"{solver.nlev} wavefronts, set up in {time.perf_counter() - t:.1f}s")
    if args.autotune > 0:
        schedule = solver.autotune(args.autotune).tolist()
    elif schedule is not None:
        solver.set_schedule(schedule)
    schedule = solver.schedule().tolist()
    gc_iters, launches_per_it = solver.graph_chunk()
    run(solver, args.warmup, batched)
    c0 = committed(solver, batched, len(meshes))
    times = time_windows(solver, args.steps, args.repeats, batched)
    c1 = committed(solver, batched, len(meshes))
    # updates committed over all windows (frozen instances do not count)
    updates = sum(m.n_cells * (b - a) for m, a, b in zip(meshes, c0, c1))
    per_window = updates / args.repeats
    med = float(np.median(times))
    value = per_window / med
    say(f"{label}: windows of {args.steps} iterations: {[round(x * 1e3, 3) for x in times]} ms, "
        f"{value:.4g} cell-updates/s")
    if batched:
        drops = [solver.residual(i)["res_drop"] for i in range(len(meshes))]
        frozen = [i for i in range(len(meshes)) if solver.status(i)]
        res_info = dict(res_drop_after_min=min(drops), res_drop_after_median=float(np.median(drops)),
                        res_drop_after_max=max(drops), frozen_instances=frozen)
    else:
        res_info = dict(res_drop_after=solver.residual()["res_drop"])
    # per-kernel durations inside iterations: HIP events on the library's
    # stream around each kernel class, direct launches
    solver.set_profiling(True)
    run(solver, args.profile_iters, batched)
    kt = solver.kernel_times()      # ms per iteration, per kernel class
    solver.set_profiling(False)
    kb = {}
    for m, f, nf in zip(meshes, flows, nfs):
        e = int(np.sum(np.diff(m.cell_ptr)))
        for k, v in kernel_bytes(m.n_cells, nf, e, f[3] >= 0, mixed).items():
            kb[k] = kb.get(k, 0) + v
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
    out = dict(value=value, ms_per_step=1e3 * med / args.steps, window_ms=[round(x * 1e3, 4) for x in times],
               cells=solver.total_cells, faces=solver.total_faces, wavefronts=solver.nlev, schedule=schedule,
               chunk=chunk, graph_replays_per_window=args.steps // gc_iters if gc_iters else 0,
               launches_per_iteration=launches_per_it, cfl_init=cfl0, cell_updates_timed=updates, **res_info)
    return solver, out, kt, kb


def roofline_of(args, solver, kt, kb, out, mixed):
    """The dominant kernel class against its roofline, from its launch
    duration inside the iterations of the profiling pass."""
    faces = solver.total_faces
    schedule = out["schedule"]
    dom = max(kt, key=lambda k: kt[k])
    sweep_wg = schedule[4] == 2
    launches = {"sweep_fwd": 1 if sweep_wg else max(solver.nlev - 1, 1),
                "sweep_bwd": 1 if sweep_wg else max(solver.nlev - 1, 1)}.get(dom, 1)
    launch_ms = kt[dom] / launches
    if dom == "flux":
        achieved = FLUX_FLOP_PER_FACE * faces / (launch_ms * 1e-3) / 1e12
        executed = FLUX_EXEC_FLOP_PER_FACE * faces / (launch_ms * 1e-3) / 1e12
        r = dict(kernel="k_flux2" if schedule[5] == 2 else "k_flux", bound="alu", achieved=achieved,
                 peak=FP64_VALU_PEAK_TFS, unit="TFLOP/s", frac=achieved / FP64_VALU_PEAK_TFS,
                 algorithmic_flop_per_launch=FLUX_FLOP_PER_FACE * faces,
                 executed_fp64_tflops=executed, executed_frac=executed / FP64_VALU_PEAK_TFS,
                 executed_note="FP64 operations the one-lane kernel issues per face (2267.6, rocprofv3 counters) "
                               "over the same launch time: the share of the FP64 vector peak the hardware spends")
        cls = "flux2" if schedule[5] == 2 else "flux"
    else:
        achieved = kb[dom] / launches / (launch_ms * 1e-3) / 1e9
        r = dict(kernel=dom, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=achieved / HBM_PEAK_GBS, algorithmic_bytes_per_launch=kb[dom] / launches)
        cls = dom
    tr = measured_traffic(args.workload, cls)
    r.update(traffic=tr, traffic_unit="HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
             launch_ms=launch_ms, launches_per_step=launches,
             algorithmic_bytes_per_launch_of_its_arrays=kb.get(dom, 0.0) / launches,
             kernel_ms_per_step={k: round(v, 5) for k, v in kt.items()},
             hbm_gbs_per_kernel={k: round(kb[k] / (kt[k] * 1e-3) / 1e9, 1) for k in kb if kt.get(k, 0) > 0})
    total = sum(kb.values())
    it_gbs = total / (out["ms_per_step"] * 1e-3) / 1e9
    r["iteration"] = dict(algorithmic_bytes=total, achieved_gbs=it_gbs, frac_of_hbm_peak=it_gbs / HBM_PEAK_GBS,
                          note="all kernel classes of one iteration: compulsory bytes over the timed ms per step")
    counted = measured_iteration_bytes(args.workload)
    if counted is not None:
        c_gbs = counted / (out["ms_per_step"] * 1e-3) / 1e9
        r["iteration"].update(counted_bytes=counted, counted_gbs=c_gbs, counted_frac_of_hbm_peak=c_gbs / HBM_PEAK_GBS,
                              counted_note="FETCH_SIZE + WRITE_SIZE of every kernel of one iteration (L2 fills and "
                                           "write-backs, some served by the Infinity Cache) over the timed ms per step")
    return r


# sweep blocks (cells, coupled_blocks) of the small time-to-solution workloads:
# the smallest that kept the iteration count (block sizes of 64-1024
# measured on each; a wave sweeps each block, all blocks at once)
SMALL_BLOCKS = 128


def plate_mesh(mg, blocks):
    """The 64x32 plate in natural order (blocks None) or renumbered block by
    block: (mesh, sweep block of each cell or None)."""
    m = mg.flat_plate()
    return (m, None) if blocks is None else mg.block_order(m, blocks, "coupled")


def time_to_drop(igks, mg, precision, target=1e-10, max_it=20000, scheme=0, cfl=10.0, chunk=100,
                 blocks=SMALL_BLOCKS, **opt):
    """Iterations and seconds from the impulsive start to a density-residual
    drop of `target` on the laminar flat plate (64x32) with sweep blocks of
    `blocks` cells (None: natural order, one workgroup per sweep); scheme 1:
    the explicit scheme (Eq.15, local steps at a fixed CFL); opt: further
    solver options (lusgs_op)."""
    import torch
    m, blk = plate_mesh(mg, blocks if scheme == 0 else None)
    s = igks.Solver(m, precision=precision, cfl_init=cfl, chunk=chunk, scheme=scheme, sweep_blocks=blk, **opt)
    s.set_freestream(*WORKLOADS["plate64x32"]["flow"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    prog = Progress(f"plate to {target:g} (scheme {scheme}, precision {precision})")
    l2_first = None
    while it < max_it:
        s.iterate(chunk)
        if l2_first is None:
            l2_first = float(s.history()[0, 0])   # ||M_rho||_2 of the impulsive-start iteration
        it += chunk
        d = s.residual()["res_drop"]
        prog(it, d)
        if d <= target:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    wl = s.wall_loads()
    say(f"plate to {target:g} (scheme {scheme}, precision {precision}, {opt}): {it} iterations, {dt:.1f}s")
    return dict(**opt, iterations=it, seconds=round(dt, 4), drop=s.residual()["res_drop"],
                drop_from_first=ratio(s.residual()["res_l2"], l2_first), cd=wl["cd"],
                cell_updates_per_s=m.n_cells * it / dt, ms_per_iteration=round(1e3 * dt / it, 4),
                schedule=("explicit" if scheme else
                          f"sweep blocks of {blocks} cells" if blocks else "natural order, one workgroup per sweep"))


def run_to_drop(igks, mesh, flow, precision, blocks=None, target=1e-10, max_it=40000, chunk=200, scheme=0,
                cfl=1000.0, max_s=60.0, label="run", **opt):
    """Iterations and seconds from the impulsive start to a density-residual
    drop of `target` (or to max_it iterations / about max_s seconds); opt:
    further solver options (limiter, limiter_freeze)."""
    import torch
    s = igks.Solver(mesh, precision=precision, cfl_init=cfl, chunk=chunk, scheme=scheme, sweep_blocks=blocks,
                    **opt)
    s.set_freestream(*flow)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    marks = {}   # first checked iteration (and seconds) at drops 1e-4, 1e-6, 1e-8 and at Eq.40 <= 3e-8
    prog = Progress(label)
    l2_first = None
    while it < max_it and time.perf_counter() - t0 < max_s:
        s.iterate(chunk)
        if l2_first is None:
            l2_first = float(s.history()[0, 0])   # ||M_rho||_2 of the impulsive-start iteration
        it += chunk
        r = s.residual()
        prog(it, r["res_drop"])
        for key, hit in (("drop_1e-4", r["res_drop"] <= 1e-4), ("drop_1e-6", r["res_drop"] <= 1e-6),
                         ("drop_1e-8", r["res_drop"] <= 1e-8), ("eq40_3e-8", r["eq40"] <= 3e-8)):
            if hit and key not in marks:
                marks[key] = dict(iterations=it, seconds=round(time.perf_counter() - t0, 3))
        if r["res_drop"] <= target:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = s.residual()
    wl = s.wall_loads()
    say(f"{label}: {it} iterations, {dt:.1f}s, drop {r['res_drop']:.3e}")
    return dict(iterations=it, seconds=round(dt, 4), drop=r["res_drop"], reached=r["res_drop"] <= target,
                drop_from_first=ratio(r["res_l2"], l2_first),
                cl=wl["cl"], cd=wl["cd"], ms_per_iteration=round(1e3 * dt / max(it, 1), 4),
                wavefronts=s.nlev, sweep_schedule=int(s.schedule()[4]), milestones=marks)


def time_to_drop_joukowski(igks, mg):
    """The 40k-cell laminar Joukowski (Ma 0.5, Re 5000, alpha 2) from the
    impulsive start to a 1e-10 drop: block LU-SGS (blocks of at most 256
    cells grown along the strongest couplings, generation order inside, a
    wave per block) in FP64 and mixed precision, against the colour order
    (3 wavefronts, fast sweeps that do not converge) and the explicit
    scheme."""
    flow = WORKLOADS["jouk40k"]["flow"]
    mb, blk = mg.workload_blocks("jouk40k", 256)
    mc = mg.workload("jouk40k")
    out = dict(workload="jouk40k: " + WORKLOADS["jouk40k"]["desc"], target=1e-10, blocks=int(blk.max()) + 1,
               block_cells=256)
    out["blocks_fp64"] = run_to_drop(igks, mb, flow, igks.IGKS_FP64, blk, max_it=60000, label="jouk40k blocks fp64")
    out["blocks_mixed"] = run_to_drop(igks, mb, flow, igks.IGKS_MIXED, blk, max_it=60000, label="jouk40k blocks mixed")
    out["colour_fp64"] = run_to_drop(igks, mc, flow, igks.IGKS_FP64, None, max_it=10000, max_s=15.0,
                                     label="jouk40k colour fp64")
    out["explicit_fp64_cfl0.9"] = run_to_drop(igks, mc, flow, igks.IGKS_FP64, None, max_it=2000000, chunk=2000,
                                             scheme=1, cfl=0.9, max_s=40.0, label="jouk40k explicit")
    return out


def roe_time_to_solution(igks, mg):
    """The small cases again with the Roe-matrix LU-SGS operator
    (lusgs_op = 1): the plate to a 1e-10 drop (sweep blocks and natural
    order), the cavity (both) and the turbulent plate to Eq.40 <= 3e-8, the 40k
    Joukowski to 1e-10 (blocks of 256).  The last two do not converge with
    it (the iteration stalls and the Eq.25 law holds the CFL number low;
    the 40k Joukowski's impulsive start at CFL 1000 gives a non-physical
    update)."""
    flow = WORKLOADS["jouk40k"]["flow"]
    mb, blk = mg.workload_blocks("jouk40k", 256)
    return {"operator": "Roe matrix |A| = R|Lambda|L at the Roe average, |lambda| >= 0.1 c, 4x4 diagonal blocks",
            "plate_fp64": time_to_drop(igks, mg, igks.IGKS_FP64, lusgs_op=1),
            "plate_fp64_natural_order": time_to_drop(igks, mg, igks.IGKS_FP64, blocks=None, lusgs_op=1),
            "batched_plates": time_to_drop_batch(igks, mg, lusgs_op=1),
            "cavity_to_eq40": time_to_converge_cavity(igks, mg, label="cavity roe", lusgs_op=1),
            "cavity_to_eq40_natural_order": time_to_converge_cavity(igks, mg, label="cavity roe natural order",
                                                                    blocks=None, lusgs_op=1),
            "turbulent_plate_to_eq40": time_to_converge_turbulent_plate(igks, mg, label="turbulent plate roe",
                                                                        lusgs_op=1),
            "kinetic_plate_fp64": time_to_drop(igks, mg, igks.IGKS_FP64, lusgs_op=2),
            "kinetic_turbulent_plate_to_eq40": time_to_converge_turbulent_plate(
                igks, mg, label="turbulent plate roe kinetic", lusgs_op=2),
            "jouk40k_blocks_fp64": guarded(run_to_drop, igks, mb, flow, igks.IGKS_FP64, blk, max_it=60000,
                                           label="jouk40k blocks fp64 roe", lusgs_op=1)}


def guarded(fn, igks, *a, **kw):
    """fn's result, or the solver's error where it rejected a non-physical
    update (the instance is frozen and the run ends there)."""
    try:
        return fn(igks, *a, **kw)
    except igks.IgksError as e:
        say(f"{kw.get('label', fn.__name__)}: {e}")
        return dict(error=str(e))


def time_to_drop_sa250k(igks, mg, max_s=40.0):
    """The 250k-cell SA Joukowski (Ma 0.15, Re 6e6, alpha 4) from the free
    stream at CFL 10 with block LU-SGS in two passes (the second with the
    first's cross-block terms) and the Eq.9 limiter held from a drop of
    1e-4, FP64 and mixed, for about max_s seconds each: the milestones on
    the way (drops 1e-4, 1e-6, 1e-8, Eq.40 <= 3e-8) and the drop reached."""
    flow = WORKLOADS["jouk250k"]["flow"]
    mb, blk = mg.workload_blocks("jouk250k", 512)
    out = dict(workload="jouk250k: " + WORKLOADS["jouk250k"]["desc"], target=1e-10, blocks=int(blk.max()) + 1,
               block_cells=512, block_passes=2, limiter="Eq.9, held from a drop of 1e-4",
               note="two block passes reach 5e-7 in 40 000 iterations and 1.5e-9 in 200 000 (200 s), below 1e-8 "
                    "the rate slows; without the limiter the wake behind the trailing edge holds a limit cycle "
                    "near 4e-2; one block pass levels off near 3e-3")
    for key, prec in (("blocks_fp64", igks.IGKS_FP64), ("blocks_mixed", igks.IGKS_MIXED)):
        out[key] = run_to_drop(igks, mb, flow, prec, blk, max_it=10 ** 6, chunk=500, cfl=10.0, max_s=max_s,
                               limiter=1, limiter_freeze=1e-4, block_passes=2, label=f"jouk250k {key}")
    return out


def batch_to_drop(igks, mg, target=1e-10, max_s=60.0, chunk=500):
    """batch64 in generation order with coupled sweep blocks (512 cells) in
    two block passes, mixed precision, the Eq.9 limiter held from a drop of
    1e-4, from the free stream at CFL 10, for about max_s seconds: per instance the first
    checked iteration at a `target` drop (None if not reached) and the final
    drop; the instances that reached it are then run alone in FP64 to the
    same target, one after another, for the wall-time comparison."""
    import torch
    items = [mg.batch_instance(b, order="natural") for b in range(64)]
    meshes, blocks = [], []
    for m, _ in items:
        mb, bk = mg.block_order(m, 512, "coupled")
        meshes.append(mb)
        blocks.append(bk)
    opt = dict(cfl_init=10.0, limiter=1, limiter_freeze=1e-4, block_passes=2)
    s = igks.BatchSolver(meshes, chunk=100, sweep_blocks=blocks, precision=igks.IGKS_MIXED, **opt)
    for i, (_, f) in enumerate(items):
        s.set_freestream(i, *f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, first, t_first = 0, [None] * 64, [None] * 64
    prog = Progress("batch64 blocks")
    l2_first = None
    while time.perf_counter() - t0 < max_s and any(x is None for x in first):
        try:
            s.iterate(chunk)
        except igks.IgksError:
            pass   # an instance frozen by a rejected update; the others go on
        if l2_first is None:
            hs = [s.history(i) for i in range(64)]
            l2_first = [float(h[0, 0]) if len(h) else 0.0 for h in hs]
        it += chunk
        for i in range(64):
            if first[i] is None and s.residual(i)["res_drop"] <= target:
                first[i], t_first[i] = it, round(time.perf_counter() - t0, 3)
        prog(it, float(np.median([s.residual(i)["res_drop"] for i in range(64)])))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    drops = [s.residual(i)["res_drop"] for i in range(64)]
    drops_first = [ratio(s.residual(i)["res_l2"], l2_first[i]) for i in range(64)]
    frozen = [i for i in range(64) if s.status(i)]
    nlev = s.nlev
    del s
    seq = {}
    for i in [i for i in range(64) if first[i] is not None]:
        seq[i] = run_to_drop(igks, meshes[i], items[i][1], igks.IGKS_FP64, blocks[i], target=target,
                             max_it=10 * first[i], chunk=100, cfl=10.0, max_s=30.0, limiter=1, limiter_freeze=1e-4,
                             block_passes=2, label=f"batch64 instance {i} alone")
    return dict(workload="batch64 in generation order, coupled sweep blocks of at most 512 cells, two block "
                         "passes, mixed, limiter held from 1e-4, CFL 10 -> Eq.25",
                target=target, iterations=it, seconds=round(t_batch, 3), ms_per_iteration=round(1e3 * t_batch / it, 3),
                wavefronts=nlev, reached=sum(x is not None for x in first), first_iteration_at_target=first,
                batch_seconds_at_target=t_first, final_drop=[float(f"{d:.3e}") for d in drops],
                final_drop_from_first=[None if d is None else float(f"{d:.3e}") for d in drops_first], frozen=frozen,
                fp64_alone={str(i): v for i, v in seq.items()},
                fp64_alone_seconds_total=round(sum(v["seconds"] for v in seq.values()), 4))


def time_to_converge_cavity(igks, mg, max_it=30000, chunk=200, label="cavity", blocks=SMALL_BLOCKS, **opt):
    """The lid-driven cavity (100x100, Re 1000, Ma 0.1 sqrt 3, isothermal
    walls) from rest, implicit CFL 1000 growing by Eq.25, sweep blocks of
    `blocks` cells (None: natural order), to the paper's criterion Eq.40 <=
    3e-8; opt: further solver options (lusgs_op)."""
    import torch
    m, blk = mg.cavity(100), None
    if blocks:
        m, blk = mg.block_order(m, blocks, "coupled")
    s = igks.Solver(m, cfl_init=1000.0, chunk=chunk, wall_temp=1.0, sweep_blocks=blk, **opt)
    s.set_freestream(0.1 * math.sqrt(3.0), 0.0, 1000.0)
    W = s.get_state()
    W[3] -= 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0]
    W[1] = W[2] = 0.0
    s.set_state(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    prog = Progress(f"{label} to Eq.40")
    while it < max_it:
        s.iterate(chunk)
        it += chunk
        r = s.residual()
        prog(it, r["res_drop"])
        if r["eq40"] <= 3e-8:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = s.residual()
    say(f"{label}: {it} iterations, {dt:.1f}s")
    return dict(**opt, workload="cavity100: 100x100 uniform, Re 1000, Ma 0.1 sqrt(3), isothermal walls, from rest",
                schedule=f"sweep blocks of {blocks} cells" if blocks else "natural order, one workgroup per sweep",
                criterion="Eq.40 <= 3e-8", iterations=it, seconds=round(dt, 4), eq40=r["eq40"],
                drop=r["res_drop"], cfl=r["cfl"], ms_per_iteration=round(1e3 * dt / it, 4),
                paper_iterations=4430, paper_seconds=543.2)


def time_to_converge_turbulent_plate(igks, mg, max_it=30000, chunk=500, label="turbulent plate",
                                     blocks=SMALL_BLOCKS, **opt):
    """The turbulent flat plate (SA, Ma 0.2, Re 5e6 per unit length, 7680
    cells, sweep blocks of `blocks` cells, None: natural order) from the free
    stream at CFL 10 growing by Eq.25, to the paper's criterion Eq.40 <=
    3e-8; opt: further solver options (lusgs_op)."""
    import torch
    m, blk = mg.turbulent_plate(), None
    if blocks:
        m, blk = mg.block_order(m, blocks, "coupled")
    s = igks.Solver(m, cfl_init=10.0, chunk=chunk, sweep_blocks=blk, **opt)
    s.set_freestream(0.2, 0.0, 5e6, 3.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    prog = Progress(f"{label} to Eq.40")
    while it < max_it:
        s.iterate(chunk)
        it += chunk
        r = s.residual()
        prog(it, r["res_drop"])
        if r["eq40"] <= 3e-8:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = s.residual()
    say(f"{label}: {it} iterations, {dt:.1f}s")
    return dict(**opt, workload="turbulent flat plate: 120x64 quads, y+ ~ 1, Ma 0.2, Re 5e6/unit length, SA, from the free stream",
                schedule=f"sweep blocks of {blocks} cells" if blocks else "natural order, one workgroup per sweep",
                criterion="Eq.40 <= 3e-8", iterations=it, seconds=round(dt, 4), eq40=r["eq40"],
                drop=r["res_drop"], cd=s.wall_loads()["cd"], ms_per_iteration=round(1e3 * dt / it, 4),
                paper_iterations=5340, paper_seconds=1087.7)


def time_to_drop_batch(igks, mg, target=1e-10, max_it=20000, blocks=SMALL_BLOCKS, **opt):
    """Eight plate flow conditions (DROP_BATCH) to a `target` drop with sweep
    blocks of `blocks` cells: one mixed-precision batch against the eight
    FP64 single runs one after another; opt: further solver options
    (lusgs_op), the same for both."""
    import torch
    m, blk = plate_mesh(mg, blocks)
    flows = [(ma, 0.0, re, -1.0) for ma, re in DROP_BATCH]
    b = igks.BatchSolver([m] * len(flows), precision=igks.IGKS_MIXED, cfl_init=10.0, chunk=100,
                         sweep_blocks=None if blk is None else [blk] * len(flows), **opt)
    for i, f in enumerate(flows):
        b.set_freestream(i, *f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, first = 0, [None] * len(flows)
    prog = Progress("batched plates")
    while it < max_it and any(x is None for x in first):
        b.iterate(100)
        it += 100
        prog(it, max(b.residual(i)["res_drop"] for i in range(len(flows))))
        for i in range(len(flows)):
            if first[i] is None and b.residual(i)["res_drop"] <= target:
                first[i] = it
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t_seq, its_seq = 0.0, []
    for f in flows:
        s = igks.Solver(m, precision=igks.IGKS_FP64, cfl_init=10.0, chunk=100, sweep_blocks=blk, **opt)
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
        say(f"plate {f[:3]} alone: {k} iterations")
    return dict(**opt, instances=len(flows), flows_ma_re=DROP_BATCH, sweep_blocks=blocks, batch_mixed_seconds=round(t_batch, 4),
                batch_iterations_to_target=first, fp64_sequential_seconds=round(t_seq, 4),
                fp64_iterations_to_target=its_seq, speedup=round(t_seq / t_batch, 3))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_threads():
    """Host cores this process may use, at most 16 (the CPU share of one GPU
    on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run_cpu_baseline(mesh, flow, name, budget_s=25.0):
    """The oracle on a bounded sample of the workload: the mesh ingest and the
    impulsive-start iteration untimed (on all threads), then iterations on
    one thread and on all host threads (the oracle's per-cell and per-face
    loops; its sweeps stay sequential; results are bitwise the same).  About
    budget_s of CPU work."""
    from oracle import pyoracle as po
    nt = host_threads()
    t = time.perf_counter()
    o = po.Oracle(mesh, threads=nt)
    o.set_freestream(*flow)
    o.iterate(1)
    setup = time.perf_counter() - t
    res = {}
    for threads, share in ((1, 0.6), (nt, 0.4)):
        o.set_threads(threads)
        t0 = time.perf_counter()
        it = 0
        while True:
            o.iterate(1)
            it += 1
            if time.perf_counter() - t0 > share * budget_s:
                break
        dt = time.perf_counter() - t0
        res[threads] = (mesh.n_cells * it / dt, it, dt)
        say(f"cpu oracle, {threads} thread(s): {it} iterations in {dt:.1f}s")
    v1, i1, d1 = res[1]
    vn, i_n, dn = res[nt]
    return dict(value=vn, unit="cell-updates/s", cores=nt, kind="oracle", cpu_model=cpu_model(),
                single_thread=dict(value=v1, cores=1, iterations=i1, seconds=round(d1, 2)),
                sample=f"{name} ({mesh.n_cells} cells): after the untimed mesh ingest and impulsive-start iteration "
                       f"({setup:.1f}s on {nt} threads), {i_n} iteration(s) on {nt} threads in {dn:.1f}s (value) and "
                       f"{i1} on one thread in {d1:.1f}s; FP64 C oracle, OpenMP over its cell and face loops, "
                       f"sequential sweeps, results independent of the thread count")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="iterations per timed window")
    ap.add_argument("--warmup", type=int, default=10, help="untimed iterations before the timed windows")
    ap.add_argument("--repeats", type=int, default=5, help="timed windows of --steps iterations (median reported)")
    ap.add_argument("--workload", default="jouk2m", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64, mixed for batch64")
    ap.add_argument("--chunk", type=int, default=20,
                    help="largest number of iterations per captured HIP graph; cut to divide --steps and to "
                         "at most --warmup, so the timed iterations replay a graph the warm-up captured")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--autotune", type=int, default=0,
                    help="autotuner iterations per candidate (0: the stored schedule of the workload)")
    ap.add_argument("--cfl-init", type=float, default=None, help="initial implicit CFL (default: 1000, 10 for batch64)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-drop", action="store_true", help="skip the time-to-1e-10 and Eq.40 runs")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-precision and batch64 extra measurements")
    ap.add_argument("--sa250k-only", type=float, default=None, metavar="SECONDS",
                    help="run only the 250k SA Joukowski from the free stream toward a 1e-10 drop (--precision, "
                         "default fp64; two-pass coupled blocks of 512 cells, limiter held from 1e-4) for at most "
                         "SECONDS and print its JSON (the full default run gives it 40 s per precision)")
    ap.add_argument("--lusgs-op", type=int, default=0, choices=[0, 1],
                    help="LU-SGS operator of the --sa250k-only run: 0 the scalar spectral radius, 1 the Roe matrix")
    ap.add_argument("--roe-only", action="store_true",
                    help="run only the time-to-solution cases with the Roe-matrix LU-SGS operator and print their JSON")
    ap.add_argument("--mesh-cache", default=None,
                    help="directory where generated meshes are stored and read back (the seeded generation "
                         "of the 2M-cell mesh takes about a minute)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the batched and single-mesh paths are single-GPU).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.repeats < 1 or args.warmup < 0:
        print("bench.py: --steps and --repeats must be >= 1, --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_00803_amd import igks
    from paper_1709_00803_amd import meshgen as mg

    torch.cuda.set_device(0)
    if args.sa250k_only is not None:
        flow = WORKLOADS["jouk250k"]["flow"]
        mb, blk = mg.workload_blocks("jouk250k", 512)
        prec = args.precision or "fp64"
        r = run_to_drop(igks, mb, flow, igks.IGKS_MIXED if prec == "mixed" else igks.IGKS_FP64, blk,
                        max_it=10 ** 7, chunk=1000, cfl=10.0, max_s=args.sa250k_only, limiter=1, limiter_freeze=1e-4,
                        block_passes=2, lusgs_op=args.lusgs_op, label=f"jouk250k to 1e-10 ({prec})")
        print(json.dumps(dict(workload="jouk250k: " + WORKLOADS["jouk250k"]["desc"], precision=prec,
                              lusgs_op=args.lusgs_op,
                              schedule="coupled sweep blocks of 512 cells, two passes, Eq.9 limiter held from a "
                                       "drop of 1e-4, CFL 10 -> Eq.25", target=1e-10, **r)), flush=True)
        return
    if args.roe_only:
        print(json.dumps(roe_time_to_solution(igks, mg)), flush=True)
        return
    wl = WORKLOADS[args.workload]
    batched = args.workload == "batch64"
    precision = args.precision or ("mixed" if batched else "fp64")
    mixed = precision == "mixed"
    t = time.perf_counter()
    meshes, flows = load_meshes(mg, args.workload, args.mesh_cache)
    say(f"{args.workload}: meshes ready in {time.perf_counter() - t:.1f}s")
    prec = igks.IGKS_MIXED if mixed else igks.IGKS_FP64
    sched = SCHEDULES.get(args.workload)
    solver, main_out, kt, kb = measure(igks, meshes, flows, prec, args, sched, args.workload)
    roofline = roofline_of(args, solver, kt, kb, main_out, mixed)
    del solver
    torch.cuda.empty_cache()

    out = {
        "metric": "cell-updates/s", "value": main_out["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_out["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": dict({"workload": f"{args.workload}: {wl['desc']}", "instances": len(meshes), "precision": precision,
                        "ordering": "colour", "repeats": args.repeats, "value_from": "median window"},
                       **{k: v for k, v in main_out.items() if k not in ("value", "ms_per_step")}),
        "roofline": roofline,
    }
    if not args.no_extra:
        if not batched and not mixed:
            _, mo, mkt, _ = measure(igks, meshes, flows, igks.IGKS_MIXED, args, sched, args.workload + " mixed")
            out["mixed"] = dict(mo, dtype="f32+f64", kernel_ms_per_step={k: round(v, 5) for k, v in mkt.items()})
            torch.cuda.empty_cache()
        if not batched:
            bm, bf = load_meshes(mg, "batch64", args.mesh_cache)
            _, bo, bkt, _ = measure(igks, bm, bf, igks.IGKS_MIXED, args, SCHEDULES["batch64"], "batch64 mixed")
            out["batch64_mixed"] = dict(bo, dtype="f32+f64", workload=WORKLOADS["batch64"]["desc"],
                                        kernel_ms_per_step={k: round(v, 5) for k, v in bkt.items()})
            counted = measured_iteration_bytes("batch64")
            if counted is not None:
                gbs = counted / (bo["ms_per_step"] * 1e-3) / 1e9
                out["batch64_mixed"].update(counted_bytes_per_iteration=counted, counted_gbs=gbs,
                                            counted_frac_of_hbm_peak=gbs / HBM_PEAK_GBS,
                                            flux_traffic_per_launch=measured_traffic("batch64", "flux2"))
            del bm
            torch.cuda.empty_cache()
    if not args.no_drop:
        out["time_to_1e-10"] = {"workload": f"plate64x32, Ma 0.3 Re_L 1e4, CFL 10 -> Eq.25, sweep blocks of "
                                            f"{SMALL_BLOCKS} cells (coupled_blocks, generation order inside)",
                                "fp64": time_to_drop(igks, mg, igks.IGKS_FP64),
                                "mixed": time_to_drop(igks, mg, igks.IGKS_MIXED),
                                "fp64_natural_order": time_to_drop(igks, mg, igks.IGKS_FP64, blocks=None),
                                "fp64_roe_operator": time_to_drop(igks, mg, igks.IGKS_FP64, lusgs_op=1),
                                "batched_plates": time_to_drop_batch(igks, mg),
                                "explicit_fp64_cfl0.9": time_to_drop(igks, mg, igks.IGKS_FP64, scheme=1, cfl=0.9,
                                                                     chunk=1000, max_it=400000)}
        out["time_to_1e-10"]["jouk40k"] = time_to_drop_joukowski(igks, mg)
        out["time_to_1e-10"]["jouk250k"] = time_to_drop_sa250k(igks, mg)
        out["time_to_1e-10"]["batch64"] = batch_to_drop(igks, mg)
        say("time to 1e-10 done")
        out["cavity_to_eq40"] = time_to_converge_cavity(igks, mg)
        out["turbulent_plate_to_eq40"] = time_to_converge_turbulent_plate(igks, mg)
        say("Eq.40 runs done")
    if not args.no_cpu:
        if batched:
            out["cpu_baseline"] = run_cpu_baseline(meshes[1], flows[1], "batch64 instance 1")
        else:
            out["cpu_baseline"] = run_cpu_baseline(meshes[0], flows[0], args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
