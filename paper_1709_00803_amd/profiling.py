"""Summaries of rocprofv3 output (kernel-trace stats and --pmc counter
collections) into the short text / JSON files kept under profiles/.

    python -m paper_1709_00803_amd.profiling stats  <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_1709_00803_amd.profiling traffic <workload> <fetch.csv> <write.csv> \
        <fetch_copy.csv> <write_copy.csv> <copy_bytes> <out.json> "<command>"
    python -m paper_1709_00803_amd.profiling copy     (calibration: 5 device copies of 256 MiB)
    python -m paper_1709_00803_amd.profiling flops <workload> <counters.csv> <faces> <out.json> "<command>"
"""
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KSRC = os.path.join(HERE, "csrc", "igks_kernels.hip")


def kernel_class(name: str):
    """Kernel class of a (demangled) kernel name, as bench.py reports them."""
    table = [("k_prep", "prep"), ("k_flux2", "flux2"), ("k_flux", "flux"), ("k_gather", "gather"),
             ("k_reduce", "reduce"), ("k_commit", "commit"),
             ("k_sweep_wg<double, true", "sweep_fwd"), ("k_sweep_wg<double, false", "sweep_bwd"),
             ("k_sweep_wg<float, true", "sweep_fwd"), ("k_sweep_wg<float, false", "sweep_bwd"),
             ("k_sweep<double, 0,", "sweep_fwd"), ("k_sweep<double, 2,", "sweep_top"),
             ("k_sweep<double, 1,", "sweep_bwd"), ("k_sweep<float, 0,", "sweep_fwd"),
             ("k_sweep<float, 2,", "sweep_top"), ("k_sweep<float, 1,", "sweep_bwd"), ("k_update", "update"),
             ("k_explicit", "update"), ("k_reset", "reset")]
    for key, cls in table:
        if key in name:
            return cls
    return None


def kernel_source_hash():
    return hashlib.sha256(open(KSRC, "rb").read()).hexdigest()[:16]


def stats(csv_path, out_txt, command):
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 kernel stats", f"# command: {command}",
             f"# kernel source sha256[:16]: {kernel_source_hash()}",
             f"{'kernel':<58} {'calls':>7} {'avg_us':>10} {'min_us':>9} {'max_us':>9} {'pct':>6}"]
    for r in rows:
        nm = r["Name"].replace("igks::", "")[:58]
        lines.append(f"{nm:<58} {int(r['Calls']):>7} {float(r['AverageNs']) / 1e3:>10.2f} "
                     f"{float(r['MinNs']) / 1e3:>9.2f} {float(r['MaxNs']) / 1e3:>9.2f} {float(r['Percentage']):>6.2f}")
    open(out_txt, "w").write("\n".join(lines) + "\n")
    return out_txt


def _per_class(path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        cls = kernel_class(r["Kernel_Name"]) or r["Kernel_Name"][:40]
        agg[cls].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()}


def traffic(workload, fetch_csv, write_csv, fetch_copy_csv, write_copy_csv, copy_bytes, out_json, command):
    """HBM bytes per dispatch of each kernel class: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) scaled so that a plain device copy of
    copy_bytes reads and writes copy_bytes."""
    f, nf = _per_class(fetch_csv, "FETCH_SIZE")
    w, _ = _per_class(write_csv, "WRITE_SIZE")
    fc, _ = _per_class(fetch_copy_csv, "FETCH_SIZE")
    wc, _ = _per_class(write_copy_csv, "WRITE_SIZE")
    copy_f = max(fc.values())
    copy_w = max(wc.values())
    sf = copy_bytes / (copy_f * 1024.0)
    sw = copy_bytes / (copy_w * 1024.0)
    out = dict(workload=workload, command=command, kernel_source_sha256_16=kernel_source_hash(),
               copy_bytes=copy_bytes, copy_fetch_kib=copy_f, copy_write_kib=copy_w,
               fetch_scale=sf, write_scale=sw, dispatches=nf,
               fetch_kib_per_dispatch=f, write_kib_per_dispatch=w,
               bytes_per_launch={k: f[k] * 1024.0 * sf + w.get(k, 0.0) * 1024.0 * sw for k in f})
    json.dump(out, open(out_json, "w"), indent=1, sort_keys=True)
    return out


F64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                "SQ_INSTS_VALU_TRANS_F64", "SQ_WAVES")


def flops(workload, csv_path, faces, out_json, command, kernel="flux"):
    """FP64 operations per face of the face-flux kernel: each FP64 VALU
    instruction of a wave does one operation per lane and a lane handles one
    face, so ops per face = (2 FMA + MUL + ADD + TRANS) per wave (all waves
    full but the last)."""
    per = {}
    for c in F64_COUNTERS:
        v, _ = _per_class(csv_path, c)
        per[c] = v.get(kernel)
    waves = per["SQ_WAVES"]
    ops = 2 * per["SQ_INSTS_VALU_FMA_F64"] + per["SQ_INSTS_VALU_MUL_F64"] + per["SQ_INSTS_VALU_ADD_F64"] \
        + per["SQ_INSTS_VALU_TRANS_F64"]
    out = dict(workload=workload, command=command, kernel_source_sha256_16=kernel_source_hash(), kernel=kernel,
               counters_per_dispatch=per, faces=faces, faces_per_wave=faces / waves,
               fp64_ops_per_wave=ops / waves, fp64_ops_per_face=ops / waves)
    json.dump(out, open(out_json, "w"), indent=1, sort_keys=True)
    return out


COPY_BYTES = 256 * 1024 * 1024


def copy_calibration(reps=5):
    """Device-to-device copies of COPY_BYTES: the kernel whose FETCH_SIZE and
    WRITE_SIZE counters give the scale from counter KiB to HBM bytes."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy calibration: {reps} copies of {COPY_BYTES // 1024} KiB", flush=True)


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "copy":
        copy_calibration()
    elif a and a[0] == "flops":
        print(json.dumps(flops(a[1], a[2], int(a[3]), a[4], a[5]), indent=1))
    elif a and a[0] == "stats":
        print(stats(a[1], a[2], a[3]))
    elif a and a[0] == "traffic":
        print(json.dumps(traffic(a[1], a[2], a[3], a[4], a[5], float(a[6]), a[7], a[8]), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
