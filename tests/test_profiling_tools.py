"""The rocprofv3 summarisers behind profiles/ (paper_1709_00803_amd.profiling),
on synthetic counter and kernel-stats tables (CPU only)."""
import csv
import json

import pytest

from paper_1709_00803_amd import profiling as pf


def write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow(dict(Kernel_Name=k, Counter_Name=c, Counter_Value=v))


@pytest.mark.parametrize("name,cls", [
    ("void igks::k_flux2<double, true>(igks::Params<double>)", "flux2"),
    ("void igks::k_flux<float, false>(igks::Params<float>)", "flux"),
    ("void igks::k_sweep<double, 0, true>(igks::Params<double>, int, int, int)", "sweep_fwd"),
    ("void igks::k_sweep<double, 2, false>(igks::Params<double>, int, int, int)", "sweep_top"),
    ("void igks::k_sweep<float, 1, true>(igks::Params<float>, int, int, int)", "sweep_bwd"),
    ("void igks::k_sweep_wg<double, true, true>(igks::Params<double>, int const*, int)", "sweep_fwd"),
    ("void igks::k_sweep_wg<float, false, false>(igks::Params<float>, int const*, int)", "sweep_bwd"),
    ("void igks::k_reduce<double>(igks::Params<double>, int)", "reduce"),
    ("void igks::k_commit<double>(igks::Params<double>, int)", "commit"),
    ("__amd_rocclr_copyBuffer", None),
])
def test_kernel_class(name, cls):
    assert pf.kernel_class(name) == cls


def test_traffic_scales_by_the_copy(tmp_path):
    flux = "void igks::k_flux<double, true>(igks::Params<double>)"
    gat = "void igks::k_gather<double, true>(igks::Params<double>)"
    copy = "__amd_rocclr_copyBuffer"
    write_counters(tmp_path / "f.csv", [(flux, "FETCH_SIZE", 100.0), (flux, "FETCH_SIZE", 140.0),
                                        (gat, "FETCH_SIZE", 50.0)])
    write_counters(tmp_path / "w.csv", [(flux, "WRITE_SIZE", 30.0), (flux, "WRITE_SIZE", 34.0),
                                        (gat, "WRITE_SIZE", 8.0)])
    nbytes = 1024.0 * 1024.0
    # the counters see half of the copied bytes on the read side and all of them on the write side
    write_counters(tmp_path / "fc.csv", [(copy, "FETCH_SIZE", nbytes / 1024.0 / 2)])
    write_counters(tmp_path / "wc.csv", [(copy, "WRITE_SIZE", nbytes / 1024.0)])
    out = pf.traffic("w", tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "fc.csv", tmp_path / "wc.csv",
                     nbytes, tmp_path / "t.json", "cmd")
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    assert out["dispatches"]["flux"] == 2
    assert out["bytes_per_launch"]["flux"] == pytest.approx((120.0 * 2.0 + 32.0) * 1024.0)
    assert out["bytes_per_launch"]["gather"] == pytest.approx((50.0 * 2.0 + 8.0) * 1024.0)
    assert json.load(open(tmp_path / "t.json"))["kernel_source_sha256_16"] == pf.kernel_source_hash()


def test_flops_counts_fma_twice(tmp_path):
    flux = "void igks::k_flux<double, true>(igks::Params<double>)"
    rows = [(flux, "SQ_INSTS_VALU_ADD_F64", 10.0), (flux, "SQ_INSTS_VALU_MUL_F64", 20.0),
            (flux, "SQ_INSTS_VALU_FMA_F64", 30.0), (flux, "SQ_INSTS_VALU_TRANS_F64", 5.0),
            (flux, "SQ_WAVES", 2.0)]
    write_counters(tmp_path / "c.csv", rows)
    out = pf.flops("w", tmp_path / "c.csv", 128, tmp_path / "o.json", "cmd")
    assert out["fp64_ops_per_face"] == pytest.approx((10 + 20 + 2 * 30 + 5) / 2.0)
    assert out["faces_per_wave"] == pytest.approx(64.0)


def test_stats_table(tmp_path):
    with open(tmp_path / "s.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writeheader()
        w.writerow(dict(Name="void igks::k_flux<double, true>(igks::Params<double>)", Calls=3, AverageNs=12500.0,
                        MinNs=12000.0, MaxNs=13000.0, Percentage=50.0))
    pf.stats(tmp_path / "s.csv", tmp_path / "s.txt", "rocprofv3 --kernel-trace --stats -- python3 bench.py")
    txt = open(tmp_path / "s.txt").read().splitlines()
    assert txt[1].endswith("python3 bench.py") and pf.kernel_source_hash() in txt[2]
    row = txt[4].split()
    assert row[-5:] == ["3", "12.50", "12.00", "13.00", "50.00"]
