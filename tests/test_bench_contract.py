"""bench.py on the CPU: the one-GPU guard and the algorithmic byte model
(no GPU is touched: the guard exits before anything is imported)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_bytes_model():
    n, f, e = 1000, 1550, 3100
    lam = bench.kernel_bytes(n, f, e, False, False)
    sa = bench.kernel_bytes(n, f, e, True, False)
    mixed = bench.kernel_bytes(n, f, e, False, True)
    assert set(lam) == {"prep", "flux", "gather", "reduce", "sweep_fwd", "sweep_bwd"}
    assert all(v > 0 for v in lam.values())
    # the backward step also reads its own increment and writes the new state
    assert lam["sweep_bwd"] > lam["sweep_fwd"]
    # SA adds face and cell terms to the flux, gather and sweeps; FP32 increments shrink the sweeps only
    for k in ("flux", "gather", "sweep_fwd", "sweep_bwd"):
        assert sa[k] > lam[k]
    for k in ("sweep_fwd", "sweep_bwd"):
        assert mixed[k] < lam[k]
    for k in ("prep", "flux", "gather", "reduce"):
        assert mixed[k] == lam[k]
    # linear in the sizes
    dbl = bench.kernel_bytes(2 * n, 2 * f, 2 * e, False, False)
    for k in lam:
        assert dbl[k] == 2 * lam[k]


@pytest.mark.parametrize("chunk,steps,warmup,want", [(20, 20, 5, 5), (100, 20, 10, 10), (20, 7, 10, 7),
                                                     (20, 20, 0, 20), (6, 20, 10, 5), (20, 20, 20, 20)])
def test_graph_chunk_divides_the_timed_steps(chunk, steps, warmup, want):
    """The timed iterations are whole graph replays of a graph the warm-up
    captured: the chunk divides --steps and is at most --warmup."""
    c = bench.graph_chunk(chunk, steps, warmup)
    assert c == want
    assert steps % c == 0 and c <= chunk and (warmup == 0 or c <= warmup)


def test_mesh_cache_round_trip(tmp_path):
    from paper_1709_00803_amd import meshgen as mg
    m1, f1 = bench.load_meshes(mg, "plate64x32", str(tmp_path))
    m2, f2 = bench.load_meshes(mg, "plate64x32", str(tmp_path))
    assert f1 == f2
    for a, b in zip(m1, m2):
        for k in ("xy", "cell_ptr", "cell_nodes", "bface_nodes", "bface_tag"):
            assert np.array_equal(getattr(a, k), getattr(b, k))
