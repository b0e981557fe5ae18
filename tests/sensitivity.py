"""How far the oracle's own residual moves when the mesh geometry moves by
rounding: the scale against which two independent FP64 codes (the GPU
library and the oracle compute the geometry and the flux with different
formulas) can be compared cell by cell.

Every node coordinate is moved by one unit in the last place, with a seeded
random sign, and the oracle evaluates the residual of the same cell state on
the moved mesh.  Per cell, the largest change over the four flow components
relative to the cell's gross flux sum_faces |F S| (and for the SA
right-hand side relative to its own gross size) is the cell's measured
sensitivity.  In exact arithmetic the change is zero for the free stream; in
thin high-aspect-ratio cells the wall-normal differences (W0 - W_c) / d of
Eq.5 lose about log10(aspect ratio) digits, and at a cusp the coordinates'
rounding is a sizeable part of a cell's width, which is where it grows.
"""
import os

import numpy as np

from oracle import pyoracle as po


def host_threads():
    """Oracle threads: the host cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def nudged(mesh, seed):
    """The mesh with every node coordinate moved by one ulp (seeded sign)."""
    m = mesh.copy()
    rng = np.random.default_rng(seed)
    sgn = rng.choice([-1.0, 1.0], size=m.xy.shape)
    m.xy = m.xy + sgn * np.spacing(np.abs(m.xy))
    return m


def residual_sensitivity(mesh, flow, W, options=None, seeds=(101, 202), threads=None):
    """Per cell: max over the seeds of max_k |M_k(nudged) - M_k| / gross_k
    (flow) and |R(nudged) - R| / gross_SA (SA right-hand side, 0 in laminar
    runs), with M, gross and R of the unmoved mesh; `options` the oracle's
    options (pyoracle.Options)."""
    threads = threads or host_threads()
    o = po.Oracle(mesh, options=options, threads=threads)
    o.set_freestream(*flow)
    o.set_state(W)
    M, G = o.compute_residual()
    Gsa = o.sa_gross()
    del o
    s_flow = np.zeros(mesh.n_cells)
    s_sa = np.zeros(mesh.n_cells)
    for seed in seeds:
        p = po.Oracle(nudged(mesh, seed), options=options, threads=threads)
        p.set_freestream(*flow)
        p.set_state(W)
        Mp, _ = p.compute_residual()
        del p
        s_flow = np.maximum(s_flow, (np.abs(Mp[:4] - M[:4]) / G).max(axis=0))
        if Gsa.any():
            s_sa = np.maximum(s_sa, np.abs(Mp[4] - M[4]) / np.where(Gsa > 0, Gsa, 1.0))
    return s_flow, s_sa


# GPU against oracle, per cell: the larger of the base bar (rounding of the
# flux arithmetic itself, a few ulp of the gross flux) and a fixed multiple
# of the cell's measured geometric sensitivity
BASE_TOL = 1e-12
SENS_FACTOR = 8.0


def tolerance(s):
    return np.maximum(BASE_TOL, SENS_FACTOR * s)
