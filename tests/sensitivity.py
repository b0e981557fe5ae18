"""How far the oracle's own residual moves when its inputs move by rounding:
the scale against which two independent FP64 codes (the GPU library and the
oracle compute the geometry, the state's derived quantities and the flux with
different formulas) can be compared cell by cell.

Two kinds of one-ulp perturbation, each with seeded random signs: every node
coordinate of the mesh (the codes compute centroids, normals, lengths and
distances from the nodes differently), and every component of the cell
state (the codes derive velocity, lambda, pressure and viscosity from the
conservative state with different formulas, which acts like a rounding of
the state).  The oracle evaluates the residual of the perturbed input.  Per
cell, the largest change over the four flow components relative to the
cell's gross flux sum_faces |F S| (and for the SA right-hand side relative to
its own gross size) is the cell's measured sensitivity.  It grows in thin
high-aspect-ratio cells, where the wall-normal differences (W0 - W_c) / d of
Eq.5 lose about log10(aspect ratio) digits, and at a cusp, where the
coordinates' rounding is a sizeable part of a cell's width.
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


def nudged_state(W, seed):
    """The state with every component moved by one ulp (seeded sign)."""
    rng = np.random.default_rng(seed)
    sgn = rng.choice([-1.0, 1.0], size=W.shape)
    return W + sgn * np.spacing(np.abs(W))


def residual_sensitivity(mesh, flow, W, options=None, seeds=(101, 202), threads=None):
    """Per cell: max over the seeds and the two kinds of perturbation (the
    mesh's nodes, the state) of max_k |M_k(nudged) - M_k| / gross_k (flow)
    and |R(nudged) - R| / gross_SA (SA right-hand side, 0 in laminar runs),
    with M, gross and R of the unperturbed input; `options` the oracle's
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
    def take(Mp):
        nonlocal s_flow, s_sa
        s_flow = np.maximum(s_flow, (np.abs(Mp[:4] - M[:4]) / G).max(axis=0))
        if Gsa.any():
            s_sa = np.maximum(s_sa, np.abs(Mp[4] - M[4]) / np.where(Gsa > 0, Gsa, 1.0))

    for seed in seeds:
        p = po.Oracle(nudged(mesh, seed), options=options, threads=threads)
        p.set_freestream(*flow)
        p.set_state(W)
        take(p.compute_residual()[0])
        del p
    o = po.Oracle(mesh, options=options, threads=threads)
    o.set_freestream(*flow)
    for seed in seeds:
        o.set_state(nudged_state(W, seed + 1))
        take(o.compute_residual()[0])
    del o
    return s_flow, s_sa


# GPU against oracle, per cell: the larger of the base bar (rounding of the
# flux arithmetic itself, a few ulp of the gross flux) and a fixed multiple
# of the cell's measured geometric sensitivity
BASE_TOL = 1e-12
SENS_FACTOR = 8.0


def tolerance(s):
    return np.maximum(BASE_TOL, SENS_FACTOR * s)
