"""Writes tests/golden/cavity100_converged.npz: the oracle's converged
state of the lid-driven cavity (100x100 uniform quads on the unit square,
lid speed U_0 = 1, Ma 0.1 sqrt(3), Re 1000 on the cavity width, walls held
at the free-stream temperature), started at rest with the lid's density
and pressure, CFL growing by Eq.25 from CFL_0, run to a 1e-6 drop of the
density residual (or max_it).  With adiabatic walls the lid's work has no
way out and there is no steady state.

Calls only the oracle and the mesh generator.  Usage:
    python tests/golden/make_cavity_state.py [n [cfl0 [max_it]]]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pyoracle as po  # noqa: E402
from paper_1709_00803_amd import meshgen as mg  # noqa: E402

MACH = 0.1 * np.sqrt(3.0)
RE = 1000.0


def rest(W):
    """The lid's density and pressure with the fluid at rest."""
    W = W.copy()
    W[3] -= 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0]
    W[1] = W[2] = 0.0
    return W


DROP = 1e-6


def main(n=100, cfl0=10.0, max_it=60000, out=None):
    m = mg.cavity(n)
    o = po.Oracle(m, cfl_init=cfl0, wall_temp=1.0)
    o.set_freestream(MACH, 0.0, RE)
    o.set_state(rest(o.get_state()))
    t = time.time()
    it = 0
    while it < max_it:
        o.iterate(500)
        it += 500
        r = o.residual()
        print(f"{it} {time.time() - t:.1f}s drop={r['res_drop']:.3e} res={r['res_l2']:.3e} cfl={r['cfl']:.3e}",
              flush=True)
        if r["res_drop"] < DROP:
            break
    out = out or os.path.join(HERE, f"cavity{n}_converged.npz")
    np.savez_compressed(out, W=o.get_state(), iterations=it, drop=r["res_drop"], n=n, cfl0=cfl0, wall_temp=1.0)
    print("wrote", out)


if __name__ == "__main__":
    a = sys.argv[1:]
    main(int(a[0]) if a else 100, float(a[1]) if len(a) > 1 else 10.0, int(a[2]) if len(a) > 2 else 60000)
