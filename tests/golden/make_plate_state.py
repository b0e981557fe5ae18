"""Writes tests/golden/plate64x32_converged.npz: the oracle's converged
state of the laminar flat plate (64x32 quads, Ma 0.3, Re_L 1e4, CFL 10
growing by Eq.25), run to a 1e-10 drop of the density residual.

Calls only the oracle and the mesh generator.  Usage:
    python tests/golden/make_plate_state.py [nx ny x1]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pyoracle as po  # noqa: E402
from paper_1709_00803_amd import meshgen as mg  # noqa: E402


def main(nx=64, ny=32, x1=1.0, out=None, max_it=20000):
    m = mg.flat_plate(nx=nx, ny=ny, x1=x1)
    o = po.Oracle(m, cfl_init=10.0)
    o.set_freestream(0.3, 0.0, 1e4)
    t = time.time()
    it = 0
    while it < max_it:
        o.iterate(500)
        it += 500
        r = o.residual()
        print(f"{it} {time.time() - t:.1f}s drop={r['res_drop']:.3e} cfl={r['cfl']:.3e}", flush=True)
        if r["res_drop"] < 1e-10:
            break
    wl = o.wall_loads()
    for x, c in zip(wl["xw"], wl["cf"]):
        if x > 0:
            xe = x - m.xy[m.bface_nodes[m.bface_tag == mg.WALL].ravel(), 0].min()
            print(f"x={x:.4f} cf={c:.5f} blasius={0.664 / np.sqrt(1e4 * xe):.5f} ratio={c / (0.664 / np.sqrt(1e4 * xe)):.4f}")
    out = out or os.path.join(HERE, f"plate{nx}x{ny}_converged.npz")
    np.savez_compressed(out, W=o.get_state(), iterations=it, drop=r["res_drop"], nx=nx, ny=ny, x1=x1)
    print("wrote", out)


if __name__ == "__main__":
    a = sys.argv[1:]
    if a:
        main(int(a[0]), int(a[1]), float(a[2]), out=a[3] if len(a) > 3 else None)
    else:
        main()
