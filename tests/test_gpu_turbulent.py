"""The turbulent flat plate on the GPU (meshgen.turbulent_plate, Ma 0.2,
Re 5e6 per unit length, SA with nu~_inf = 3 nu_inf), from the free stream
at CFL 10 to the paper's convergence criterion (Eq.40 <= 3e-8): skin
friction within 1 % of the oracle's converged state
(tests/golden/turbulent_plate_converged.npz) on x in [0.25, 1.5], and the
same correlation and law-of-the-wall pins as the oracle's state."""
import os
import sys

import numpy as np
import pytest

from paper_1709_00803_amd import meshgen as mg
from tests import turbulent_plate as tp

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def igks():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1709_00803_amd import igks as m
    return m


def test_turbulent_plate_converges(igks):
    from oracle import pyoracle as po
    fx = np.load(os.path.join(HERE, "golden", "turbulent_plate_converged.npz"))
    m = mg.turbulent_plate()
    s = igks.Solver(m, cfl_init=10.0, chunk=250)
    s.set_freestream(float(fx["mach"]), 0.0, float(fx["re"]), float(fx["nut"]))
    it = 0
    while it < 25000:
        s.iterate(500)
        it += 500
        r = s.residual()
        if r["eq40"] <= 3e-8:
            break
    say(f"[turbulent plate] Eq.40 = {r['eq40']:.2e} after {it} iterations, drop {r['res_drop']:.2e}")
    assert r["eq40"] <= 3e-8
    W = s.get_state()
    wl = s.wall_loads()
    o = po.Oracle(m)
    o.set_freestream(float(fx["mach"]), 0.0, float(fx["re"]), float(fx["nut"]))
    o.set_state(fx["W"])
    o.compute_residual()
    wo, c = o.wall_loads(), o.cells()
    assert np.allclose(wl["xw"], wo["xw"])
    sel = (wo["xw"] >= tp.X_RANGE[0]) & (wo["xw"] <= tp.X_RANGE[1])
    dcf = np.abs(wl["cf"][sel] / wo["cf"][sel] - 1).max()
    say(f"[turbulent plate] max |cf_gpu / cf_oracle - 1| = {dcf:.2e}, cd gpu {wl['cd']:.6f} oracle {wo['cd']:.6f}")
    assert dcf <= 0.01
    assert tp.check(W, c["xc"], c["yc"], wl["xw"], wl["cf"]) == []
