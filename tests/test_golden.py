"""Physics pins of the oracle's converged states: the laminar flat plate
against the Blasius boundary layer (textbook solution of the boundary-layer
equations), stored in tests/golden/plate64x32_converged.npz; the
lid-driven cavity against the vortex data of Table 1, stored in
tests/golden/cavity100_converged.npz; the turbulent flat plate (SA)
against White's skin-friction correlation and the law of the wall, stored
in tests/golden/turbulent_plate_converged.npz.

Fixture: tests/golden/make_plate_state.py runs the oracle alone on the
64x32 plate mesh (x in [-0.2, 1], plate from x = 0, first cell 1e-3,
y-ratio 1.1, top at y = 0.2), Ma 0.3, Re_L 1e4, CFL 10 growing by Eq.25,
to a 1e-10 drop of the density residual.

Pins (the tolerances cover what separates this finite, compressible,
low-Re computation from the leading-order incompressible Blasius solution:
the second-order leading-edge correction, about +6% to +11% in C_f over
Re_x = 1e3 - 3e3, and the outflow rule of Sec. 2.5 at x = 1, which
imposes the free-stream incoming Riemann invariant inside the boundary
layer and raises C_f increasingly toward the exit):
  * the stored state is a steady state of the oracle (residual <= 1e-9 of
    the gross face flux),
  * C_f sqrt(Re_x) / 0.664 in [1.0, 1.16] for x in [0.08, 0.3], and C_f
    decreasing along the plate there,
  * the velocity profile u/U_inf at x ~ 0.2 within 0.03 of Blasius f'(eta),
    eta = y sqrt(U_inf / (nu x)), for eta < 6,
  * C_f = 0 ahead of the plate (symmetry boundary).
A viscosity off by a factor 2 (C_f off by 1.41), a slip wall (C_f = 0) or
a missing viscous flux fails them.
"""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import pyoracle as po
from paper_1709_00803_amd import meshgen as mg

from tests import cavity_vortex as cv
from tests import turbulent_plate as tp

HERE = os.path.dirname(os.path.abspath(__file__))
RE = 1e4


@pytest.fixture(scope="module")
def plate():
    fx = np.load(os.path.join(HERE, "golden", "plate64x32_converged.npz"))
    m = mg.flat_plate()
    o = po.Oracle(m, cfl_init=10.0)
    o.set_freestream(0.3, 0.0, RE)
    o.set_state(fx["W"])
    return m, o, fx["W"]


def blasius():
    """f''' + f f'' / 2 = 0, f(0) = f'(0) = 0, f'(inf) = 1 (f''(0) = 0.332057...)."""
    sol = solve_ivp(lambda t, y: [y[1], y[2], -0.5 * y[0] * y[2]], [0.0, 12.0], [0.0, 0.0, 0.332057336],
                    dense_output=True, rtol=1e-11, atol=1e-12)
    assert abs(sol.y[1, -1] - 1.0) < 1e-6       # the shooting value reaches f'(inf) = 1
    return sol


def test_fixture_is_steady(plate):
    m, o, W = plate
    M, G = o.compute_residual()
    assert (np.abs(M[:4]) / G).max() <= 1e-9


def test_skin_friction_against_blasius(plate):
    m, o, W = plate
    wl = o.wall_loads()
    x, cf = wl["xw"], wl["cf"]
    plate_faces = x > 0.0
    assert np.all(np.abs(cf[~plate_faces]) < 1e-10)      # symmetry part: no shear
    sel = (x >= 0.08) & (x <= 0.3)
    ratio = cf[sel] / (0.664 / np.sqrt(RE * x[sel]))
    assert ratio.min() >= 1.0 and ratio.max() <= 1.16, ratio
    assert np.all(np.diff(cf[sel][np.argsort(x[sel])]) < 0)


def test_velocity_profile_against_blasius(plate):
    m, o, W = plate
    c = o.cells()
    sol = blasius()
    xs = c["xc"][np.argmin(np.abs(c["xc"] - 0.2))]
    col = np.abs(c["xc"] - xs) < 1e-9
    u = W[1][col] / W[0][col]
    eta = c["yc"][col] * np.sqrt(RE / xs)
    keep = eta < 6.0
    assert keep.sum() >= 10
    err = np.abs(u[keep] - sol.sol(eta[keep])[1])
    assert err.max() <= 0.03, err.max()


# ---------------------------------------------------------------- cavity

def test_vortex_analysis_on_a_known_stream_function():
    """psi = -A sin^2(pi x) sin^2(pi y): minimum -A at (1/2, 1/2) with
    vorticity -laplacian(psi) = 4 pi^2 A there; the bottom corners hold no
    secondary vortex (psi ~ x^2 y^2 > -A, found at the corner cells)."""
    n, A = 100, 0.1
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    sx, cx, sy, cy = np.sin(np.pi * X), np.cos(np.pi * X), np.sin(np.pi * Y), np.cos(np.pi * Y)
    u = -A * sx ** 2 * 2 * np.pi * sy * cy          # d psi / dy
    v = A * 2 * np.pi * sx * cx * sy ** 2           # -d psi / dx
    W = np.zeros((5, n * n))
    W[0] = 1.0
    W[1], W[2] = u.ravel(), v.ravel()
    t = cv.table(W, n)
    assert abs(t["psi"] + A) <= 2e-4 * A
    assert abs(t["x"] - 0.5) <= 1e-3 and abs(t["y"] - 0.5) <= 1e-3
    assert abs(t["omega"] - 4 * np.pi ** 2 * A) <= 2e-3 * 4 * np.pi ** 2 * A
    assert t["x_l"] < 0.02 and t["y_r"] < 0.02 and abs(t["psi_l"]) < 1e-6


@pytest.fixture(scope="module")
def cavity():
    fx = np.load(os.path.join(HERE, "golden", "cavity100_converged.npz"))
    n = int(fx["n"])
    o = po.Oracle(mg.cavity(n), wall_temp=float(fx["wall_temp"]))
    o.set_freestream(0.1 * np.sqrt(3.0), 0.0, 1000.0)
    o.set_state(fx["W"])
    return n, o, fx["W"]


def test_cavity_fixture_is_steady(cavity):
    n, o, W = cavity
    M, G = o.compute_residual()
    assert np.abs(M[:4]).max() <= 1e-8 * G.max()
    # the lid's work leaves through the isothermal walls: what is left in
    # the cells is under 0.1 % of what the lid puts in
    f = o.faces()
    lid = (f["fr"] < 0) & (f["bc"] == mg.MOVING_WALL)
    work = -o.debug()["flux"][3][lid].sum()
    assert work > 0 and abs(M[3].sum()) <= 1e-3 * work


def test_cavity_vortices_against_table1(cavity):
    n, o, W = cavity
    t = cv.table(W, n)
    assert cv.check_table1(t, 1.0 / n) == [], t


# ---------------------------------------------------------------- turbulent plate

@pytest.fixture(scope="module")
def turbulent():
    fx = np.load(os.path.join(HERE, "golden", "turbulent_plate_converged.npz"))
    m = mg.turbulent_plate()
    o = po.Oracle(m)
    o.set_freestream(float(fx["mach"]), 0.0, float(fx["re"]), float(fx["nut"]))
    o.set_state(fx["W"])
    return m, o, fx["W"]


def test_turbulent_plate_fixture_is_steady(turbulent):
    m, o, W = turbulent
    M, G = o.compute_residual()
    assert np.abs(M[:4]).max() <= 1e-9 * G.max()
    assert W[4].min() >= 0.0


def test_turbulent_plate_against_white_and_law_of_the_wall(turbulent):
    """C_f within 6 % of White's correlation on x in [0.25, 1.5]; u+ on the
    log law (30 <= y+ <= 300) to 0.3 and on the sublayer (y+ < 3) to 5 %
    at x ~ 1.  A laminar solution (C_f ~ 0.664 / sqrt(Re_x), ten times
    lower) or a wrong von Karman constant fails."""
    m, o, W = turbulent
    o.compute_residual()
    wl, c = o.wall_loads(), o.cells()
    assert tp.check(W, c["xc"], c["yc"], wl["xw"], wl["cf"]) == []
