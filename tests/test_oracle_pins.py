"""Pins of oracle parts that the physics and invariance pins elsewhere do
not fix: the viscosity law, the Eq.9 limiter factor on hand-built cells
whose factor follows by hand, the wall loads (Cp, C_L, C_D) on states
whose loads are known in closed form or by symmetry, and the full SA
implicit diagonal of Eq.31-32.  CPU only.
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1709_00803_amd import meshgen as mg

GAM = 1.4
S_STAR = 110.4 / 288.15       # Sutherland's constant over the 288.15 K free-stream temperature


# ------------------------------------------------------------ viscosity law

@pytest.mark.parametrize("theta", [0.5, 1.0, 2.0, 4.0])
def test_sutherland_viscosity(theta):
    """mu / mu_inf = theta^(3/2) (1 + S*) / (theta + S*) with theta = T / T_inf
    = lambda_inf / lambda (Sutherland's law, free stream at 288.15 K);
    constant viscosity with mu_law = 1."""
    m = mg.random_hybrid(3, 3, seed=1)
    ma, re = 0.4, 2.5e4
    lam_inf = GAM * ma * ma / 2.0          # rho_inf = 1, p_inf = 1 / (gamma Ma^2), lambda = rho / (2 p)
    mu_inf = 1.0 / re
    o = po.Oracle(m)
    o.set_freestream(ma, 0.0, re)
    want = mu_inf * theta ** 1.5 * (1.0 + S_STAR) / (theta + S_STAR)
    assert o.mu(lam_inf / theta) == pytest.approx(want, rel=1e-14)
    c = po.Oracle(m, mu_law=1)
    c.set_freestream(ma, 0.0, re)
    assert c.mu(lam_inf / theta) == pytest.approx(mu_inf, rel=1e-15)


def test_sutherland_exponent_and_constant_distinguished():
    """The pin above fails a wrong exponent or a wrong S*: at theta = 4 a
    power 1 gives 0.5 of the value, S* = 110.4 / 273.15 gives 1.01."""
    th = 4.0
    good = th ** 1.5 * (1.0 + S_STAR) / (th + S_STAR)
    assert abs(th * (1.0 + S_STAR) / (th + S_STAR) / good - 0.5) < 1e-12
    s2 = 110.4 / 273.15
    assert abs(th ** 1.5 * (1.0 + s2) / (th + s2) / good - 1.0) > 5e-3


# ------------------------------------------------------------ limiter (Eq.9)

def grid3(h=0.1):
    """Nine unit squares of side h; cell 4 is the middle one, with its four
    face neighbours 1 (below), 3 (left), 5 (right), 7 (above) at distance h."""
    xs = np.arange(4) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], 1)
    nid = lambda i, j: j * 4 + i
    cells = []
    for j in range(3):
        for i in range(3):
            cells += [nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)]
    bn = []
    for i in range(3):
        bn += [[nid(i, 0), nid(i + 1, 0)], [nid(i, 3), nid(i + 1, 3)], [nid(0, i), nid(0, i + 1)],
               [nid(3, i), nid(3, i + 1)]]
    return mg.Mesh(xy=xy, cell_ptr=np.arange(0, 37, 4, dtype=np.int32), cell_nodes=np.array(cells, np.int32),
                   bface_nodes=np.array(bn, np.int32), bface_tag=np.full(len(bn), mg.FREESTREAM, np.int32),
                   meta={})


@pytest.mark.parametrize("beta", [0.0, 0.1, 0.2, 1.0 / 3.0, 0.5, 1.0])
@pytest.mark.parametrize("side", [+1, -1])
def test_limiter_factor_by_hand(beta, side):
    """Density linear in x, rho = 1 + a (x - x_c), in the middle cell and its
    neighbours, except that the neighbour on side `side` holds
    1 + side beta a h instead of 1 + side a h.  The least-squares gradient of
    the middle cell over its four face neighbours is then (1 + beta) a / 2
    along x and 0 along y, its largest vertex excess (1 + beta) a h / 4 on the
    modified side, and the stencil's extreme there beta a h, so the Eq.9
    factor is min(1, 4 beta / (1 + beta)) (the other side allows
    4 / (1 + beta) >= 1): phi < 1 for beta < 1/3, phi = 1 from 1/3 on, 0 at
    beta = 0.  Momentum 0 and energy uniform: their factors are 1."""
    h, a = 0.1, 0.3
    m = grid3(h)
    o = po.Oracle(m, limiter=1)
    o.set_freestream(0.3, 0.0, 1e3)
    c = o.cells()
    W = o.get_state()
    xc = c["xc"][4]
    W[0] = 1.0 + a * (c["xc"] - xc)
    nb = 5 if side > 0 else 3
    W[0][nb] = 1.0 + side * beta * a * h
    W[1] = 0.0
    W[2] = 0.0
    W[3] = 2.0
    o.set_state(W)
    o.compute_residual()
    phi, _ = o.limiter()
    want = min(1.0, 4.0 * beta / (1.0 + beta))
    assert phi[0][4] == pytest.approx(want, rel=1e-12, abs=1e-14)
    assert phi[1][4] == 1.0 and phi[2][4] == 1.0 and phi[3][4] == 1.0
    g = o.debug()["grad"]
    assert g[0][4] == pytest.approx(want * (1.0 + beta) * a / 2.0, rel=1e-12, abs=1e-14)
    assert abs(g[4][4]) <= 1e-14


# ------------------------------------------------------------ wall loads

def box(nx=6, ny=5, tags=None, lx=1.0, ly=0.8, seed=7):
    """Jittered hybrid box, every side a no-slip wall unless tagged."""
    t = dict(bottom=mg.WALL, top=mg.WALL, left=mg.WALL, right=mg.WALL)
    t.update(tags or {})
    return mg.random_hybrid(nx, ny, seed=seed, tags=t, jitter=0.25, lx=lx, ly=ly)


def rest_state(o, p):
    """Gas at rest with density 1 and uniform pressure p."""
    W = o.get_state()
    W[0] = 1.0
    W[1] = W[2] = 0.0
    W[3] = p / (GAM - 1.0)
    return W


@pytest.mark.parametrize("kappa", [1.0, 1.25, 0.8])
def test_wall_loads_of_a_closed_box_at_rest(kappa):
    """Gas at rest at uniform pressure kappa p_inf in a box of no-slip walls:
    the gas-kinetic momentum flux through each wall face is the pressure
    times its normal, so Cp = (kappa - 1) p_inf / q_inf on every face
    (q_inf = 1/2, p_inf = 1 / (gamma Ma^2)), Cf = 0, and the closed walls
    give C_L = C_D = 0."""
    ma = 0.3
    m = box()
    o = po.Oracle(m)
    o.set_freestream(ma, 17.0, 1e3)
    pinf = 1.0 / (GAM * ma * ma)
    o.set_state(rest_state(o, kappa * pinf))
    wl = o.wall_loads()
    want = (kappa - 1.0) * pinf / 0.5
    assert len(wl["cp"]) == o.nwall > 0
    assert np.allclose(wl["cp"], want, rtol=0, atol=1e-12 * pinf)
    assert np.abs(wl["cf"]).max() <= 1e-12 * pinf
    assert abs(wl["cl"]) <= 1e-12 * pinf and abs(wl["cd"]) <= 1e-12 * pinf


@pytest.mark.parametrize("alpha", [0.0, 30.0, 90.0, -50.0])
def test_wall_loads_of_a_floor_at_rest(alpha):
    """Only the floor (y = 0, length 1) is a wall; the other sides are
    symmetry faces.  Gas at rest at pressure p pushes the floor down with
    force (0, -p) per unit length, so with the reference 0.5 rho |V|^2 c =
    1/2: C_D = -2 p sin(alpha) (drag along (cos alpha, sin alpha)) and
    C_L = -2 p cos(alpha) (lift along (-sin alpha, cos alpha)); Cp =
    2 (p - p_inf) on every floor face."""
    ma = 0.4
    m = box(tags=dict(top=mg.SYMMETRY, left=mg.SYMMETRY, right=mg.SYMMETRY))
    o = po.Oracle(m)
    o.set_freestream(ma, alpha, 1e3)
    pinf = 1.0 / (GAM * ma * ma)
    p = 1.1 * pinf
    o.set_state(rest_state(o, p))
    wl = o.wall_loads()
    a = math.radians(alpha)
    tol = 1e-12 * p
    assert wl["cd"] == pytest.approx(-2.0 * p * math.sin(a), abs=tol)
    assert wl["cl"] == pytest.approx(-2.0 * p * math.cos(a), abs=tol)
    assert np.allclose(wl["cp"], 2.0 * (p - pinf), rtol=0, atol=tol)
    assert np.abs(wl["cf"]).max() <= tol


def small_airfoil():
    return mg.joukowski_hybrid(32, 6, 2e-3, 1.3, r_far=6.0, seed=5, target_cells=1500)


def evolved_state(o, iters=4):
    o.iterate(iters)
    return o.get_state()


def test_wall_loads_rotate_with_mesh_and_stream():
    """C_L and C_D are measured against the free-stream direction: rotating
    the mesh and the stream by the same angle (the state's momentum rotated
    with them) leaves them unchanged, and Cp, Cf per face too.  A C_L or
    C_D that used the angle with a wrong sign or in the wrong place fails."""
    m = small_airfoil()
    flow = (0.3, 4.0, 5e3, -1.0)
    o = po.Oracle(m, cfl_init=5.0)
    o.set_freestream(*flow)
    W = evolved_state(o)
    ref = o.wall_loads()
    assert abs(ref["cl"]) > 1e-3 and abs(ref["cd"]) > 1e-3
    for deg in (25.0, -110.0):
        th = math.radians(deg)
        r = po.Oracle(mg.transform(m, theta=th), cfl_init=5.0)
        r.set_freestream(flow[0], flow[1] + deg, flow[2], flow[3])
        Wr = W.copy()
        Wr[1] = math.cos(th) * W[1] - math.sin(th) * W[2]
        Wr[2] = math.sin(th) * W[1] + math.cos(th) * W[2]
        r.set_state(Wr)
        got = r.wall_loads()
        for k in ("cl", "cd"):
            assert got[k] == pytest.approx(ref[k], rel=1e-10, abs=1e-12), (deg, k)
        assert np.allclose(got["cp"], ref["cp"], rtol=1e-9, atol=1e-10)
        assert np.allclose(got["cf"], ref["cf"], rtol=1e-9, atol=1e-10)


def test_wall_loads_mirror():
    """Mirroring the mesh in y with alpha -> -alpha (and the state's
    y-momentum negated) turns the lift over and keeps the drag: C_L -> -C_L,
    C_D -> C_D."""
    m = small_airfoil()
    flow = (0.3, 4.0, 5e3, -1.0)
    o = po.Oracle(m, cfl_init=5.0)
    o.set_freestream(*flow)
    W = evolved_state(o)
    ref = o.wall_loads()
    r = po.Oracle(mg.transform(m, mirror_y=True), cfl_init=5.0)
    r.set_freestream(flow[0], -flow[1], flow[2], flow[3])
    Wm = W.copy()
    Wm[2] = -W[2]
    r.set_state(Wm)
    got = r.wall_loads()
    assert got["cl"] == pytest.approx(-ref["cl"], rel=1e-10)
    assert got["cd"] == pytest.approx(ref["cd"], rel=1e-10)


def test_plate_drag_is_its_skin_friction():
    """On the flat plate at alpha = 0 the wall normals are vertical, so the
    drag is all shear, C_D = sum over the wall faces of Cf S (reference
    length 1), and the lift is minus the pressure integral,
    C_L = -sum (Cp + 2 p_inf) S (the one-sided plate carries p_inf too)."""
    m = mg.flat_plate(16, 8)
    o = po.Oracle(m, cfl_init=10.0)
    ma = 0.3
    o.set_freestream(ma, 0.0, 1e4)
    o.iterate(5)
    wl = o.wall_loads()
    f = o.faces()
    wall = np.where(f["bc"] == mg.WALL)[0]
    order = np.argsort(f["xm"][wall])
    S = f["len"][wall][order]
    cf = wl["cf"][np.argsort(wl["xw"])]
    cp = wl["cp"][np.argsort(wl["xw"])]
    pinf = 1.0 / (GAM * ma * ma)
    assert wl["cd"] == pytest.approx(np.sum(cf * S), rel=1e-12)
    assert wl["cl"] == pytest.approx(-np.sum((cp + 2.0 * pinf) * S), rel=1e-12)
    assert wl["cd"] > 0.0 and (cf[wl["xw"][np.argsort(wl["xw"])] > 0.1] > 0.0).all()
    # the plate mirrored to the top of the flow (its wall faces' own tangent
    # now points against the stream): the same skin friction and drag, the
    # lift reversed
    r = po.Oracle(mg.transform(m, mirror_y=True), cfl_init=10.0)
    r.set_freestream(ma, 0.0, 1e4)
    W = o.get_state()
    W[2] = -W[2]
    r.set_state(W)
    wm = r.wall_loads()
    assert np.allclose(wm["cf"], wl["cf"], rtol=1e-10, atol=1e-14)
    assert wm["cd"] == pytest.approx(wl["cd"], rel=1e-10)
    assert wm["cl"] == pytest.approx(-wl["cl"], rel=1e-10)


# ------------------------------------------------------------ SA diagonal

SA_CB1, SA_CB2, SA_SIG, SA_KAP, SA_CW2, SA_CW3, SA_CV1 = 0.1355, 0.622, 2.0 / 3.0, 0.41, 0.3, 2.0, 7.1


def sa_destruction_jacobian(nut, nu, d, om):
    """max(2 c_w1 f_w nu~ / d^2 - c_b1 S~, 0) of the standard SA model
    (no f_t2) with the S~ clipping of Allmaras et al. (2012)."""
    cw1 = SA_CB1 / SA_KAP ** 2 + (1.0 + SA_CB2) / SA_SIG
    chi = nut / nu
    fv1 = chi ** 3 / (chi ** 3 + SA_CV1 ** 3)
    fv2 = 1.0 - chi / (1.0 + chi * fv1)
    sbar = nut * fv2 / (SA_KAP ** 2 * d * d)
    if sbar >= -0.7 * om:
        st = om + sbar
    else:
        st = om + om * (0.7 ** 2 * om + 0.9 * sbar) / ((0.9 - 2.0 * 0.7) * om - sbar)
    r = min(nut / (st * SA_KAP ** 2 * d * d), 10.0) if st > 0 else 10.0
    g = r + SA_CW2 * (r ** 6 - r)
    fw = g * ((1.0 + SA_CW3 ** 6) / (g ** 6 + SA_CW3 ** 6)) ** (1.0 / 6.0)
    return max(2.0 * cw1 * fw * nut / (d * d) - SA_CB1 * st, 0.0)


def test_sa_diagonal_assembly():
    """Eq.31-32: the SA diagonal of every cell is Omega / dt_imp (= Lambda_c /
    CFL) plus, per face, the upwind outflow u^+ S and the diffusion
    coefficient k S / |r.n|, plus Omega times the non-negative destruction-
    minus-production Jacobian, each part computed here from its definition
    (the source part with the SA formulas above, the vorticity and wall
    distance the oracle reports)."""
    tags = dict(bottom=mg.WALL, top=mg.FARFIELD, left=mg.FREESTREAM, right=mg.SYMMETRY)
    m = mg.random_hybrid(6, 5, seed=19, tags=tags, jitter=0.25)
    o = po.Oracle(m)
    o.set_freestream(0.3, 3.0, 5e5, 3.0)
    W = o.get_state()
    c = o.cells()
    rng = np.random.default_rng(3)
    W[0] *= 1 + 0.05 * np.sin(3 * c["xc"])
    W[1] += 0.1 * np.cos(2 * c["yc"] + 0.3)
    W[4] *= 1 + 20.0 * rng.uniform(0, 1, o.n) * (c["yc"] < 0.3)     # a range of chi, production and destruction
    o.set_state(W)
    cfl = 40.0
    o.compute_residual()
    o.lusgs_solve(cfl)
    dbg = o.debug()
    f = o.faces()

    def nu_lam(w):
        lam = 5.0 * w[0] / (4.0 * (w[3] - 0.5 * (w[1] ** 2 + w[2] ** 2) / w[0]))
        return o.mu(lam) / w[0]

    want = dbg["lamc"] / cfl
    for q in range(o.nf):
        i, j = f["fl"][q], f["fr"][q]
        nx, ny, S = f["nx"][q], f["ny"][q], f["len"][q]
        wj = W[:, j] if j >= 0 else dbg["wg"][:, q]
        if j >= 0:
            rn = abs((c["xc"][j] - c["xc"][i]) * nx + (c["yc"][j] - c["yc"][i]) * ny)
        else:
            rn = 2.0 * ((f["xm"][q] - c["xc"][i]) * nx + (f["ym"][q] - c["yc"][i]) * ny)
        k = (0.5 * (nu_lam(W[:, i]) + nu_lam(wj)) + (1.0 + SA_CB2) * 0.5 * (W[4, i] + wj[4])) / SA_SIG
        for a, sg in ((i, 1.0), (j, -1.0)):
            if a < 0:
                continue
            qa = sg * (W[1, a] * nx + W[2, a] * ny) / W[0, a]
            want[a] += 0.5 * (qa + abs(qa)) * S + k * S / rn
    jd = np.array([sa_destruction_jacobian(W[4, i], nu_lam(W[:, i]), c["dwall"][i], dbg["vort"][i])
                   for i in range(o.n)])
    assert (jd > 0).any() and (jd == 0).any()
    want += c["area"] * jd
    assert np.allclose(dbg["Dsa"], want, rtol=1e-12, atol=0)
