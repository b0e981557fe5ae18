"""Pins of the oracle's optional Roe-matrix LU-SGS operator (lusgs_op = 1):
the dissipation |A| of the first-order Roe flux (Eq.18) in place of the
scalar spectral radius of Eq.20.  CPU only."""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_1709_00803_amd import meshgen as mg
from tests.test_oracle_solver import GAM, _euler_flux_n, _jac_fd, smooth_state

DELTA = 0.1   # entropy fix: |lambda| >= DELTA c


def _prim(W):
    r = W[0]; u = W[1] / r; v = W[2] / r
    p = (GAM - 1) * (W[3] - 0.5 * r * (u * u + v * v))
    return r, u, v, p, (W[3] + p) / r


def _roe_state(Wl, Wr):
    """Conservative state with the Roe-averaged velocity and total enthalpy
    (density sqrt(rho_l rho_r)); the flux Jacobian depends on u, v, H only."""
    rl, ul, vl, _, Hl = _prim(Wl)
    rr, ur, vr, _, Hr = _prim(Wr)
    sl, sr = math.sqrt(rl), math.sqrt(rr)
    u = (sl * ul + sr * ur) / (sl + sr); v = (sl * vl + sr * vr) / (sl + sr); H = (sl * Hl + sr * Hr) / (sl + sr)
    r = sl * sr
    E = (r * H + (GAM - 1) * 0.5 * r * (u * u + v * v)) / GAM
    return np.array([r, r * u, r * v, E, 0.0]), math.sqrt((GAM - 1) * (H - 0.5 * (u * u + v * v)))


def _jac_cs(W, nx, ny):
    """The flux Jacobian by complex-step differentiation (exact to rounding,
    so that the double eigenvalue q keeps two independent eigenvectors)."""
    J = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(5, dtype=complex); e[k] = 1e-30j
        J[:, k] = np.imag(_euler_flux_n(W + e, nx, ny)) / 1e-30
    return J


def _kin_mag(s, c):
    """The mean of |u| for u normal with mean s and variance RT = c^2/gamma,
    by adaptive quadrature of each side of the kink at u = 0 (independent of
    the closed form the oracle uses)."""
    from scipy.integrate import quad
    sig = c / math.sqrt(GAM)
    pdf = lambda u: math.exp(-0.5 * ((u - s) / sig) ** 2) / (sig * math.sqrt(2 * math.pi))
    lo = quad(lambda u: -u * pdf(u), -np.inf, 0.0, epsabs=1e-14, epsrel=1e-13)[0]
    hi = quad(lambda u: u * pdf(u), 0.0, np.inf, epsabs=1e-14, epsrel=1e-13)[0]
    return lo + hi


def _abs_by_eig(Wl, Wr, nx, ny, kin=False):
    """|A| as a function of the Jacobian J at the Roe state: J is
    diagonalisable with the three distinct eigenvalues q - c, q, q + c, so
    f(J) = sum_m f(l_m) prod_{k != m} (J - l_k I) / (l_m - l_k) (Sylvester's
    formula), f(l) = max(|l|, delta c).  Unlike an eigenvector matrix this
    stays well conditioned where q is 0 (a wall's mirrored states)."""
    Wa, c = _roe_state(Wl, Wr)
    J = _jac_cs(Wa, nx, ny)
    q = (Wa[1] * nx + Wa[2] * ny) / Wa[0]
    ls = (q - c, q, q + c)
    A = np.zeros((4, 4))
    for m, lm in enumerate(ls):
        P = np.eye(4)
        for k, lk in enumerate(ls):
            if k != m:
                P = P @ (J - lk * np.eye(4)) / (lm - lk)
        A += (_kin_mag(lm, c) if kin else max(abs(lm), DELTA * c)) * P
    return A, Wa


CASES = [  # (Wl, Wr, n): subsonic, supersonic, a stagnation-like low normal speed (the floor active)
    ([1.2, 0.3, -0.1, 2.5], [0.9, 0.5, 0.2, 2.2], (0.6, 0.8)),
    ([1.0, 2.4, 0.3, 5.5], [1.1, 2.5, 0.1, 5.9], (1.0, 0.0)),
    ([1.0, 0.01, 0.4, 1.9], [1.05, -0.01, 0.45, 2.0], (math.cos(0.03), math.sin(0.03))),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_roe_abs_kinetic_magnitudes(case):
    """lusgs_op 2: the same matrix function with each eigenvalue s replaced
    by the mean of |u| over a Maxwellian spread of normal velocities about s
    (quadrature here): at least |s|, about 0.674 c at s = 0 (sqrt(2/(pi
    gamma)) c), and |s| far from 0."""
    Wl, Wr, (nx, ny) = CASES[case]
    Wl = np.array(Wl + [0.0]); Wr = np.array(Wr + [0.0])
    want, _ = _abs_by_eig(Wl, Wr, nx, ny, kin=True)
    got = po.roe_abs(Wl, Wr, nx, ny, kinetic=True)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    _, c = _roe_state(Wl, Wr)
    assert _kin_mag(0.0, c) == pytest.approx(math.sqrt(2.0 / (math.pi * GAM)) * c, rel=1e-12)
    assert _kin_mag(5.0 * c, c) == pytest.approx(5.0 * c, rel=1e-6)
    ev = np.sort(np.real(np.linalg.eigvals(got)))
    assert ev[0] >= 0.67 * c


@pytest.mark.parametrize("case", range(len(CASES)))
def test_roe_abs_is_the_eigen_decomposition(case):
    """|A| = V max(|Lambda|, delta c) V^-1 of the Euler flux Jacobian (taken
    here by complex-step differentiation of the flux, then Sylvester's
    formula and numpy's eigen-solver) at the Roe-averaged state; that state is pinned by Roe's property
    A (W_r - W_l) = F(W_r) - F(W_l).  |A| does not depend on the sign of n
    or the order of the two states, and a viscous part adds to the diagonal."""
    Wl, Wr, (nx, ny) = CASES[case]
    Wl = np.array(Wl + [0.0]); Wr = np.array(Wr + [0.0])
    want, Wa = _abs_by_eig(Wl, Wr, nx, ny)
    J = _jac_cs(Wa, nx, ny)
    dF = _euler_flux_n(Wr, nx, ny) - _euler_flux_n(Wl, nx, ny)
    assert np.abs(J @ (Wr - Wl)[:4] - dF).max() <= 1e-8 * np.abs(dF).max()
    got = po.roe_abs(Wl, Wr, nx, ny)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the same matrix from numpy's eigenvectors (well conditioned here)
    lam, V = np.linalg.eig(J)
    _, c = _roe_state(Wl, Wr)
    byeig = np.real(V @ np.diag(np.maximum(np.abs(np.real(lam)), DELTA * c)) @ np.linalg.inv(V))
    assert np.abs(byeig - want).max() <= 1e-10 * np.abs(want).max()
    assert np.allclose(po.roe_abs(Wl, Wr, -nx, -ny), got, rtol=1e-12, atol=1e-13)
    assert np.allclose(po.roe_abs(Wr, Wl, nx, ny), got, rtol=1e-12, atol=1e-13)
    assert np.allclose(po.roe_abs(Wl, Wr, nx, ny, 0.7) - got, 0.7 * np.eye(4), rtol=0, atol=1e-12)
    if case == 2:   # the floor is what sets the two slow eigenvalues here
        _, c = _roe_state(Wl, Wr)
        ev = np.sort(np.abs(np.real(np.linalg.eigvals(J))))
        assert ev[0] < DELTA * c
        assert np.sort(np.real(np.linalg.eigvals(got)))[0] == pytest.approx(DELTA * c, rel=1e-9)


def test_roe_abs_of_equal_states_is_abs_jacobian():
    """With W_l = W_r the Roe average is the state itself; away from the
    floor |A| then squares to J^2 and has the eigenvalue magnitudes
    |q - c|, |q|, |q + c|."""
    W = np.array([1.3, 0.9, -0.4, 3.1, 0.0])
    nx, ny = 0.8, -0.6
    r, u, v, p, _ = _prim(W)
    c = math.sqrt(GAM * p / r); q = u * nx + v * ny
    A = po.roe_abs(W, W, nx, ny)
    J = _jac_fd(W, nx, ny)
    assert np.abs(A @ A - J @ J).max() <= 1e-7 * np.abs(J @ J).max()
    ev = np.sort(np.real(np.linalg.eigvals(A)))
    assert np.allclose(ev, np.sort([abs(q - c), abs(q), abs(q), abs(q + c)]), rtol=1e-10)


@pytest.mark.parametrize("top,blocks,op", [(mg.OUTFLOW, 0, 1), (mg.MOVING_WALL, 0, 1), (mg.OUTFLOW, 1, 1),
                                           (mg.OUTFLOW, 2, 1), (mg.MOVING_WALL, 1, 2)],
                         ids=["outflow", "moving_wall", "blocks", "blocks2", "kinetic"])
def test_roe_lusgs_solves_factored_system(top, blocks, op):
    """With the Roe operator the sweeps solve (L + D) D^-1 (D + U) dW = M with
    4x4 blocks D_i = Omega/dt I + 1/2 sum |A_ij| S_ij (dt of Eq.24) and
    off-diagonal blocks 1/2 (J_j - |A_ij|) S_ij, the lagged ghost increments
    of Sec. 2.5 in the backward sweep as in the scalar form.  The stored
    |A_ij| of each face is the Roe matrix of its two cell-centre states (the
    ghost state at a boundary) plus the viscous part of the spectral radius
    times the identity.  With sweep blocks a face between two blocks keeps
    lambda_ij I in D, its pair is left out of L and U, and with two passes
    the second solves again with M - X dW1 on the right (X: those pairs'
    1/2 (J_j - lambda_ij I) S_ij).  op 2: the kinetic wave magnitudes."""
    tags = dict(bottom=mg.WALL, top=top, left=mg.FREESTREAM, right=mg.SYMMETRY)
    m = mg.colour_order(mg.random_hybrid(5, 4, seed=7, tags=tags))[0]
    o = po.Oracle(m, lusgs_op=op)
    blk = mg.sweep_blocks(m, 7) if blocks else np.zeros(m.n_cells, dtype=np.int32)
    if blocks:
        assert blk.max() >= 3
        o.set_sweep_blocks(blk)
        o.set_block_passes(blocks)
    o.set_freestream(0.4, 5.0, 1e3)
    W = smooth_state(o, 0.1, 3)
    o.set_state(W)
    cfl = 50.0
    M, _ = o.compute_residual()
    dW = o.lusgs_solve(cfl)
    dbg = o.debug(); f = o.faces(); n = o.n
    lam, wg = dbg["lam"], dbg["wg"]
    A = o.roe()
    for k in range(o.nf):
        i, j = f["fl"][k], f["fr"][k]
        nx, ny = f["nx"][k], f["ny"][k]
        Wj = W[:, j] if j >= 0 else wg[:, k]
        sr = []
        for Wc in (W[:, i], Wj):
            r, u, v, p, _ = _prim(Wc)
            sr.append(abs(u * nx + v * ny) + math.sqrt(GAM * p / r))
        vis = lam[k] - max(sr)
        assert vis > 0.0
        want, _ = _abs_by_eig(W[:, i], Wj, nx, ny, kin=op == 2)
        assert np.abs(A[k] - vis * np.eye(4) - want).max() <= (1e-9 if op == 2 else 1e-12) * np.abs(want).max()
    Dm = np.zeros((4 * n, 4 * n)); L = np.zeros_like(Dm); U = np.zeros_like(Dm); G = np.zeros_like(Dm)
    X = np.zeros_like(Dm)
    for i in range(n):
        Dm[4 * i:4 * i + 4, 4 * i:4 * i + 4] = dbg["lamc"][i] / cfl * np.eye(4)
    for k in range(o.nf):
        i, j = f["fl"][k], f["fr"][k]
        nx, ny, S = f["nx"][k], f["ny"][k], f["len"][k]
        if j >= 0 and blk[i] != blk[j]:
            for a, b, sg in ((i, j, 1.0), (j, i, -1.0)):
                Dm[4 * a:4 * a + 4, 4 * a:4 * a + 4] += 0.5 * lam[k] * S * np.eye(4)
                X[4 * a:4 * a + 4, 4 * b:4 * b + 4] += 0.5 * (_jac_fd(W[:, b], sg * nx, sg * ny) - lam[k] * np.eye(4)) * S
            continue
        for a in (i, j):
            if a >= 0:
                Dm[4 * a:4 * a + 4, 4 * a:4 * a + 4] += 0.5 * A[k] * S
        if j >= 0:
            for a, b, sg in ((i, j, 1.0), (j, i, -1.0)):
                jb = 0.5 * (_jac_fd(W[:, b], sg * nx, sg * ny) - A[k]) * S
                (L if b < a else U)[4 * a:4 * a + 4, 4 * b:4 * b + 4] += jb
        else:
            bc = f["bc"][k]
            if bc == mg.WALL:
                B = np.diag([1.0, -1.0, -1.0, 1.0])
            elif bc == mg.MOVING_WALL:
                al = math.radians(5.0)
                vt = -math.cos(al) * ny + math.sin(al) * nx
                vw = vt * np.array([-ny, nx])
                B = np.array([[1.0, 0, 0, 0], [2 * vw[0], -1, 0, 0], [2 * vw[1], 0, -1, 0],
                              [2 * vw @ vw, -2 * vw[0], -2 * vw[1], 1]])
            elif bc == mg.SYMMETRY:
                nn = np.array([nx, ny]); B = np.eye(4); B[1:3, 1:3] = np.eye(2) - 2 * np.outer(nn, nn)
            else:
                B = np.zeros((4, 4))
            G[4 * i:4 * i + 4, 4 * i:4 * i + 4] += 0.5 * (_jac_fd(wg[:, k], nx, ny) - A[k]) * S @ B
    Mv = M[:4].T.reshape(-1)
    dws = np.linalg.solve(L + Dm, Mv)
    want = np.linalg.solve(Dm + U, (Dm - G) @ dws)
    if blocks == 2:
        dws = np.linalg.solve(L + Dm, Mv - X @ want)
        want = np.linalg.solve(Dm + U, (Dm - G) @ dws)
    got = dW[:4].T.reshape(-1)
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    # the scalar operator solves another system
    s = po.Oracle(m)
    if blocks:
        s.set_sweep_blocks(blk)
        s.set_block_passes(blocks)
    s.set_freestream(0.4, 5.0, 1e3)
    s.set_state(W)
    other = s.lusgs_solve(cfl)[:4].T.reshape(-1)
    assert np.abs(other - want).max() > 1e-4 * np.abs(want).max()


def test_roe_operator_keeps_the_fixed_point():
    """The implicit operator changes the path, not the steady solution: a
    laminar plate converged with either operator gives the same state and
    wall drag, the Roe operator in fewer iterations."""
    m = mg.flat_plate(24, 12)
    runs = {}
    for op in (0, 1):
        o = po.Oracle(m, lusgs_op=op, cfl_init=10.0)
        o.set_freestream(0.3, 0.0, 1e4)
        it = 0
        while it < 20000:
            o.iterate(50)
            it += 50
            if o.residual()["res_drop"] <= 1e-10:
                break
        assert o.residual()["res_drop"] <= 1e-10
        runs[op] = (it, o.get_state(), o.wall_loads()["cd"])
    (n0, W0, d0), (n1, W1, d1) = runs[0], runs[1]
    assert np.abs(W1[:4] - W0[:4]).max() <= 1e-8 * np.abs(W0[:4]).max()
    assert d1 == pytest.approx(d0, rel=1e-7)
    assert n1 < n0


def test_lusgs_op_is_validated():
    m = mg.random_hybrid(3, 3, seed=1)
    with pytest.raises(po.OracleError):
        po.Oracle(m, lusgs_op=3)
    o = po.Oracle(m)
    o.set_freestream(0.3, 0.0, 1e3)
    with pytest.raises(po.OracleError):
        o.roe()
