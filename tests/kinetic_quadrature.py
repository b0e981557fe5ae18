"""Brute-force velocity-space and time quadrature of the paper's kinetic
expressions (Sec. 2.1: Eq.2, the slope expansion and moment relations after Eq.4, Eq.11-14), independent of the
oracle's moment recursions and closed-form time integrals.

A Maxwellian g = rho (lam/pi)^((K+2)/2) exp(-lam((u-U)^2 + (v-V)^2 + xi^2))
is integrated on a tensor grid: Gauss-Legendre in u (split at u = 0 for the
Heaviside half spaces), Gauss-Hermite in v, and Gauss-Legendre in the radius
of the K-dimensional internal variable xi (weight r^(K-1) exp(-lam r^2)).
"""
import numpy as np
from numpy.polynomial.hermite import hermgauss
from numpy.polynomial.legendre import leggauss

K = 3
NU, NV, NR = 160, 48, 48


def _gl(a, b, n):
    x, w = leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def grid(U, V, lam, region):
    """Nodes (u, v, xi2) and weights of the normalised Maxwellian with mean
    (U, V) and parameter lam, restricted to u > 0 (region=+1), u < 0 (-1) or
    the whole line (0).  Returns arrays broadcastable to (NU, NV, NR)."""
    s = 1.0 / np.sqrt(2.0 * lam)
    lo, hi = U - 16 * s, U + 16 * s
    if region > 0:
        lo = max(lo, 0.0)
    elif region < 0:
        hi = min(hi, 0.0)
    if hi <= lo:
        z = np.zeros((1, 1, 1))
        return z, z, z, z
    u, wu = _gl(lo, hi, NU)
    wu = wu * np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)
    xh, wh = hermgauss(NV)
    v = V + xh / np.sqrt(lam)
    wv = wh / np.sqrt(np.pi)
    r, wr = _gl(0.0, 12.0 / np.sqrt(lam), NR)
    wr = wr * r ** (K - 1) * np.exp(-lam * r * r)
    wr = wr / wr.sum()
    return (u[:, None, None], v[None, :, None], (r * r)[None, None, :],
            wu[:, None, None] * wv[None, :, None] * wr[None, None, :])


def integ(fn, U, V, lam, region, rho=1.0):
    """rho * integral of fn(u, v, xi2) (a list of arrays, one per output
    component) against the normalised Maxwellian over the region."""
    u, v, x2, w = grid(U, V, lam, region)
    vals = fn(u, v, x2)
    return np.array([rho * np.sum(w * np.broadcast_to(f, w.shape)) for f in vals])


def psi(u, v, x2):
    one = np.ones_like(u * v * x2)
    return [one, u * one, v * one, 0.5 * (u * u + v * v + x2)]


def poly(a, u, v, x2):
    """Slope expansion of Sec. 2.1 (after Eq.4): a1 + a2 u + a3 v + a4 (u^2 + v^2 + xi^2) / 2"""
    return a[0] + a[1] * u + a[2] * v + 0.5 * a[3] * (u * u + v * v + x2)


def prim(W):
    r = W[0]
    U, V = W[1] / r, W[2] / r
    lam = (K + 2) * r / (4.0 * (W[3] - 0.5 * r * (U * U + V * V)))
    return r, U, V, lam


def moments_quad(U, lam, region, kmax):
    """<u^k>, k = 0..kmax, by quadrature (the v, xi parts integrate to 1)."""
    out = []
    for k in range(kmax + 1):
        out.append(integ(lambda u, v, x2, k=k: [u ** k + 0 * v * x2], U, 0.0, lam, region)[0])
    return np.array(out)


def xi_moments_quad(lam, kmax):
    u, v, x2, w = grid(0.0, 0.0, lam, 0)
    return np.array([np.sum(w * np.broadcast_to(x2 ** k, w.shape)) for k in range(kmax + 1)])


def time_factors(t, tau):
    """The six time factors of Eq.13, in order."""
    e = np.exp(-t / tau)
    return [1.0 - e, tau * (-1.0 + e) + t * e, t - tau + tau * e, e, -(t + tau) * e, -tau * e]


def time_integrals_quad(dt, tau, n=64):
    """Composite Gauss-Legendre on [0, dt], panels graded geometrically
    from t = 0 so that exp(-t/tau) is resolved for any dt/tau."""
    edges = [0.0]
    h = 0.25 * tau
    while edges[-1] + h < dt:
        edges.append(edges[-1] + h)
        h *= 2.0
    edges.append(dt)
    out = np.zeros(6)
    for a, b in zip(edges[:-1], edges[1:]):
        t, w = _gl(a, b, n)
        out += np.array([np.sum(w * c) for c in time_factors(t, tau)])
    return out


def eq13_velocity_parts(d, Wl, Wr):
    """The velocity-space parts of the six Eq.13 terms integrated against
    u psi (flux moments) and against psi (conservative moments), given the
    coefficients in ``d`` (the oracle's face_detail dictionary)."""
    rl, Ul, Vl, laml = prim(Wl)
    rr, Ur, Vr, lamr = prim(Wr)
    W0 = d["W0"]
    r0, U0, V0, lam0 = prim(W0)
    res = {}
    for wt_name, wt in (("F", lambda u: u), ("C", lambda u: 1.0 + 0 * u)):
        parts = []
        # 1: g0
        parts.append(integ(lambda u, v, x2: [wt(u) * p for p in psi(u, v, x2)], U0, V0, lam0, 0, r0))
        # 2: ((abar_n^l H + abar_n^r (1-H)) u + abar_t v) g0
        p2 = (integ(lambda u, v, x2: [wt(u) * p * u * poly(d["abnl"], u, v, x2) for p in psi(u, v, x2)], U0, V0, lam0, +1, r0)
              + integ(lambda u, v, x2: [wt(u) * p * u * poly(d["abnr"], u, v, x2) for p in psi(u, v, x2)], U0, V0, lam0, -1, r0)
              + integ(lambda u, v, x2: [wt(u) * p * v * poly(d["abt"], u, v, x2) for p in psi(u, v, x2)], U0, V0, lam0, 0, r0))
        parts.append(p2)
        # 3: Abar g0
        parts.append(integ(lambda u, v, x2: [wt(u) * p * poly(d["Ab"], u, v, x2) for p in psi(u, v, x2)], U0, V0, lam0, 0, r0))
        # 4: H g^l + (1-H) g^r
        parts.append(integ(lambda u, v, x2: [wt(u) * p for p in psi(u, v, x2)], Ul, Vl, laml, +1, rl)
                     + integ(lambda u, v, x2: [wt(u) * p for p in psi(u, v, x2)], Ur, Vr, lamr, -1, rr))
        # 5: (u a_n + v a_t) H g^l + (...)(1-H) g^r
        parts.append(integ(lambda u, v, x2: [wt(u) * p * (u * poly(d["aln"], u, v, x2) + v * poly(d["alt"], u, v, x2))
                                             for p in psi(u, v, x2)], Ul, Vl, laml, +1, rl)
                     + integ(lambda u, v, x2: [wt(u) * p * (u * poly(d["arn"], u, v, x2) + v * poly(d["art"], u, v, x2))
                                               for p in psi(u, v, x2)], Ur, Vr, lamr, -1, rr))
        # 6: A^l H g^l + A^r (1-H) g^r
        parts.append(integ(lambda u, v, x2: [wt(u) * p * poly(d["Al"], u, v, x2) for p in psi(u, v, x2)], Ul, Vl, laml, +1, rl)
                     + integ(lambda u, v, x2: [wt(u) * p * poly(d["Ar"], u, v, x2) for p in psi(u, v, x2)], Ur, Vr, lamr, -1, rr))
        res[wt_name] = parts
    return res
