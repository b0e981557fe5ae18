"""Checks of a converged turbulent flat-plate state (meshgen.turbulent_plate,
Ma 0.2, Re 5e6 per unit length, SA): skin friction against White's
correlation for turbulent flat plates, C_f = 0.455 / ln^2(0.06 Re_x), and
the velocity profile in wall units against the viscous sublayer (u+ = y+)
and the log law u+ = ln(y+) / 0.41 + 5.0.  Test infrastructure only.

Bounds: White's correlation represents smooth flat-plate data to a few per
cent; the SA model's skin friction on a well-resolved plate lies within
about 5 % of it over Re_x = 1e6 - 8e6 (measured here 0.96 - 1.04); past
x = 1.5 the outflow rule (Sec. 2.5) raises C_f toward the exit, so the
check stops there.  The log law is checked where it holds, 30 <= y+ <= 300,
to 0.3 in u+, and the sublayer below y+ = 3 to 5 %.
"""
import numpy as np

RE = 5e6
X_RANGE = (0.25, 1.5)


def white(rex):
    return 0.455 / np.log(0.06 * rex) ** 2


def skin_friction_ratio(xw, cf):
    sel = (xw >= X_RANGE[0]) & (xw <= X_RANGE[1])
    return xw[sel], cf[sel] / white(RE * xw[sel])


def wall_units(W, xc, yc, xw, cf, x=1.0):
    """u+ and y+ of the column of cells nearest x (rho_inf = U_inf = 1)."""
    xs = xc[np.argmin(np.abs(xc - x))]
    col = np.abs(xc - xs) < 1e-12
    ut = np.sqrt(0.5 * cf[np.argmin(np.abs(xw - xs))])
    yp = yc[col] * ut * RE
    up = W[1][col] / W[0][col] / ut
    o = np.argsort(yp)
    return yp[o], up[o]


def check(W, xc, yc, xw, cf):
    """List of failed pins (empty when the state passes)."""
    bad = []
    _, r = skin_friction_ratio(xw, cf)
    if len(r) < 10 or r.min() < 0.94 or r.max() > 1.06:
        bad.append(("cf/white", float(r.min()), float(r.max())))
    yp, up = wall_units(W, xc, yc, xw, cf)
    log = (yp >= 30) & (yp <= 300)
    dlog = np.abs(up[log] - (np.log(yp[log]) / 0.41 + 5.0))
    if log.sum() < 5 or dlog.max() > 0.3:
        bad.append(("log law", int(log.sum()), float(dlog.max()) if log.any() else None))
    sub = yp < 3
    dsub = np.abs(up[sub] / yp[sub] - 1)
    if sub.sum() < 1 or dsub.max() > 0.05:
        bad.append(("sublayer", int(sub.sum()), float(dsub.max()) if sub.any() else None))
    return bad
