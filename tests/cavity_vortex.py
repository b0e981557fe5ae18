"""Vortex data of a lid-driven cavity state on the n x n uniform mesh of
meshgen.cavity (cells numbered row by row from the bottom), in the form of
Table 1: the stream function psi at the centres of the primary vortex and
of the two bottom secondary vortices, their locations, and the vorticity
at the primary centre (magnitude).

psi is u = d(psi)/dy with psi = 0 on the bottom wall, integrated up each
column of cell centres (midpoint rule); each extremum is located by a
quadratic fit to the 3 x 3 cells around the extreme cell; the vorticity
dv/dx - du/dy is taken by central differences and interpolated bilinearly.
Test infrastructure only.
"""
import numpy as np
from scipy.interpolate import RegularGridInterpolator

# Table 1, structured-grid row of the paper (100 x 100 uniform grid)
TABLE1 = dict(omega=2.0861, psi=-0.1178, x=0.5335, y=0.5681,
              psi_l=2.2461e-4, x_l=0.0820, y_l=0.0716,
              psi_r=1.7123e-3, x_r=0.8720, y_r=0.1132)
# Table 1, unstructured-mesh row (the adaptive 8933-cell polygon mesh)
TABLE1_UNSTRUCTURED = dict(omega=2.0902, psi=-0.1179, x=0.5405, y=0.5721,
                           psi_l=2.2870e-4, x_l=0.0899, y_l=0.0862,
                           psi_r=1.7289e-3, x_r=0.8752, y_r=0.1145)


def fields(W, n):
    r = W[0].reshape(n, n)
    u = W[1].reshape(n, n) / r
    v = W[2].reshape(n, n) / r
    h = 1.0 / n
    psi = h * (np.cumsum(u, axis=0) - 0.5 * u)
    x = (np.arange(n) + 0.5) * h
    om = np.gradient(v, h, axis=1) - np.gradient(u, h, axis=0)
    return x, psi, om


def extremum(psi, x, box, sign):
    """Extremum of sign * psi over cells with centres in box = (x0, x1, y0, y1)."""
    n = len(x)
    X, Y = np.meshgrid(x, x, indexing="xy")
    inside = (X >= box[0]) & (X <= box[1]) & (Y >= box[2]) & (Y <= box[3])
    j, i = np.unravel_index(np.argmax(np.where(inside, sign * psi, -np.inf)), psi.shape)
    j, i = min(max(j, 1), n - 2), min(max(i, 1), n - 2)
    h = x[1] - x[0]
    A, b = [], []
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            dx, dy = di * h, dj * h
            A.append([1.0, dx, dy, dx * dx, dx * dy, dy * dy])
            b.append(psi[j + dj, i + di])
    c = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    d = np.linalg.solve(np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]]), -c[1:3])
    val = c[0] + c[1] * d[0] + c[2] * d[1] + c[3] * d[0] ** 2 + c[4] * d[0] * d[1] + c[5] * d[1] ** 2
    return float(val), float(x[i] + d[0]), float(x[j] + d[1])


def table(W, n):
    x, psi, om = fields(W, n)
    p = extremum(psi, x, (0.3, 0.8, 0.3, 0.8), -1)
    l = extremum(psi, x, (0.0, 0.25, 0.0, 0.25), +1)
    r = extremum(psi, x, (0.65, 1.0, 0.0, 0.4), +1)
    w = RegularGridInterpolator((x, x), om)((p[2], p[1]))
    return dict(omega=abs(float(w)), psi=p[0], x=p[1], y=p[2], psi_l=l[0], x_l=l[1], y_l=l[2],
                psi_r=r[0], x_r=r[1], y_r=r[2])


def resample(W, xc, yc, n=100):
    """Cell-centre velocities of any mesh of the unit square, interpolated
    linearly (nearest value outside the centroids' hull) to the cell centres
    of an n x n grid, as a state (rho = 1) that table() reads."""
    from scipy.interpolate import griddata
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    pts = np.stack([xc, yc], 1)
    out = np.zeros((5, n * n))
    out[0] = 1.0
    for k in (1, 2):
        u = W[k] / W[0]
        g = griddata(pts, u, (X, Y), method="linear")
        gn = griddata(pts, u, (X, Y), method="nearest")
        out[k] = np.where(np.isnan(g), gn, g).ravel()
    return out


def check_table1(t, h, ref=None, omega_tol=0.02):
    """Table 1 pins: primary psi and omega within 2 % (the paper's own
    differences from the reference solutions it lists reach 2.0 %, and a
    second-order solution at Ma 0.17 carries O(h^2) and O(Ma^2) errors of
    that size), secondary psi within 5 %, every centre within one cell
    width h.  Returns the list of failures."""
    ref = TABLE1 if ref is None else ref
    bad = []
    for k, tol in (("omega", omega_tol), ("psi", 0.02), ("psi_l", 0.05), ("psi_r", 0.05)):
        if abs(t[k] - ref[k]) > tol * abs(ref[k]):
            bad.append((k, t[k], ref[k]))
    for k in ("x", "y", "x_l", "y_l", "x_r", "y_r"):
        if abs(t[k] - ref[k]) > h:
            bad.append((k, t[k], ref[k]))
    return bad
