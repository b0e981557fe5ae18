"""ctypes wrapper of liboigks.so (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# OIGKS_LIB names another build of the same source (the mutation tests load
# copies with a planted mistake this way)
LIB_PATH = os.environ.get("OIGKS_LIB") or os.path.join(HERE, "liboigks.so")

_lib = None


class Options(C.Structure):
    _fields_ = [("limiter", C.c_int), ("cfl_init", C.c_double), ("cfl_min", C.c_double),
                ("cfl_max", C.c_double), ("cfl_mode", C.c_int), ("cfl_flux", C.c_double),
                ("visc_sr", C.c_int), ("mu_law", C.c_int), ("scheme", C.c_int),
                ("wall_temp", C.c_double), ("limiter_freeze", C.c_double),
                ("tau_jump", C.c_int), ("lusgs_op", C.c_int)]


class Residual(C.Structure):
    _fields_ = [("iteration", C.c_int), ("res_l2", C.c_double), ("res_drop", C.c_double),
                ("res_inf", C.c_double), ("eq40", C.c_double), ("cfl", C.c_double),
                ("dt_flux", C.c_double), ("sa_l2", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = C.CDLL(LIB_PATH)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        dp = C.POINTER(C.c_double)
        L.oigks_create.argtypes = [C.POINTER(p), C.POINTER(Options)]
        L.oigks_destroy.argtypes = [p]
        L.oigks_last_error.argtypes = [p]; L.oigks_last_error.restype = C.c_char_p
        L.oigks_default_options.argtypes = [C.POINTER(Options)]
        L.oigks_mesh_upload.argtypes = [p, i, dp, i, C.POINTER(C.c_int), C.POINTER(C.c_int), i,
                                        C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.oigks_set_freestream.argtypes = [p, d, d, d, d]
        L.oigks_iterate.argtypes = [p, i, C.POINTER(C.c_int)]
        L.oigks_get_residual.argtypes = [p, C.POINTER(Residual)]
        L.oigks_get_limiter.argtypes = [p, dp, C.POINTER(C.c_int)]
        L.oigks_get_state.argtypes = [p, dp]
        L.oigks_set_state.argtypes = [p, dp]
        L.oigks_compute_residual.argtypes = [p, dp, dp]
        L.oigks_lusgs_solve.argtypes = [p, d, dp]
        L.oigks_get_wall_loads.argtypes = [p, dp, dp, dp, dp, dp]
        for nm in ("oigks_n_cells", "oigks_n_faces", "oigks_n_wall_faces"):
            getattr(L, nm).argtypes = [p]; getattr(L, nm).restype = i
        L.oigks_dt_flux.argtypes = [p]; L.oigks_dt_flux.restype = d
        L.oigks_get_faces.argtypes = [p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      dp, dp, dp, dp, dp]
        L.oigks_get_cells.argtypes = [p, dp, dp, dp, dp]
        L.oigks_get_debug.argtypes = [p] + [dp] * 9
        L.oigks_moments.argtypes = [d, d, i, i, dp]
        L.oigks_moment_matrix.argtypes = [d, d, d, dp]
        L.oigks_slope.argtypes = [dp, dp, dp]
        L.oigks_face_detail.argtypes = [dp] * 8 + [d, d, d, d, dp]
        L.oigks_sa_source.argtypes = [d, d, d, d, dp]
        L.oigks_jac_vec.argtypes = [dp, d, d, dp, dp]
        L.oigks_collision_time.argtypes = [p, d, d, d]; L.oigks_collision_time.restype = d
        L.oigks_ghost_state.argtypes = [p, i, dp, d, d, dp]
        L.oigks_mu.argtypes = [p, d]; L.oigks_mu.restype = d
        L.oigks_set_threads.argtypes = [p, i]
        L.oigks_sa_gross.argtypes = [p, dp]
        L.oigks_set_sweep_blocks.argtypes = [p, C.POINTER(C.c_int)]
        L.oigks_set_block_passes.argtypes = [p, i]
        L.oigks_get_roe.argtypes = [p, dp]
        L.oigks_roe_abs.argtypes = [dp, dp, d, d, d, i, dp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


def default_options(**kw) -> Options:
    o = Options()
    lib().oigks_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class OracleError(RuntimeError):
    pass


class Oracle:
    """FP64 CPU oracle bound to one mesh and one flow condition."""

    def __init__(self, mesh, options: Options | None = None, threads: int = 1, **kw):
        self.L = lib()
        self.opt = options or default_options(**kw)
        self.ctx = C.c_void_p()
        self._chk(self.L.oigks_create(C.byref(self.ctx), C.byref(self.opt)))
        if threads != 1:
            self.set_threads(threads)
        self.mesh = mesh
        xy, pxy = _d(mesh.xy.reshape(-1))
        cp, pcp = _i(mesh.cell_ptr)
        cn, pcn = _i(mesh.cell_nodes)
        bn, pbn = _i(mesh.bface_nodes.reshape(-1))
        bt, pbt = _i(mesh.bface_tag)
        self._chk(self.L.oigks_mesh_upload(self.ctx, mesh.n_nodes, pxy, mesh.n_cells, pcp, pcn,
                                            mesh.n_bfaces, pbn, pbt))
        self.n = self.L.oigks_n_cells(self.ctx)
        self.nf = self.L.oigks_n_faces(self.ctx)
        self.nwall = self.L.oigks_n_wall_faces(self.ctx)

    def _chk(self, rc):
        if rc != 0:
            raise OracleError(f"oracle error {rc}: {self.L.oigks_last_error(self.ctx).decode()}")
        return rc

    def __del__(self):
        try:
            if self.ctx:
                self.L.oigks_destroy(self.ctx)
                self.ctx = C.c_void_p()
        except Exception:
            pass

    def set_threads(self, n):
        """OpenMP threads of the per-cell and per-face loops (1 by default);
        the results are the same bit for bit whatever the count."""
        self._chk(self.L.oigks_set_threads(self.ctx, int(n)))

    def set_freestream(self, mach, alpha_deg, reynolds, nut_ratio=-1.0):
        self._chk(self.L.oigks_set_freestream(self.ctx, mach, alpha_deg, reynolds, nut_ratio))
        self.flow = (mach, alpha_deg, reynolds, nut_ratio)

    def iterate(self, n):
        done = C.c_int(0)
        rc = self.L.oigks_iterate(self.ctx, n, C.byref(done))
        self._chk(rc)
        return done.value

    def residual(self) -> dict:
        r = Residual()
        self.L.oigks_get_residual(self.ctx, C.byref(r))
        return r.as_dict()

    def get_state(self):
        W = np.zeros((5, self.n))
        _, p = _d(W)
        self.L.oigks_get_state(self.ctx, W.ctypes.data_as(C.POINTER(C.c_double)))
        return W

    def set_state(self, W):
        W, p = _d(np.asarray(W).reshape(5, self.n))
        self._chk(self.L.oigks_set_state(self.ctx, p))

    def compute_residual(self):
        M = np.zeros((5, self.n)); G = np.zeros((4, self.n))
        self._chk(self.L.oigks_compute_residual(self.ctx, M.ctypes.data_as(C.POINTER(C.c_double)),
                                                G.ctypes.data_as(C.POINTER(C.c_double))))
        return M, G

    def set_sweep_blocks(self, blk):
        """Sweep block of each cell (None: one block)."""
        if blk is None:
            self._chk(self.L.oigks_set_sweep_blocks(self.ctx, None))
            return
        b, p = _i(np.asarray(blk).reshape(self.n))
        self._chk(self.L.oigks_set_sweep_blocks(self.ctx, p))

    def set_block_passes(self, n):
        """Passes of the block sweeps: 1, or 2 (the second with the first's
        cross-block terms on its right-hand side)."""
        self._chk(self.L.oigks_set_block_passes(self.ctx, int(n)))

    def sa_gross(self):
        """Per cell, the gross size of the SA right-hand side (sum of the
        magnitudes of its face terms times S, plus Omega |Sr|)."""
        out = np.zeros(self.n)
        self._chk(self.L.oigks_sa_gross(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def lusgs_solve(self, cfl):
        dW = np.zeros((5, self.n))
        self._chk(self.L.oigks_lusgs_solve(self.ctx, cfl, dW.ctypes.data_as(C.POINTER(C.c_double))))
        return dW

    def limiter(self):
        """(phi, frozen): the last computed (or held) Eq.9 factors, 4 x n."""
        phi = np.zeros((4, self.n))
        fr = C.c_int()
        self.L.oigks_get_limiter(self.ctx, phi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(fr))
        return phi, bool(fr.value)

    def wall_loads(self):
        cl, cd = C.c_double(), C.c_double()
        cf = np.zeros(self.nwall); cp = np.zeros(self.nwall); xw = np.zeros(self.nwall)
        P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self._chk(self.L.oigks_get_wall_loads(self.ctx, C.byref(cl), C.byref(cd), P(cf), P(cp), P(xw)))
        return dict(cl=cl.value, cd=cd.value, cf=cf, cp=cp, xw=xw)

    def faces(self):
        nf = self.nf
        fl = np.zeros(nf, np.int32); fr = np.zeros(nf, np.int32); bc = np.zeros(nf, np.int32)
        nx, ny, ln, xm, ym = (np.zeros(nf) for _ in range(5))
        IP = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
        P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self.L.oigks_get_faces(self.ctx, IP(fl), IP(fr), IP(bc), P(nx), P(ny), P(ln), P(xm), P(ym))
        return dict(fl=fl, fr=fr, bc=bc, nx=nx, ny=ny, len=ln, xm=xm, ym=ym)

    def cells(self):
        a, x, y, d = (np.zeros(self.n) for _ in range(4))
        P = lambda v: v.ctypes.data_as(C.POINTER(C.c_double))
        self.L.oigks_get_cells(self.ctx, P(a), P(x), P(y), P(d))
        return dict(area=a, xc=x, yc=y, dwall=d)

    def debug(self):
        nf, n = self.nf, self.n
        out = dict(flux=np.zeros((4, nf)), lam=np.zeros(nf), wg=np.zeros((5, nf)), D=np.zeros(n),
                   Dsa=np.zeros(n), lamc=np.zeros(n), dtimp=np.zeros(n), grad=np.zeros((8, n)),
                   vort=np.zeros(n))
        P = lambda v: v.ctypes.data_as(C.POINTER(C.c_double))
        self.L.oigks_get_debug(self.ctx, *(P(out[k]) for k in
                                           ("flux", "lam", "wg", "D", "Dsa", "lamc", "dtimp", "grad", "vort")))
        out["dt_flux"] = self.L.oigks_dt_flux(self.ctx)
        return out

    def roe(self):
        """The per-face Roe dissipation matrices |A| (+ viscous part) of the
        last residual, shape (nf, 4, 4); needs lusgs_op = 1."""
        out = np.zeros((self.nf, 4, 4))
        if self.L.oigks_get_roe(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double))) != 0:
            raise OracleError("the Roe operator is not in use (lusgs_op = 0)")
        return out

    def collision_time(self, rho0, lam0, nut_f=0.0):
        return self.L.oigks_collision_time(self.ctx, rho0, lam0, nut_f)

    def ghost_state(self, bc, Wi, nx, ny):
        Wi, p = _d(Wi)
        out = np.zeros(5)
        self.L.oigks_ghost_state(self.ctx, bc, p, nx, ny, out.ctypes.data_as(C.POINTER(C.c_double)))
        return out

    def mu(self, lam):
        return self.L.oigks_mu(self.ctx, lam)


# ---------------- kernel-level helpers ----------------

def moments(U, lam, kind, n=10):
    out = np.zeros(n)
    lib().oigks_moments(U, lam, kind, n, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def moment_matrix(U, V, lam):
    M = np.zeros(16)
    lib().oigks_moment_matrix(U, V, lam, M.ctypes.data_as(C.POINTER(C.c_double)))
    return M.reshape(4, 4)


def slope(W, dW):
    W, pw = _d(W); dW, pd = _d(dW)
    a = np.zeros(4)
    lib().oigks_slope(pw, pd, a.ctypes.data_as(C.POINTER(C.c_double)))
    return a


FACE_KEYS = ["W0", "lam0", "aln", "alt", "arn", "art", "abnl", "abnr", "abt", "Al", "Ar", "Ab", "T", "F"]
_SIZES = dict(W0=4, lam0=1, T=6, F=4)


def face_detail(Wl, Gln, Glt, Wr, Grn, Grt, Wlc, Wrc, dl, dr, dt, tau) -> dict:
    args = [_d(a) for a in (Wl, Gln, Glt, Wr, Grn, Grt, Wlc, Wrc)]
    out = np.zeros(59)
    lib().oigks_face_detail(*(p for _, p in args), dl, dr, dt, tau, out.ctypes.data_as(C.POINTER(C.c_double)))
    res, k = {}, 0
    for key in FACE_KEYS:
        n = _SIZES.get(key, 4)
        res[key] = out[k:k + n].copy() if n > 1 else float(out[k])
        k += n
    return res


def sa_source(nut, nu, d, omega):
    out = np.zeros(4)
    lib().oigks_sa_source(nut, nu, d, omega, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def roe_abs(Wl, Wr, nx, ny, vis=0.0, kinetic=False):
    Wl, pl = _d(Wl); Wr, pr = _d(Wr)
    out = np.zeros(16)
    lib().oigks_roe_abs(pl, pr, nx, ny, vis, int(kinetic), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out.reshape(4, 4)


def jac_vec(W, nx, ny, d):
    W, pw = _d(W); d, pd = _d(d)
    out = np.zeros(4)
    lib().oigks_jac_vec(pw, nx, ny, pd, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out
