"""Python binding of libigks.so (include/igks.h): argument marshalling only.

Every step of the solver runs in the HIP library.  PyTorch provides the
device workspace (a uint8 tensor) and the stream.  If the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libigks.so")

IGKS_OK, IGKS_EINVAL, IGKS_EMESH, IGKS_ENOMEM, IGKS_ENONPHYS, IGKS_EHIP = 0, -1, -2, -3, -4, -5
IGKS_FP64, IGKS_MIXED = 0, 1
HIST_W = 6

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1709_00803_amd.build "
                      "(or __graft_entry__.build())")
# PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Loading torch first makes libigks bind to that already-loaded runtime, so
# the process holds a single HIP runtime; the other order loads two, and the
# one initialised second finds no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


class igks_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("limiter", C.c_int), ("cfl_init", C.c_double),
                ("cfl_min", C.c_double), ("cfl_max", C.c_double), ("cfl_mode", C.c_int),
                ("cfl_flux", C.c_double), ("visc_sr", C.c_int), ("mu_law", C.c_int),
                ("chunk", C.c_int), ("block", C.c_int), ("sweep", C.c_int), ("flux_lanes", C.c_int),
                ("scheme", C.c_int), ("wall_temp", C.c_double), ("limiter_freeze", C.c_double),
                ("tau_jump", C.c_int), ("block_passes", C.c_int), ("lusgs_op", C.c_int)]


class igks_residual(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("res_l2", C.c_double), ("res_drop", C.c_double),
                ("res_inf", C.c_double), ("eq40", C.c_double), ("cfl", C.c_double),
                ("dt_flux", C.c_double), ("sa_l2", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class igks_scalars(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("cfl", C.c_double), ("res_inf_prev", C.c_double),
                ("res0", C.c_double)]


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
_SIGS = {
    "igks_default_options": (None, [C.POINTER(igks_options)]),
    "igks_create": (C.c_int, [C.POINTER(_P), C.POINTER(igks_options), _P]),
    "igks_destroy": (None, [_P]),
    "igks_last_error": (C.c_char_p, [_P]),
    "igks_mesh_upload": (C.c_int, [_P, C.c_int32, _DP, C.c_int32, _IP, _IP, C.c_int32, _IP, _IP]),
    "igks_mesh_info": (C.c_int, [_P, _IP, _IP, _IP, _IP]),
    "igks_set_sweep_blocks": (C.c_int, [_P, C.c_int32, _IP]),
    "igks_wavefront_sizes": (C.c_int, [_P, _IP, C.c_int32]),
    "igks_workspace_size": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "igks_bind_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "igks_bind_static_workspace": (C.c_int, [_P]),
    "igks_set_freestream": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double]),
    "igks_iterate": (C.c_int, [_P, C.c_int32, _IP]),
    "igks_get_residual": (C.c_int, [_P, C.POINTER(igks_residual)]),
    "igks_get_history": (C.c_int, [_P, _DP, C.c_int32, _IP]),
    "igks_get_state": (C.c_int, [_P, _DP]),
    "igks_set_state": (C.c_int, [_P, _DP, C.POINTER(igks_scalars)]),
    "igks_get_scalars": (C.c_int, [_P, C.POINTER(igks_scalars)]),
    "igks_compute_residual": (C.c_int, [_P, _DP]),
    "igks_get_wall_loads": (C.c_int, [_P, _DP, _DP, _DP, _DP, _DP]),
    "igks_set_profiling": (C.c_int, [_P, C.c_int]),
    "igks_get_kernel_times": (C.c_int, [_P, _DP]),
    "igks_time_kernel": (C.c_int, [_P, C.c_int32, C.c_int32, _DP]),
    "igks_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(igks_options), _P, C.c_int32]),
    "igks_batch_mesh_upload": (C.c_int, [_P, C.c_int32, C.c_int32, _DP, C.c_int32, _IP, _IP, C.c_int32, _IP, _IP]),
    "igks_batch_mesh_info": (C.c_int, [_P, C.c_int32, _IP, _IP, _IP]),
    "igks_batch_set_freestream": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double]),
    "igks_batch_get_residual": (C.c_int, [_P, C.c_int32, C.POINTER(igks_residual)]),
    "igks_batch_get_history": (C.c_int, [_P, C.c_int32, _DP, C.c_int32, _IP]),
    "igks_batch_get_state": (C.c_int, [_P, C.c_int32, _DP]),
    "igks_batch_set_state": (C.c_int, [_P, C.c_int32, _DP, C.POINTER(igks_scalars)]),
    "igks_batch_get_scalars": (C.c_int, [_P, C.c_int32, C.POINTER(igks_scalars)]),
    "igks_batch_compute_residual": (C.c_int, [_P, C.c_int32, _DP]),
    "igks_batch_get_wall_loads": (C.c_int, [_P, C.c_int32, _DP, _DP, _DP, _DP, _DP]),
    "igks_batch_status": (C.c_int, [_P, C.c_int32, _IP]),
    "igks_autotune": (C.c_int, [_P, C.c_int32, _IP]),
    "igks_get_schedule": (C.c_int, [_P, _IP]),
    "igks_set_schedule": (C.c_int, [_P, _IP]),
    "igks_graph_chunk": (C.c_int, [_P, _IP, _IP]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_SIGS)


class IgksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"igks error {code}: {msg}")
        self.code = code


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_DP)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_IP)


def default_options(**kw) -> igks_options:
    o = igks_options()
    igks_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _mesh_args(mesh):
    keep = (_d(mesh.xy.reshape(-1)), _i(mesh.cell_ptr), _i(mesh.cell_nodes), _i(mesh.bface_nodes.reshape(-1)),
            _i(mesh.bface_tag))
    (_, pxy), (_, pcp), (_, pcn), (_, pbn), (_, pbt) = keep
    return keep, (mesh.n_nodes, pxy, mesh.n_cells, pcp, pcn, mesh.n_bfaces, pbn, pbt)


KERNEL_CLASSES = ("prep", "flux", "gather", "reduce", "sweep_fwd", "sweep_bwd")


class _Context:
    """Owns an igks context, its stream and its device workspace."""

    def _open(self, n_inst, options, stream, device, kw):
        import torch
        self.torch = torch
        self.opt = options or default_options(**kw)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.ctx = _P()
        self._device = device
        self._chk(igks_batch_create(C.byref(self.ctx), C.byref(self.opt), _P(self.stream.cuda_stream), n_inst))

    def _bind(self):
        nc, nf, nw, nl = (C.c_int32() for _ in range(4))
        self._chk(igks_mesh_info(self.ctx, C.byref(nc), C.byref(nf), C.byref(nw), C.byref(nl)))
        self.total_cells, self.total_faces, self.total_wall, self.nlev = nc.value, nf.value, nw.value, nl.value
        sz = C.c_size_t()
        self._chk(igks_workspace_size(self.ctx, C.byref(sz)))
        self.ws_bytes = sz.value
        self.workspace = self.torch.empty(self.ws_bytes + 256, dtype=self.torch.uint8, device=self._device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._chk(igks_bind_workspace(self.ctx, _P(aligned), self.ws_bytes))

    def _chk(self, rc):
        if rc != IGKS_OK:
            msg = igks_last_error(self.ctx).decode() if self.ctx else ""
            raise IgksError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            igks_destroy(self.ctx)
            self.ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, n):
        done = C.c_int32(0)
        rc = igks_iterate(self.ctx, n, C.byref(done))
        self._chk(rc)
        return done.value

    def set_profiling(self, on=True):
        self._chk(igks_set_profiling(self.ctx, 1 if on else 0))

    def wavefront_sizes(self):
        """Cells per sweep wavefront (all instances), in sweep order."""
        out = np.zeros(max(1, self.nlev), dtype=np.int32)
        self._chk(igks_wavefront_sizes(self.ctx, out.ctypes.data_as(_IP), len(out)))
        return out

    def time_kernel(self, klass, reps=50):
        """ms per launch of kernel class klass ("prep", "flux" or "gather"),
        from back-to-back launches between two events."""
        ms = C.c_double()
        self._chk(igks_time_kernel(self.ctx, ("prep", "flux", "gather").index(klass), reps, C.byref(ms)))
        return ms.value

    def kernel_times(self):
        t = np.zeros(len(KERNEL_CLASSES))
        self._chk(igks_get_kernel_times(self.ctx, t.ctypes.data_as(_DP)))
        return dict(zip(KERNEL_CLASSES, t))

    def autotune(self, iters=10):
        s = np.zeros(6, dtype=np.int32)
        self._chk(igks_autotune(self.ctx, iters, s.ctypes.data_as(_IP)))
        return s

    def schedule(self):
        s = np.zeros(6, dtype=np.int32)
        self._chk(igks_get_schedule(self.ctx, s.ctypes.data_as(_IP)))
        return s

    def set_schedule(self, s6):
        s = np.ascontiguousarray(s6, dtype=np.int32)
        self._chk(igks_set_schedule(self.ctx, s.ctypes.data_as(_IP)))

    def graph_chunk(self):
        """(iterations per captured graph, kernel launches per iteration)."""
        it, nl = C.c_int32(), C.c_int32()
        self._chk(igks_graph_chunk(self.ctx, C.byref(it), C.byref(nl)))
        return it.value, nl.value


class Solver(_Context):
    """One mesh + flow condition on one GPU.

    ``mesh`` needs xy, cell_ptr, cell_nodes, bface_nodes, bface_tag (see
    meshgen.Mesh).  ``stream``: a torch.cuda.Stream (default: a new one).
    ``sweep_blocks``: the sweep block of each cell (igks_set_sweep_blocks),
    None for one block.
    """

    def __init__(self, mesh, options: igks_options | None = None, stream=None, device="cuda", sweep_blocks=None,
                 **kw):
        self._open(1, options, stream, device, kw)
        keep, args = _mesh_args(mesh)
        self._chk(igks_mesh_upload(self.ctx, *args))
        if sweep_blocks is not None:
            b, pb = _i(np.asarray(sweep_blocks).reshape(mesh.n_cells))
            self._chk(igks_set_sweep_blocks(self.ctx, 0, pb))
        self._bind()
        self.n, self.nf, self.nwall = self.total_cells, self.total_faces, self.total_wall

    def set_freestream(self, mach, alpha_deg, reynolds, nut_ratio=-1.0):
        self._chk(igks_set_freestream(self.ctx, mach, alpha_deg, reynolds, nut_ratio))

    def residual(self) -> dict:
        r = igks_residual()
        self._chk(igks_get_residual(self.ctx, C.byref(r)))
        return r.as_dict()

    def history(self, max_entries=1 << 20):
        out = np.zeros((max_entries, HIST_W))
        n = C.c_int32()
        self._chk(igks_get_history(self.ctx, out.ctypes.data_as(_DP), max_entries, C.byref(n)))
        return out[:n.value]

    def get_state(self):
        W = np.zeros((5, self.n))
        self._chk(igks_get_state(self.ctx, W.ctypes.data_as(_DP)))
        return W

    def set_state(self, W, scalars: igks_scalars | None = None):
        W, p = _d(np.asarray(W).reshape(5, self.n))
        self._chk(igks_set_state(self.ctx, p, C.byref(scalars) if scalars is not None else None))

    def scalars(self) -> igks_scalars:
        s = igks_scalars()
        self._chk(igks_get_scalars(self.ctx, C.byref(s)))
        return s

    def compute_residual(self):
        M = np.zeros((5, self.n))
        self._chk(igks_compute_residual(self.ctx, M.ctypes.data_as(_DP)))
        return M

    def wall_loads(self):
        cl, cd = C.c_double(), C.c_double()
        cf, cp, xw = (np.zeros(max(self.nwall, 1)) for _ in range(3))
        P = lambda a: a.ctypes.data_as(_DP)
        self._chk(igks_get_wall_loads(self.ctx, C.byref(cl), C.byref(cd), P(cf), P(cp), P(xw)))
        n = self.nwall
        return dict(cl=cl.value, cd=cd.value, cf=cf[:n], cp=cp[:n], xw=xw[:n])


class BatchSolver(_Context):
    """Many independent instances (meshes of any sizes, one flow condition
    each) iterated together in the same kernel launches."""

    def __init__(self, meshes, options: igks_options | None = None, stream=None, device="cuda", sweep_blocks=None,
                 **kw):
        self._open(len(meshes), options, stream, device, kw)
        self.ninst = len(meshes)
        for i, m in enumerate(meshes):
            keep, args = _mesh_args(m)
            self._chk(igks_batch_mesh_upload(self.ctx, i, *args))
            if sweep_blocks is not None and sweep_blocks[i] is not None:
                b, pb = _i(np.asarray(sweep_blocks[i]).reshape(m.n_cells))
                self._chk(igks_set_sweep_blocks(self.ctx, i, pb))
        self._bind()
        self.n, self.nf, self.nwall = [], [], []
        for i in range(self.ninst):
            nc, nf, nw = (C.c_int32() for _ in range(3))
            self._chk(igks_batch_mesh_info(self.ctx, i, C.byref(nc), C.byref(nf), C.byref(nw)))
            self.n.append(nc.value)
            self.nf.append(nf.value)
            self.nwall.append(nw.value)

    def set_freestream(self, i, mach, alpha_deg, reynolds, nut_ratio=-1.0):
        self._chk(igks_batch_set_freestream(self.ctx, i, mach, alpha_deg, reynolds, nut_ratio))

    def status(self, i) -> bool:
        h = C.c_int32()
        self._chk(igks_batch_status(self.ctx, i, C.byref(h)))
        return bool(h.value)

    def residual(self, i) -> dict:
        r = igks_residual()
        self._chk(igks_batch_get_residual(self.ctx, i, C.byref(r)))
        return r.as_dict()

    def history(self, i, max_entries=1 << 20):
        out = np.zeros((max_entries, HIST_W))
        n = C.c_int32()
        self._chk(igks_batch_get_history(self.ctx, i, out.ctypes.data_as(_DP), max_entries, C.byref(n)))
        return out[:n.value]

    def get_state(self, i):
        W = np.zeros((5, self.n[i]))
        self._chk(igks_batch_get_state(self.ctx, i, W.ctypes.data_as(_DP)))
        return W

    def set_state(self, i, W, scalars: igks_scalars | None = None):
        W, p = _d(np.asarray(W).reshape(5, self.n[i]))
        self._chk(igks_batch_set_state(self.ctx, i, p, C.byref(scalars) if scalars is not None else None))

    def scalars(self, i) -> igks_scalars:
        s = igks_scalars()
        self._chk(igks_batch_get_scalars(self.ctx, i, C.byref(s)))
        return s

    def compute_residual(self, i):
        M = np.zeros((5, self.n[i]))
        self._chk(igks_batch_compute_residual(self.ctx, i, M.ctypes.data_as(_DP)))
        return M

    def wall_loads(self, i):
        cl, cd = C.c_double(), C.c_double()
        nw = self.nwall[i]
        cf, cp, xw = (np.zeros(max(nw, 1)) for _ in range(3))
        P = lambda a: a.ctypes.data_as(_DP)
        self._chk(igks_batch_get_wall_loads(self.ctx, i, C.byref(cl), C.byref(cd), P(cf), P(cp), P(xw)))
        return dict(cl=cl.value, cd=cd.value, cf=cf[:nw], cp=cp[:nw], xw=xw[:nw])
