"""The entry point that allocates nothing (igks_bind_static_workspace, the
library's own static device array in place of a caller's workspace) against
the caller-workspace entry point (igks_bind_workspace), through the C ABI:
bitwise the same iterates, residual and wall loads on two meshes in a row,
the second smaller; a context whose static workspace another context has
since bound is refused."""
import ctypes as C

import numpy as np
import pytest

from paper_1709_00803_amd import meshgen as mg

pytestmark = pytest.mark.gpu

TAGS = dict(bottom=lambda x: np.where(x < 0.3, mg.SYMMETRY, mg.WALL), top=mg.FARFIELD, left=mg.FREESTREAM,
            right=mg.OUTFLOW)


@pytest.fixture(scope="module")
def igks():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1709_00803_amd import igks as m
    return m


def run_caller_workspace(igks, mesh, flow, n):
    s = igks.Solver(mesh, cfl_init=5.0, chunk=4)
    s.set_freestream(*flow)
    s.iterate(n)
    out = (s.get_state(), s.compute_residual(), s.wall_loads()["cd"], s.residual())
    s.close()
    return out


def static_ctx(igks, mesh, stream):
    ctx = C.c_void_p()
    o = igks.default_options(cfl_init=5.0, chunk=4)
    assert igks.igks_create(C.byref(ctx), C.byref(o), C.c_void_p(stream.cuda_stream)) == igks.IGKS_OK
    keep, args = igks._mesh_args(mesh)
    assert igks.igks_mesh_upload(ctx, *args) == igks.IGKS_OK
    rc = igks.igks_bind_static_workspace(ctx)
    assert rc == igks.IGKS_OK, igks.igks_last_error(ctx).decode()
    return ctx


def run_static_workspace(igks, mesh, flow, n):
    import torch
    stream = torch.cuda.Stream()
    ctx = static_ctx(igks, mesh, stream)
    try:
        assert igks.igks_set_freestream(ctx, *flow) == igks.IGKS_OK
        done = C.c_int32()
        assert igks.igks_iterate(ctx, n, C.byref(done)) == igks.IGKS_OK and done.value == n
        W = np.zeros((5, mesh.n_cells))
        M = np.zeros((5, mesh.n_cells))
        dp = C.POINTER(C.c_double)
        assert igks.igks_get_state(ctx, W.ctypes.data_as(dp)) == igks.IGKS_OK
        assert igks.igks_compute_residual(ctx, M.ctypes.data_as(dp)) == igks.IGKS_OK
        cd = C.c_double()
        assert igks.igks_get_wall_loads(ctx, None, C.byref(cd), None, None, None) == igks.IGKS_OK
        r = igks.igks_residual()
        assert igks.igks_get_residual(ctx, C.byref(r)) == igks.IGKS_OK
        return W, M, cd.value, r.as_dict()
    finally:
        igks.igks_destroy(ctx)


def test_static_workspace_matches_caller_workspace(igks):
    big = mg.colour_order(mg.random_hybrid(40, 30, seed=4, tags=TAGS))[0]
    small = mg.random_hybrid(12, 9, seed=5, tags=TAGS)
    for tag, mesh, flow, n in (("first, larger mesh", big, (0.4, 3.0, 3e4, 3.0), 8),
                               ("second, smaller mesh", small, (0.3, -2.0, 2e3, -1.0), 6)):
        print(f"case: {tag}, {mesh.n_cells} cells", flush=True)
        Wr, Mr, cdr, rr = run_caller_workspace(igks, mesh, flow, n)
        Ws, Ms, cds, rs = run_static_workspace(igks, mesh, flow, n)
        assert np.array_equal(Ws, Wr), tag
        assert np.array_equal(Ms, Mr), tag
        assert cds == cdr and rs == rr, tag


def test_static_workspace_taken_over(igks):
    import torch
    mesh = mg.random_hybrid(8, 6, seed=6)
    stream = torch.cuda.Stream()
    a = static_ctx(igks, mesh, stream)
    b = static_ctx(igks, mesh, stream)
    try:
        assert igks.igks_set_freestream(b, 0.3, 1.0, 1e3, -1.0) == igks.IGKS_OK
        assert igks.igks_set_freestream(a, 0.3, 1.0, 1e3, -1.0) == igks.IGKS_EINVAL
        assert b"another context" in igks.igks_last_error(a)
        done = C.c_int32()
        assert igks.igks_iterate(b, 3, C.byref(done)) == igks.IGKS_OK
    finally:
        igks.igks_destroy(a)
        igks.igks_destroy(b)
