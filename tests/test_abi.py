"""The C-ABI library loads and exports every entry point include/igks.h
declares (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igks.h")
LIB = os.path.join(ROOT, "paper_1709_00803_amd", "libigks.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(igks_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1709_00803_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("igks_create", "igks_mesh_upload", "igks_workspace_size", "igks_bind_workspace",
              "igks_set_freestream", "igks_iterate", "igks_get_residual", "igks_get_wall_loads",
              "igks_get_state", "igks_set_state", "igks_compute_residual", "igks_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in declared_functions():
        assert n in syms, n


def test_binding_covers_the_header():
    from paper_1709_00803_amd import igks
    assert set(igks.EXPORTED) == set(declared_functions())


def test_default_options_without_gpu(lib):
    from paper_1709_00803_amd import igks
    o = igks.default_options()
    assert o.precision == igks.IGKS_FP64 and o.cfl_init == 1000.0 and o.chunk == 20 and o.block == 256
    assert o.sweep == 0 and o.flux_lanes == 0 and o.scheme == 0 and o.wall_temp == 0.0 and o.limiter_freeze == 0.0
    assert o.tau_jump == 0
