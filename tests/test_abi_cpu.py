"""The C-ABI library loads without a GPU, exports every symbol the header
declares, and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chefsi.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(chefsi_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def raw():
    import paper_1606_03416_amd as chefsi
    return chefsi.lib


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("chefsi_bounds", "chefsi_filter", "chefsi_orthonormalize", "chefsi_rayleigh_ritz", "chefsi_sweep"):
        assert n in names


def test_library_exports_every_declared_symbol(raw):
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing
    assert raw.chefsi_version().startswith(b"chefsi")


def _J(n, v=32):
    return np.full(n, v, dtype=np.int32)


def test_plan_create_rejects_bad_arguments_on_host(raw):
    h = ctypes.c_void_p()
    J = _J(8)
    ptr = J.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    cases = [
        (2, 2, 2, 6, ptr),     # stencil
        (0, 2, 2, 7, ptr),     # grid
        (2, -1, 2, 7, ptr),
        (2, 2, 2, 7, None),    # counts NULL
    ]
    for nx, ny, nz, s, p in cases:
        assert raw.chefsi_plan_create(ctypes.byref(h), nx, ny, nz, s, p) == 1
        assert h.value is None
    bad = _J(8)
    bad[3] = 0
    assert raw.chefsi_plan_create(ctypes.byref(h), 2, 2, 2, 7, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == 1
    assert b"alb_counts[3]" in raw.chefsi_last_error()
    big = _J(8, 257)
    assert raw.chefsi_plan_create(ctypes.byref(h), 2, 2, 2, 7, big.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == 1
    assert raw.chefsi_plan_create(None, 2, 2, 2, 7, ptr) == 1


def test_null_plan_and_orthonormalize_checks(raw):
    out = ctypes.c_size_t(0)
    assert raw.chefsi_workspace_bytes(None, 1, 8, 0, 2, 20, ctypes.byref(out)) == 1
    assert raw.chefsi_filter(None, None, 3, 0.0, 1.0, -1.0, 0, None, 8, None, 8, 8, None, 0, None) == 1
    assert raw.chefsi_sweep(None, None, 3, 0, 2, 20, None, None, 0, None, 8, 8, None, None, None, None,
                            None, 0, None) == 1
    dummy = ctypes.c_void_p(0x1000)
    # passes, shapes, leading dimension
    assert raw.chefsi_orthonormalize(100, 10, dummy, 10, 3, None, None, 0, None) == 1
    assert raw.chefsi_orthonormalize(100, 0, dummy, 10, 2, None, None, 0, None) == 1
    assert raw.chefsi_orthonormalize(5, 10, dummy, 10, 2, None, None, 0, None) == 1
    assert raw.chefsi_orthonormalize(100, 10, dummy, 5, 2, None, None, 0, None) == 1
    assert raw.chefsi_orthonormalize(100, 10, None, 10, 2, None, None, 0, None) == 1
    # a valid shape with a missing workspace is a workspace error, still before any HIP call
    assert raw.chefsi_orthonormalize(100, 10, dummy, 10, 2, None, None, 0, None) == 3
    ws = ctypes.c_void_p(0x1001)
    assert raw.chefsi_orthonormalize(100, 10, dummy, 10, 2, None, ws, 1 << 30, None) == 3
    assert raw.chefsi_orthonormalize_workspace_bytes(100, 10, 2, ctypes.byref(out)) == 0
    assert out.value >= 3 * 10 * 10 * 8


def test_post_cycle_entry_points_check_arguments_on_host(raw):
    """Occupations, density blocks and re-alignment reject bad arguments
    before any HIP call."""
    d = ctypes.c_double
    a = ctypes.c_void_p(0x10000)
    f = ctypes.c_void_p(0x20000)
    mu = ctypes.c_void_p(0x30000)
    occ = raw.chefsi_occupations
    occ.argtypes = [ctypes.c_int, ctypes.c_void_p, d, d, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert occ(0, a, d(0.5), d(1e-3), f, mu, None) == 1          # ns
    assert occ(10, a, d(0.0), d(1e-3), f, mu, None) == 1         # n_occ at 0
    assert occ(10, a, d(10.0), d(1e-3), f, mu, None) == 1        # n_occ at ns
    assert occ(10, a, d(5.0), d(0.0), f, mu, None) == 1          # kT
    assert occ(10, a, d(5.0), d(float("inf")), f, mu, None) == 1
    assert occ(10, None, d(5.0), d(1e-3), f, mu, None) == 1      # NULL ritz
    assert occ(10, a, d(5.0), d(1e-3), f, ctypes.c_void_p(0x10008), None) == 1   # mu inside ritz
    assert occ(10, a, d(5.0), d(1e-3), ctypes.c_void_p(0x10008), mu, None) == 1  # f partly over ritz
    assert raw.chefsi_density_blocks(None, a, 8, 8, f, mu, None, 0, None) == 1
    assert raw.chefsi_realign(None, 8, a, f, mu, 8, 8, None, 0, None) == 1
    out = ctypes.c_size_t(0)
    assert raw.chefsi_realign_workspace_bytes(None, 8, ctypes.byref(out)) == 1
    assert raw.chefsi_plan_block_elems(None) == -1
