"""The C-ABI library: it loads, exports every function include/zx.h declares,
and rejects bad arguments on the host (no GPU needed for any of this)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "zx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zx_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_01059_amd import zx
    return zx.load()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    from paper_2604_01059_amd import zx
    assert set(zx.exported_symbols()) == set(names)


def test_version_and_sizes(lib):
    assert lib.zx_version() == 100
    assert lib.zx_graph_bytes(64, 8, 8) > 64 * 8 * 2
    assert lib.zx_graph_bytes(0, 0, 0) == 0
    assert lib.zx_gf2_workspace_bytes(4096, 16384) >= 8 * 4096 * 8
    assert lib.zx_simplify_workspace_bytes(4096) >= 4096 * 8
    assert lib.zx_simplify_variants() >= 2


def test_host_argument_errors(lib):
    from paper_2604_01059_amd import zx
    P = C.c_void_p
    dummy = P(256)
    # null pointers and bad shapes are caught before any device work
    assert lib.zx_gf2_eliminate(None, None, 4, 64, 1, None, None, None, 0, None, 0, None) == zx.ZX_EINVAL
    assert b"null" in lib.zx_last_error()
    assert lib.zx_gf2_eliminate(dummy, dummy, 0, 64, 1, dummy, dummy, None, 0, dummy, 1 << 20, None) == zx.ZX_EINVAL
    assert lib.zx_gf2_eliminate(dummy, dummy, 4, 640, 2, dummy, dummy, None, 0, dummy, 1 << 20, None) == zx.ZX_EINVAL
    # the transform needs ceil(m/64) words per row and may not overlap A
    assert lib.zx_gf2_eliminate(dummy, dummy, 100, 64, 1, dummy, dummy, P(1 << 20), 1, dummy, 1 << 20,
                                None) == zx.ZX_EINVAL
    assert lib.zx_gf2_eliminate(P(4096), P(4096), 4, 64, 1, dummy, dummy, P(4096), 1, dummy, 1 << 20,
                                None) == zx.ZX_EINVAL
    # the allocation-free elimination: same checks, and m beyond its static scratch
    assert lib.zx_gf2_eliminate_noalloc(None, None, 4, 64, 1, None, None, None, 0, None) == zx.ZX_EINVAL
    assert lib.zx_gf2_eliminate_noalloc(dummy, dummy, 0, 64, 1, dummy, dummy, None, 0, None) == zx.ZX_EINVAL
    assert lib.zx_gf2_eliminate_noalloc(dummy, dummy, 16385, 64, 1, dummy, dummy, None, 0,
                                        None) == zx.ZX_ECAPACITY
    assert b"16385" in lib.zx_last_error()
    assert lib.zx_pauli_commute(None, None, 10, 10, 1, None, 1, 0, None) == zx.ZX_EINVAL
    assert lib.zx_local_comp(None, 0, 0, None) == zx.ZX_EINVAL
    assert lib.zx_batch_simplify(None, None, None) == zx.ZX_EINVAL
    g = P()
    assert lib.zx_graph_create(C.byref(g), None, 0, 4, None, None, None, 0, None, 0, None, None) == zx.ZX_EINVAL


def test_graph_create_validates_input(lib):
    """Asymmetric adjacency / bad phases / duplicate boundary are host errors."""
    import numpy as np
    from paper_2604_01059_amd import zx
    P = C.c_void_p
    g = P()
    adj = np.array([[2], [0], [0]], np.uint64)  # 0-1 edge only one way
    ph = np.zeros(3, np.int8)
    ins = np.array([0], np.int32)
    outs = np.array([2], np.int32)
    rc = lib.zx_graph_create(C.byref(g), P(256), 1 << 20, 3, adj.ctypes.data_as(P), ph.ctypes.data_as(P),
                             ins.ctypes.data_as(P), 1, outs.ctypes.data_as(P), 1, None, None)
    assert rc == zx.ZX_EINVAL and b"symmetric" in lib.zx_last_error()
    adj = np.array([[2], [1], [0]], np.uint64)
    ph = np.array([0, 9, 0], np.int8)
    rc = lib.zx_graph_create(C.byref(g), P(256), 1 << 20, 3, adj.ctypes.data_as(P), ph.ctypes.data_as(P),
                             ins.ctypes.data_as(P), 1, outs.ctypes.data_as(P), 1, None, None)
    assert rc == zx.ZX_EINVAL and b"phase" in lib.zx_last_error()
    ph = np.zeros(3, np.int8)
    outs = np.array([0], np.int32)
    rc = lib.zx_graph_create(C.byref(g), P(256), 1 << 20, 3, adj.ctypes.data_as(P), ph.ctypes.data_as(P),
                             ins.ctypes.data_as(P), 1, outs.ctypes.data_as(P), 1, None, None)
    assert rc == zx.ZX_EINVAL and b"two boundary" in lib.zx_last_error()
