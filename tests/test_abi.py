"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-only entry points validate arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_06926_amd import _lib
    if not os.path.exists(_lib.library_path()):
        from paper_1804_06926_amd import build
        build.build()
    return _lib._load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("tc_create", "tc_destroy", "tc_workspace_size", "tc_count_triangles", "tc_edge_counts",
                     "tc_build_csr", "tc_radix_sort_u64", "tc_status_string", "tc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_size_host_checks(lib):
    from paper_1804_06926_amd import _lib
    out = ctypes.c_size_t()
    o = _lib.Options()
    assert lib.tc_workspace_size(1000, 100, ctypes.byref(o), ctypes.byref(out)) == 0
    small = out.value
    assert lib.tc_workspace_size(100000, 100, ctypes.byref(o), ctypes.byref(out)) == 0
    assert out.value > small
    assert lib.tc_workspace_size(-1, 100, ctypes.byref(o), ctypes.byref(out)) == 1
    assert lib.tc_workspace_size(10, -1, ctypes.byref(o), ctypes.byref(out)) == 1
    assert lib.tc_workspace_size((1 << 31) - (1 << 19), 10, ctypes.byref(o), ctypes.byref(out)) == 5
    o.select = 9
    assert lib.tc_workspace_size(10, 10, ctypes.byref(o), ctypes.byref(out)) == 1
    o.select = 0
    o.reserved[2] = 1
    assert lib.tc_workspace_size(10, 10, ctypes.byref(o), ctypes.byref(out)) == 1


def test_status_strings(lib):
    lib.tc_status_string.restype = ctypes.c_char_p
    assert lib.tc_status_string(0) == b"ok"
    assert b"range" in lib.tc_status_string(2)


def test_null_context_is_rejected(lib):
    count = ctypes.c_uint64()
    assert lib.tc_count_triangles(None, None, 0, 0, None, 0, None, ctypes.byref(count), None) == 1
    assert lib.tc_destroy(None) == 1


def test_binding_refuses_host_tensors():
    import numpy as np
    import torch
    import paper_1804_06926_amd as tc
    with pytest.raises(TypeError):
        tc.count_triangles(torch.from_numpy(np.zeros((3, 2), np.int32)), 4)


def test_formulation_workspace_size_host_checks(lib):
    """The full-list and matrix forms add the symmetric adjacency (4 (n + 1) + 8 E
    bytes, each rounded up to 256) to the plain workspace; the filtered and
    upper-triangle forms need no more than the plain count."""
    from paper_1804_06926_amd import _lib
    o = _lib.Options()
    E, n = 100000, 5000
    plain, out = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.tc_workspace_size(E, n, ctypes.byref(o), ctypes.byref(plain)) == 0
    up = lambda x: (x + 255) // 256 * 256
    for form, extra in ((0, 0), (1, up(4 * (n + 1)) + up(8 * E)), (2, up(4 * (n + 1)) + up(8 * E)), (3, 0)):
        assert lib.tc_formulation_workspace_size(E, n, ctypes.byref(o), form, ctypes.byref(out)) == 0
        assert out.value == plain.value + extra, form
    for bad in (-1, 4):
        assert lib.tc_formulation_workspace_size(E, n, ctypes.byref(o), bad, ctypes.byref(out)) == 1
    assert lib.tc_formulation_workspace_size(-1, n, ctypes.byref(o), 1, ctypes.byref(out)) == 1
    assert lib.tc_formulation_workspace_size((1 << 31) - (1 << 19), n, ctypes.byref(o), 1, ctypes.byref(out)) == 5
    count = ctypes.c_uint64()
    assert lib.tc_count_triangles_formulation(None, None, 0, 0, None, 0, None, 1, ctypes.byref(count), None) == 1


def test_formulation_binding_names():
    import paper_1804_06926_amd as tc
    assert tc.FORMULATIONS == {"filtered": 0, "full": 1, "matrix": 2, "matrix_upper": 3}
