"""The C-ABI library loads and exports every symbol of include/csaw.h, and its
host-side validation works without a GPU (no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csaw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csaw_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def csaw():
    from paper_2009_09103_amd import csaw as c
    return c


def test_every_declared_symbol_is_exported(csaw):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(csaw.lib, name), name
    assert set(names) == set(csaw.EXPORTS)


def test_version_and_error_string(csaw):
    assert "gfx950" in csaw.version()
    assert isinstance(csaw.lib.csaw_last_error(), bytes)


def test_graph_create_rejects_bad_csr_on_host(csaw):
    h = ctypes.c_void_p()
    rowptr = np.array([0, 2, 1], dtype=np.int64)          # decreasing
    col = np.array([1, 0], dtype=np.int32)
    st = csaw.lib.csaw_graph_create(2, 1, rowptr.ctypes.data, col.ctypes.data, None, 0, None, ctypes.byref(h))
    assert st == 1 and b"decreases" in csaw.lib.csaw_last_error()
    rowptr = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 5], dtype=np.int32)                # id out of range
    st = csaw.lib.csaw_graph_create(2, 2, rowptr.ctypes.data, col.ctypes.data, None, 0, None, ctypes.byref(h))
    assert st == 1 and b"out of range" in csaw.lib.csaw_last_error()
    st = csaw.lib.csaw_graph_create(2, 2, rowptr.ctypes.data, col.ctypes.data, None, 7, None, ctypes.byref(h))
    assert st == 1                                        # flags must be 0
    st = csaw.lib.csaw_graph_create(-1, 0, rowptr.ctypes.data, col.ctypes.data, None, 0, None, ctypes.byref(h))
    assert st == 1


def test_null_handles_are_rejected(csaw):
    a = csaw.SampleArgs()
    mx = ctypes.c_int64()
    assert csaw.lib.csaw_sample_bound(None, ctypes.byref(a), ctypes.byref(mx)) == 1
    assert csaw.lib.csaw_walk(None, None, None, None, None) == 1
    assert csaw.lib.csaw_graph_destroy(None) == 1


def test_profile_calls_without_records(csaw):
    csaw.profile_reset()
    t, c = csaw.profile_read("select")
    assert t == 0.0 and c == 0


def test_no_cpu_fallback_in_binding():
    """The binding has no compute path of its own and never touches the oracle."""
    src = open(os.path.join(ROOT, "paper_2009_09103_amd", "csaw.py")).read()
    assert "oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2009_09103_amd")):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_2009_09103_amd", f)).read()


def test_tuning_calls_validate_on_host(csaw):
    t = csaw.Tuning(16, 32)
    assert csaw.lib.csaw_set_tuning(None, ctypes.byref(t)) == 1
    assert csaw.lib.csaw_get_tuning(None, ctypes.byref(t)) == 1
    assert csaw.lib.csaw_autotune_sample(None, None, None, 3, None, None) == 1
