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


STRUCTS = {  # C struct -> ctypes mirror in the binding
    "csaw_sample_args": "SampleArgs",
    "csaw_sample_out": "SampleOut",
    "csaw_tuning": "Tuning",
    "csaw_walk_args": "WalkArgs",
    "csaw_mdrw_args": "MdrwArgs",
    "csaw_layer_args": "LayerArgs",
    "csaw_server_config": "ServerConfig",
    "csaw_request": "Request",
    "csaw_result": "Result",
}


def test_binding_structs_match_the_header(csaw, tmp_path):
    """Every struct of include/csaw.h has the same size and field offsets in
    the ctypes binding (compiled with the host C compiler)."""
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "csaw.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in getattr(csaw, pyname)._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(ln.rsplit(" ", 1) for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                           check=True).stdout.strip().splitlines())
    for cname, pyname in STRUCTS.items():
        st = getattr(csaw, pyname)
        assert int(out["%s size" % cname]) == ctypes.sizeof(st), cname
        for fname, _ in st._fields_:
            assert int(out["%s.%s" % (cname, fname)]) == getattr(st, fname).offset, (cname, fname)


def test_set_allocator_validates_on_host(csaw):
    a = csaw.AllocFn(lambda n, u: None)
    assert csaw.lib.csaw_set_allocator(a, csaw.FreeFn(), None) == 1     # one of two NULL
    assert csaw.lib.csaw_set_allocator(csaw.AllocFn(), csaw.FreeFn(), None) == 0
